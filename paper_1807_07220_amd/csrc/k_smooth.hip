// The smoother S r = eta * sum_i ext((L_i^+)^{-1} R_i^+ r) (paper section 5,
// eq. smooth) on the oversampled blocks K_i^+ = K_i enlarged by the overlap.
//
// On K_i^+ with zero normal flux on its boundary, the local saddle solve has the
// divergence-free solution v = C psi with psi = (C^T A C)^{-1} C^T r on the
// patch's interior vertices (the 9-point stencil of the stream-function
// operator restricted to them).  The local matrices are factorised once per
// setup in the twisted block form described in patch.h; every smoother
// application is one launch over all patches (the overlapping solutions are
// summed by the gather kernels of k_pcg.hip).
#include <hip/hip_ext.h>

#include "common.h"
#include "patch.h"

#ifndef TGMS_PF_DIRECT
#define TGMS_PF_DIRECT 1  // link lines in flight per chain when the factor is read from global memory
#endif

namespace {

// ------------------------------------------------------------------ factorisation
// One wavefront per patch.  LDS: the scaled stencil (c, e, n, ne, nw per vertex),
// the scale S, and three m x m work matrices.
constexpr int FAC_MAXE = 16;  // m*m <= 1024 entries, 16 per lane

// In-place Gauss-Jordan inversion of the SPD matrix W (m x m, row-major) by one
// wavefront; the pivots are Schur-complement diagonals, positive for SPD input.
__device__ void gj_invert(double* W, int m, int* fail) {
    const int lane = threadIdx.x;
    const int mm = m * m;
    for (int p = 0; p < m; ++p) {
        const double piv = W[p * m + p];
        if (!(piv > 0.0) && lane == 0) atomicOr(fail, 1);
        const double d = 1.0 / piv;
        double nv[FAC_MAXE];
#pragma unroll
        for (int t = 0; t < FAC_MAXE; ++t) {
            const int e = lane + 64 * t;
            nv[t] = 0.0;
            if (e < mm) {
                const int i = e / m, j = e - i * m;
                const double wip = W[i * m + p], wpj = W[p * m + j];
                if (i == p && j == p)
                    nv[t] = d;
                else if (i == p)
                    nv[t] = wpj * d;
                else if (j == p)
                    nv[t] = -wip * d;
                else
                    nv[t] = W[e] - wip * wpj * d;
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < FAC_MAXE; ++t) {
            const int e = lane + 64 * t;
            if (e < mm) W[e] = nv[t];
        }
        __syncthreads();
    }
}

struct PatchStencil {
    const double *c, *e, *n, *ne, *nw;
    int m;
    // diagonal block of vertex row j
    __device__ double A(int j, int r, int s) const {
        if (r == s) return c[j * m + r];
        if (s == r + 1) return e[j * m + r];
        if (r == s + 1) return e[j * m + s];
        return 0.0;
    }
};

__global__ void __launch_bounds__(64) k_patch_factor(const Rect* __restrict__ rects, const double* __restrict__ a,
                                                     int nx, double sx2, double sy2, double* __restrict__ Fpool,
                                                     int* __restrict__ fail, int npatch) {
    extern __shared__ double sm[];
    // a grid-stride loop over the patches: a smaller grid leaves room on the GPU for
    // kernels of other streams
    for (int pid = blockIdx.x; pid < npatch; pid += gridDim.x) {
        const Rect R = rects[pid];
        const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
        const int n = m * mh, mm = m * m, k = mh / 2;
        const int lane = threadIdx.x;
        double* kc = sm;
        double* ke = kc + n;
        double* kn = ke + n;
        double* kne = kn + n;
        double* knw = kne + n;
        double* S = knw + n;
        double* W = S + n;
        double* G = W + mm;
        double* Mid = G + mm;
        double* F = Fpool + R.off;
        double* Pout = F;
        double* Lout = F + tw_links(m, mh);
        double* Sout = F + tw_scale(m, mh);
        // stencil couplings of each interior vertex with its east, north, north-east
        // and north-west neighbours (zero where the neighbour is not a patch vertex)
        for (int r = lane; r < n; r += 64) {
            const int aa = r % m, bb = r / m;
            const int i = R.i0 + 1 + aa, j = R.j0 + 1 + bb;
            const long long v = (long long)j * nx + i;
            const Stencil9 st = stencil9(a[v - nx - 1], a[v - nx], a[v - 1], a[v], sx2, sy2);
            kc[r] = st.c;
            ke[r] = (aa + 1 < m) ? st.e : 0.0;
            const bool up = bb + 1 < mh;
            kn[r] = up ? st.n : 0.0;
            kne[r] = (up && aa + 1 < m) ? st.ne : 0.0;
            knw[r] = (up && aa >= 1) ? st.nw : 0.0;
            S[r] = 1.0 / sqrt(st.c);
        }
        __syncthreads();
        for (int r = lane; r < n; r += 64) {
            const int aa = r % m, bb = r / m;
            const double s = S[r];
            kc[r] *= s * s;
            if (aa + 1 < m) ke[r] *= s * S[r + 1];
            if (bb + 1 < mh) {
                kn[r] *= s * S[r + m];
                if (aa + 1 < m) kne[r] *= s * S[r + m + 1];
                if (aa >= 1) knw[r] *= s * S[r + m - 1];
            }
            Sout[r] = s;
        }
        __syncthreads();
        const PatchStencil P{kc, ke, kn, kne, knw, m};
        for (int e = lane; e < mm; e += 64) Mid[e] = P.A(k, e / m, e % m);
        auto store_pivot = [&](int j) {
            for (int e = lane; e < mm; e += 64) {
                const int r = e / m, s = e - r * m;
                if (r >= s) Pout[(long long)j * tw_tri(m) + tw_offP(s, m) + (r - s)] = W[e];
            }
        };
        // top sweep: rows 0..k-1
        if (k >= 1)
            for (int e = lane; e < mm; e += 64) W[e] = P.A(0, e / m, e % m);
        __syncthreads();
        for (int j = 0; j < k; ++j) {
            gj_invert(W, m, fail);
            store_pivot(j);
            // G = B_j T_j^{-1}; B_j[r][s] = kn(s) (r = s), kne(s) (r = s+1), knw(s) (r = s-1) at row j
            const int o = j * m;
            for (int e = lane; e < mm; e += 64) {
                const int r = e / m, s = e - r * m;
                double g = kn[o + r] * W[r * m + s];
                if (r >= 1) g += kne[o + r - 1] * W[(r - 1) * m + s];
                if (r + 1 < m) g += knw[o + r + 1] * W[(r + 1) * m + s];
                G[e] = g;
                Lout[(long long)j * mm + e] = g;
            }
            __syncthreads();
            // G B_j^T, subtracted from the next diagonal block (or from the middle one)
            for (int e = lane; e < mm; e += 64) {
                const int r = e / m, s = e - r * m;
                double cb = G[r * m + s] * kn[o + s];
                if (s >= 1) cb += G[r * m + s - 1] * kne[o + s - 1];
                if (s + 1 < m) cb += G[r * m + s + 1] * knw[o + s + 1];
                if (j + 1 < k)
                    W[e] = P.A(j + 1, r, s) - cb;
                else
                    Mid[e] -= cb;
            }
            __syncthreads();
        }
        // bottom sweep: rows mh-1..k+1
        if (mh - 1 > k)
            for (int e = lane; e < mm; e += 64) W[e] = P.A(mh - 1, e / m, e % m);
        __syncthreads();
        for (int j = mh - 1; j > k; --j) {
            gj_invert(W, m, fail);
            store_pivot(j);
            // H = B_{j-1}^T U_j^{-1}
            const int o = (j - 1) * m;
            for (int e = lane; e < mm; e += 64) {
                const int r = e / m, s = e - r * m;
                double h = kn[o + r] * W[r * m + s];
                if (r + 1 < m) h += kne[o + r] * W[(r + 1) * m + s];
                if (r >= 1) h += knw[o + r] * W[(r - 1) * m + s];
                G[e] = h;
                Lout[(long long)(j - 1) * mm + e] = h;
            }
            __syncthreads();
            // H B_{j-1}
            for (int e = lane; e < mm; e += 64) {
                const int r = e / m, s = e - r * m;
                double cb = G[r * m + s] * kn[o + s];
                if (s + 1 < m) cb += G[r * m + s + 1] * kne[o + s];
                if (s >= 1) cb += G[r * m + s - 1] * knw[o + s];
                if (j - 1 > k)
                    W[e] = P.A(j - 1, r, s) - cb;
                else
                    Mid[e] -= cb;
            }
            __syncthreads();
        }
        for (int e = lane; e < mm; e += 64) W[e] = Mid[e];
        __syncthreads();
        gj_invert(W, m, fail);
        store_pivot(k);
        __syncthreads();  // LDS is reused by the next patch
    }
}

// ------------------------------------------------------------------ application
// Per patch: psi = S K~^{-1} S g on the patch's interior vertices.  Waves 0 and 1
// run the top and bottom chains; lane a < m holds entry a of the current block
// vector, and the entries a matrix-vector product needs are broadcast from their
// lanes with readlane.  The line of the link used by step t+1 (and the entry of
// b or u) is loaded while step t computes.  Between the forward and backward
// chains all four waves form the independent products u_j = P_j w_j.
//
// M: the compile-time row width (registers, unrolled loops, fixed offsets).
template <typename T, int M>
struct Lines {
    int a;
    // row a of a dense M x M row-major matrix
    __device__ void row(T (&v)[M], const T* p) const {
#pragma unroll
        for (int c = 0; c < M; ++c) v[c] = p[a * M + c];
    }
    // column a of a dense M x M row-major matrix
    __device__ void column(T (&v)[M], const T* p) const {
#pragma unroll
        for (int c = 0; c < M; ++c) v[c] = p[c * M + a];
    }
};

template <typename T, int M>
__device__ inline T dot_lanes(const T (&v)[M], T x) {
    T s[4] = {T(0), T(0), T(0), T(0)};  // four independent accumulation chains
#pragma unroll
    for (int c = 0; c < M; ++c) s[c & 3] += v[c] * readlane(x, c);
    return (s[0] + s[1]) + (s[2] + s[3]);
}

// Where a patch solution goes: the patch's own vector (slot layout off), or the
// slot of the patch among four vertex planes (own block, x neighbour, y neighbour,
// diagonal neighbour): every vertex lies in at most one patch of each kind, so a
// patch writes whole row segments of each plane and summing the overlapping
// solutions is four coalesced reads per vertex.
template <typename T>
struct PatchOut {
    T* base;        // own vector (m*mh entries), used when w4 is null
    T* w4;          // four planes of nx*ny vertices
    long long plane;
    int m, nx, i0, j0;
    int bxlo, bxhi, bylo, byhi;  // the cells of the patch's own coarse block
    __device__ void put(int row, int a, T v) const {
        if (!w4) {
            base[row * m + a] = v;
            return;
        }
        const int i = i0 + 1 + a, j = j0 + 1 + row;
        const int slot = (i < bxlo || i >= bxhi ? 1 : 0) + (j < bylo || j >= byhi ? 2 : 0);
        w4[slot * plane + (long long)j * nx + i] = v;
    }
};

// One chain of steps t = 0..steps-1 on link lk(t): line(t) . x with line = row
// (ROW) or column of the link; then x = base[r(t)] - product, handed to put(r(t), .)
// (scaled by scale[r(t)] when given), except that with TO_MID the last product
// goes to mid instead.  The lines of the next PF steps are in flight while a step
// computes (PF + 1 register buffers, rotated by unrolling).
template <typename T, int M, bool ROW, bool TO_MID, int PF, typename RowOf, typename LinkOf, typename Put>
__device__ inline void chain(const Lines<T, M>& ln, int steps, const T* Lk, const T* base, Put put, const T* scale,
                             T* mid, T x, bool act, RowOf rr, LinkOf lk) {
    if (steps <= 0) return;
    constexpr long long mm = (long long)M * M;
    constexpr int NB = PF + 1;
    const int a = ln.a;
    T L[NB][M];
    T bv[NB], sv[NB];
    auto load = [&](T(&Ld)[M], T& b, T& sc, int t) {
        if (ROW)
            ln.row(Ld, Lk + lk(t) * mm);
        else
            ln.column(Ld, Lk + lk(t) * mm);
        b = (!TO_MID || t + 1 < steps) ? base[rr(t) * M + a] : T(0);
        sc = scale ? scale[rr(t) * M + a] : T(1);
    };
#pragma unroll
    for (int d = 0; d < PF; ++d)
        if (d < steps) load(L[d], bv[d], sv[d], d);
    for (int t0 = 0; t0 < steps; t0 += NB) {
#pragma unroll
        for (int d = 0; d < NB; ++d) {
            const int t = t0 + d;
            if (t < steps) {
                const T s = dot_lanes<T, M>(L[d], x);
                __builtin_amdgcn_sched_barrier(0);  // keep the next loads behind this step's products
                const int dn = (d + PF) % NB;  // a constant once the loop is unrolled
                if (t + PF < steps) load(L[dn], bv[dn], sv[dn], t + PF);
                if (TO_MID && t + 1 == steps) {
                    if (act) mid[a] = s;
                } else {
                    x = bv[d] - s;
                    if (act) put(rr(t), scale ? sv[d] * x : x);
                }
            }
        }
    }
}

// Fg: the factor in global memory, read by the forward sweeps; F: the factor the rest
// reads (Fg, or its LDS copy).  With stage (F in LDS, not yet filled): waves 2 and 3
// copy the factor from Fg to F while waves 0 and 1 run the forward sweeps.
template <typename T, int M, int PF>
__device__ inline void solve_patch(int mh, const T* F, const T* Fg, T* vec, T* u, T* mid, const PatchOut<T>& out,
                                   long long stage) {
    constexpr int m = M, tri = M * (M + 1) / 2;
    const int k = mh / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool act = lane < m;
    const Lines<T, M> ln{act ? lane : m - 1};
    const int a = ln.a;
    const T* P = F;
    const T* Lk = F + tw_links(m, mh);
    const T* Lf = Fg + tw_links(m, mh);  // the forward sweeps' links
    const T* S = F + tw_scale(m, mh);
    if (stage > 0 && wave >= 2) {
        // 16-byte copies, eight in flight per thread (128 threads)
        using V = float4;
        constexpr int PER = 16 / sizeof(T), U = 8;
        const V* src = reinterpret_cast<const V*>(Fg);
        V* dst = reinterpret_cast<V*>(const_cast<T*>(F));
        const int nvec = (int)((stage + PER - 1) / PER), t2 = tid - 128;
        int e = t2;
        for (; e + (U - 1) * 128 < nvec; e += U * 128) {
            V v[U];
#pragma unroll
            for (int q = 0; q < U; ++q) v[q] = src[e + q * 128];
#pragma unroll
            for (int q = 0; q < U; ++q) dst[e + q * 128] = v[q];
        }
        for (; e < nvec; e += 128) dst[e] = src[e];
    }
    if (wave == 0) {
        // w_{t+1} = b_{t+1} - G_t w_t for t < k-1, stored over b; G_{k-1} w_{k-1} -> mid
        auto to_vec = [&](int row, T v) { vec[row * M + a] = v; };
        chain<T, M, true, true, PF>(ln, k, Lf, vec, to_vec, (const T*)nullptr, mid, vec[a], act,
                                [](int t) { return t + 1; }, [](int t) { return (long long)t; });
        if (k == 0 && act) mid[a] = T(0);
    } else if (wave == 1) {
        // w_{r-1} = b_{r-1} - H_{r-1} w_r from r = mh-1 down; H_k w_{k+1} -> mid + M
        auto to_vec = [&](int row, T v) { vec[row * M + a] = v; };
        chain<T, M, true, true, PF>(ln, mh - 1 - k, Lf, vec, to_vec, (const T*)nullptr, mid + M, vec[(mh - 1) * M + a],
                                act, [=](int t) { return mh - 2 - t; }, [=](int t) { return (long long)(mh - 2 - t); });
        if (mh - 1 == k && act) mid[M + a] = T(0);
    }
    __syncthreads();
    // u_j = P_j w_j for every row j (w_k = b_k - G_{k-1} w_{k-1} - H_k w_{k+1})
    {
        int idx[M];  // position of P_j[a][c] in the packed lower triangle
#pragma unroll
        for (int c = 0; c < M; ++c) idx[c] = (c <= a) ? tw_offP(c, M) - c + a : tw_offP(a, M) - a + c;
        for (int j = wave; j < mh; j += 4) {
            const T* Pj = P + (long long)j * tri;
            T pr[M];
#pragma unroll
            for (int c = 0; c < M; ++c) pr[c] = Pj[idx[c]];
            T wj = vec[j * M + a];
            if (j == k) wj -= mid[a] + mid[M + a];
            const T uj = dot_lanes<T, M>(pr, wj);
            if (act) u[j * M + a] = uj;
        }
    }
    __syncthreads();
    const T xk = u[k * M + a];
    auto to_out = [&](int row, T v) { out.put(row, a, v); };
    if (wave == 0) {
        if (act) out.put(k, a, S[k * M + a] * xk);
        // x_l = u_l - G_l^T x_{l+1}, l = k-1 .. 0
        chain<T, M, false, false, PF>(ln, k, Lk, u, to_out, S, mid, xk, act, [=](int t) { return k - 1 - t; },
                                  [=](int t) { return (long long)(k - 1 - t); });
    } else if (wave == 1) {
        // x_{l+1} = u_{l+1} - H_l^T x_l, l = k .. mh-2
        chain<T, M, false, false, PF>(ln, mh - 1 - k, Lk, u, to_out, S, mid, xk, act, [=](int t) { return k + 1 + t; },
                                  [=](int t) { return (long long)(k + t); });
    }
}

// Any row width m <= 64: the same two-sided sweeps with runtime loops over the
// columns (no register lines, no prefetch).  Used for widths without a
// fixed-width instantiation.
template <typename T>
__device__ inline void solve_patch_any(int m, int mh, const T* F, T* vec, T* u, T* mid, const PatchOut<T>& out) {
    const int k = mh / 2, tri = tw_tri(m);
    const long long mm = (long long)m * m;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool act = lane < m;
    const int a = act ? lane : 0;
    const T* P = F;
    const T* Lk = F + tw_links(m, mh);
    const T* S = F + tw_scale(m, mh);
    auto psym = [&](const T* Pj, int c) { return c <= a ? Pj[tw_offP(c, m) + a - c] : Pj[tw_offP(a, m) + c - a]; };
    if (wave < 2) {
        const bool top = wave == 0;
        const int steps = top ? k : mh - 1 - k;
        T* md = mid + (top ? 0 : 64);
        if (steps == 0 && act) md[a] = T(0);
        int r = top ? 0 : mh - 1;
        T w = act ? vec[r * m + a] : T(0);
        for (int t = 0; t < steps; ++t) {
            const long long l = top ? t : mh - 2 - t;
            const T* Lr = Lk + l * mm + (long long)a * m;
            const T* Pj = P + (long long)r * tri;
            T s = T(0), p = T(0);
            for (int c = 0; c < m; ++c) {
                const T xc = readlane(w, c);
                s += Lr[c] * xc;
                p += psym(Pj, c) * xc;
            }
            if (act) u[r * m + a] = p;
            r += top ? 1 : -1;
            if (t + 1 < steps)
                w = act ? vec[r * m + a] - s : T(0);
            else if (act)
                md[a] = s;
        }
    }
    __syncthreads();
    if (wave < 2) {
        const bool top = wave == 0;
        T wk = act ? vec[k * m + a] - mid[a] - mid[64 + a] : T(0);
        const T* Pk = P + (long long)k * tri;
        T x = T(0);
        for (int c = 0; c < m; ++c) x += psym(Pk, c) * readlane(wk, c);
        if (!act) x = T(0);
        if (top && act) out.put(k, a, S[k * m + a] * x);
        const int steps = top ? k : mh - 1 - k;
        for (int t = 0; t < steps; ++t) {
            const long long l = top ? k - 1 - t : k + t;
            const int r = top ? k - 1 - t : k + 1 + t;
            const T* Lc = Lk + l * mm + a;
            T s = T(0);
            for (int c = 0; c < m; ++c) s += Lc[(long long)c * m] * readlane(x, c);
            x = act ? u[r * m + a] - s : T(0);
            if (act) out.put(r, a, S[r * m + a] * x);
        }
    }
}

// One workgroup (4 waves) per patch.  MODE 1: the factor is first copied to LDS
// with 16-byte loads (eight in flight per thread); MODE 0: the chains read it from
// global memory with the lines of the next steps in flight; MODE 2: the forward
// chains read global memory while waves 2 and 3 copy the factor to LDS, which the
// pivot products and the backward chains then read (the staging is hidden behind
// the forward sweeps and the links are read from HBM once).  GENERIC: every patch
// takes the clamped path of width M1 (m <= M1; MODE 2 runs as MODE 0); otherwise
// every patch has width M1 or M2 and takes the fixed-width path of its width.
template <typename T, int M1, int M2, bool GENERIC, int MODE>
__global__ void __launch_bounds__(256) k_smooth_twisted(const Rect* __restrict__ rects, const T* __restrict__ Fpool,
                                                        const T* __restrict__ g, int nx, int ny, T* __restrict__ wout,
                                                        T* __restrict__ w4, int bx, int by, int Nx,
                                                        const double* __restrict__ sc, FusedUpdate U,
                                                        PreResidual<T> Pr) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;  // PCG already converged
    double al = 0.0;
    if (U.gin) {
        // alpha = rho' / p.q from the partials of k_dir_apply (every workgroup forms it)
        __shared__ double red[4];
        const int t = threadIdx.x;
        double v = 0.0;
        for (int j = t; j < U.nred; j += 256) v += U.part[j];
        v = wave_sum(v);
        if ((t & 63) == 0) red[t >> 6] = v;
        __syncthreads();
        const double pq = red[0] + red[1] + red[2] + red[3];
        const double rho = U.sc[SC_RHO_NEW];
        al = rho / pq;
        const bool bad = !(pq > 0.0) || !(pq < INFINITY);
        if (blockIdx.x == 0 && t == 0) {
            U.sc[SC_RHO] = rho;
            U.sc[SC_PENDING] = 0.0;
            U.sc[SC_PQ] = pq;
            U.sc[SC_ALPHA] = al;
            U.hist[2 * (int)U.sc[SC_IT]] = al;
            if (bad) {
                U.sc[SC_FLAG] = 1.0;
                U.sc[SC_DONE] = 1.0;
            }
        }
        if (bad) return;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const Rect R = rects[blockIdx.x];
    const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
    const int n = m * mh;
    const long long fs = tw_size(m, mh);
    const T* Fg = Fpool + R.off;
    const int tid = threadIdx.x;
    const T* F;
    T* vec;
    constexpr bool STAGED = MODE == 1;          // staged before the sweeps
    constexpr bool OVERLAP = MODE == 2 && !GENERIC;  // staged during the forward sweeps
    if constexpr (STAGED) {
        using V = float4;
        constexpr int PER = 16 / sizeof(T);
        constexpr int U = 8;
        const V* src = reinterpret_cast<const V*>(Fg);
        V* dst = reinterpret_cast<V*>(sm);
        const int nvec = (int)((fs + PER - 1) / PER);
        int e = tid;
        for (; e + (U - 1) * 256 < nvec; e += U * 256) {
            V v[U];
#pragma unroll
            for (int q = 0; q < U; ++q) v[q] = src[e + q * 256];
#pragma unroll
            for (int q = 0; q < U; ++q) dst[e + q * 256] = v[q];
        }
        for (; e < nvec; e += 256) dst[e] = src[e];
        F = sm;
        vec = sm + ((fs + 3) & ~3LL);
    } else if constexpr (OVERLAP) {
        F = sm;  // filled by waves 2 and 3 during the forward sweeps
        vec = sm + ((fs + 3) & ~3LL);
    } else {
        F = Fg;
        vec = sm;
    }
    T* u = vec + ((n + 3) & ~3);
    T* mid = u + ((n + 3) & ~3);  // 2 * 64
    // the scale from the staged copy (read once from global memory)
    if constexpr (STAGED) __syncthreads();
    const T* Sg = (OVERLAP ? Fg : F) + tw_scale(m, mh);
    const int I = blockIdx.x % Nx, J = blockIdx.x / Nx;
    if (Pr.z1) {
        // z1' = z1 + W c on the patch and its one-vertex halo (LDS, FP64 of the stored
        // value), the own block's z1' written out, then t = g - K z1' in FP64, rounded once
        const int pw = m + 2, ph = mh + 2, mu = Pr.mu, nown = bx * by;
        const size_t zoff = ((reinterpret_cast<size_t>(mid + 2 * 64) + 15) & ~(size_t)15);
        double* Zt = reinterpret_cast<double*>(zoff);
        T* cb = reinterpret_cast<T*>(Zt + pw * ph);  // [9][mu]: the 3 x 3 blocks around K_i
        const int Ny = ny / by;
        for (int e = tid; e < 9 * mu; e += 256) {
            const int nb = e / mu, u = e % mu, Ib = I + nb % 3 - 1, Jb = J + nb / 3 - 1;
            T val = T(0);
            if (Ib >= 0 && Ib < Nx && Jb >= 0 && Jb < Ny) {
                const int b = Jb * Nx + Ib;
                if (u < Pr.nunk[b]) val = Pr.c[Pr.unk[(long long)b * mu + u]];
            }
            cb[e] = val;
        }
        __syncthreads();
        for (int e = tid; e < pw * ph; e += 256) {
            const int ii = R.i0 + e % pw, jj = R.j0 + e / pw;
            const bool own = ii >= I * bx && ii < (I + 1) * bx && jj >= J * by && jj < (J + 1) * by;
            const long long v = (long long)jj * nx + ii;
            double val = 0.0;
            if (ii >= 1 && ii < nx && jj >= 1 && jj < ny) {
                // vertex (ii, jj) lies in block (ii / bx, jj / by): neighbour nb of K_i
                const int Ib = ii / bx, Jb = jj / by, b = Jb * Nx + Ib;
                const int nb = (Jb - J + 1) * 3 + (Ib - I + 1);
                const T* Wv = Pr.W + ((long long)b * nown + (jj % by) * bx + ii % bx) * mu;
                const T* cv = cb + nb * mu;
                const int nu = Pr.nunk[b];
                T s = T(0);
                for (int u = 0; u < nu; ++u) s += Wv[u] * cv[u];
                const T zz = Pr.z1[v] + s;
                val = double(zz);
                if (own) Pr.z1p[v] = zz;
            } else if (own && ii < nx && jj < ny) {
                Pr.z1p[v] = T(0);
            }
            Zt[e] = val;
        }
        __syncthreads();
        for (int r = tid; r < n; r += 256) {
            const int aa = r % m, bb = r / m;
            const long long v = (long long)(R.j0 + 1 + bb) * nx + R.i0 + 1 + aa;
            const VertexData d = vertex_data(Pr.g, Pr.a, v, nx, true);
            vec[r] = Sg[r] * T(d.g - stencil_at4(Zt, pw, aa + 1, bb + 1, d.A, Pr.sx2, Pr.sy2));
        }
    } else
    for (int r = tid; r < n; r += 256) {
        const int aa = r % m, bb = r / m, i = R.i0 + 1 + aa, j = R.j0 + 1 + bb;
        const long long v = (long long)j * nx + i;
        T gv;
        if (U.gin) {
            const double gn = U.gin[v] - al * U.q[v];
            if (i >= I * bx && i < (I + 1) * bx && j >= J * by && j < (J + 1) * by) {
                U.gout[v] = gn;
                U.x[v] += al * U.p[v];
            }
            gv = T(gn);
        } else {
            gv = g[v];
        }
        vec[r] = Sg[r] * gv;
    }
    __syncthreads();
    const long long plane = (long long)nx * ny;
    const PatchOut<T> out{wout + R.voff, w4, plane, m, nx, R.i0, R.j0, I * bx, (I + 1) * bx, J * by, (J + 1) * by};
    if constexpr (GENERIC)
        solve_patch_any<T>(m, mh, F, vec, u, mid, out);
    else if (m == M1)
        solve_patch<T, M1, STAGED ? 1 : TGMS_PF_DIRECT>(mh, F, STAGED ? F : Fg, vec, u, mid, out, OVERLAP ? fs : 0);
    else
        solve_patch<T, M2, STAGED ? 1 : TGMS_PF_DIRECT>(mh, F, STAGED ? F : Fg, vec, u, mid, out, OVERLAP ? fs : 0);
}

// Fixed-width pairs (interior width, boundary-clipped width) with an overlap of
// two cells for blocks of 4, 6, 8, 12, 16, 20, 24 and 28 cells; other widths take
// the clamped path.
#define TGMS_TW_PAIRS(X) X(7, 5) X(9, 7) X(11, 9) X(15, 13) X(19, 17) X(23, 21) X(27, 25) X(31, 29)

template <typename T, int M1, int M2, bool GENERIC, int MODE>
void launch_tw(tgms_ctx* c, const T* L, const T* g, T* w, size_t lds, const double* sc, const FusedUpdate& U,
               const PreResidual<T>& Pr) {
    T* w4 = nullptr;
    if (c->slots) w4 = sizeof(T) == 8 ? (T*)c->patW4 : (T*)c->patW4_32;
    if (c->prof) {
        // events recorded by the dispatch itself (kernel execution only)
        hipEvent_t e1 = tgms::take_event(c), e2 = tgms::take_event(c);
        hipExtLaunchKernelGGL((k_smooth_twisted<T, M1, M2, GENERIC, MODE>), dim3(c->nblk), dim3(256), lds,
                              c->stream, e1, e2, 0, c->patch, L, g, c->nx, c->ny, w, w4, c->bx, c->by, c->Nx, sc, U, Pr);
        c->prof_rec.push_back({tgms::PK_SMOOTH, c->prof_iter, e1, e2});
    } else {
        hipLaunchKernelGGL((k_smooth_twisted<T, M1, M2, GENERIC, MODE>), dim3(c->nblk), dim3(256), lds, c->stream,
                           c->patch, L, g, c->nx, c->ny, w, w4, c->bx, c->by, c->Nx, sc, U, Pr);
    }
}

// m1 >= m2: the two row widths present among the patches (equal when all
// patches have one width, -1 when there are more than two)
template <typename T, int MODE>
void dispatch_mode(tgms_ctx* c, int m1, int m2, const T* L, const T* g, T* w, size_t lds, const double* sc,
                   const FusedUpdate& U, const PreResidual<T>& Pr) {
#define TGMS_TW_CASE(A, B)                                        \
    if (m1 == A && (m2 == B || m2 == A)) {                        \
        launch_tw<T, A, B, false, MODE>(c, L, g, w, lds, sc, U, Pr); \
        return;                                                   \
    }
    TGMS_TW_PAIRS(TGMS_TW_CASE)
#undef TGMS_TW_CASE
    launch_tw<T, 0, 0, true, MODE == 1 ? 1 : 0>(c, L, g, w, lds, sc, U, Pr);
}

template <typename T>
void dispatch_twisted(tgms_ctx* c, int m1, int m2, int mode, const T* L, const T* g, T* w, size_t lds,
                      const double* sc, const FusedUpdate& U, const PreResidual<T>& Pr) {
    if (mode == 1)
        dispatch_mode<T, 1>(c, m1, m2, L, g, w, lds, sc, U, Pr);
    else if (mode == 2)
        dispatch_mode<T, 2>(c, m1, m2, L, g, w, lds, sc, U, Pr);
    else
        dispatch_mode<T, 0>(c, m1, m2, L, g, w, lds, sc, U, Pr);
}

template <typename T>
void allow_lds(int lds_max) {
    auto set = [&](const void* f) { (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max); };
#define TGMS_TW_ATTR(A, B)                                 \
    set((const void*)k_smooth_twisted<T, A, B, false, 1>); \
    set((const void*)k_smooth_twisted<T, A, B, false, 2>);
    TGMS_TW_PAIRS(TGMS_TW_ATTR)
#undef TGMS_TW_ATTR
    set((const void*)k_smooth_twisted<T, 0, 0, true, 1>);
}

}  // namespace

namespace tgms {

long long patch_factor_size(int m, int mh) { return tw_size(m, mh); }

void factor_patches_launch(tgms_ctx* c, int* fail, int max_groups) {
    const int m = c->pat_bmax - 1;
    if (m > 32) throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patch wider than 33 cells"};
    const size_t lds = (size_t)(6 * c->pat_nmax + 3 * m * m) * sizeof(double);
    if (lds > (size_t)c->lds_max) throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patch too large for LDS"};
    (void)hipFuncSetAttribute((const void*)k_patch_factor, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    allow_lds<double>(c->lds_max);
    allow_lds<float>(c->lds_max);
    (void)hipGetLastError();
    const int groups = max_groups > 0 ? std::min(c->nblk, max_groups) : c->nblk;
    hipLaunchKernelGGL(k_patch_factor, dim3(groups), dim3(64), lds, c->stream, c->patch, c->a, c->nx,
                       c->sx * c->sx, c->sy * c->sy, c->patL, fail, c->nblk);
    LAUNCH_OK();
    if (c->patL32) cast_d2f(c, c->pat_pool, c->patL, c->patL32);
}

void factor_patches(tgms_ctx* c) {
    int* fail = c->alloc_scratch_int();
    factor_patches_launch(c, fail, 0);
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (h) throw TgmsError{TGMS_E_INVAL, "smoother patch matrix is not positive definite"};
}

// local solves of every patch on g into the patch solution pool (patW / patW32)
template <typename T>
void smooth_patches(tgms_ctx* c, const T* g, const double* sc, const FusedUpdate* fu, const PreResidual<T>* pr) {
    const T* L;
    T* w;
    if constexpr (sizeof(T) == 8) {
        L = (const T*)c->patL;
        w = (T*)c->patW;
    } else {
        L = (const T*)c->patL32;
        w = (T*)c->patW32;
    }
    size_t work = (size_t)(2 * ((c->pat_nmax + 3) & ~3) + 2 * 64) * sizeof(T);
    if (pr && pr->z1)  // the patch tile of z1' (16-byte aligned) and the coarse coefficients
        work += 16 + (size_t)c->pat_zmax * sizeof(double) + 9 * (size_t)pr->mu * sizeof(T);
    const size_t staged = (size_t)((c->pat_fmax + 3) & ~3LL) * sizeof(T) + work;
    // 1 / 2 (staged before / during the forward sweeps) where the factor fits in LDS (+ the
    // static scalars), else 0 (direct reads); -1: staged before where it fits
    int mode = c->smooth_staged < 0 ? 1 : c->smooth_staged;
    if (mode != 0 && staged + 64 > (size_t)c->lds_max) mode = 0;
    const FusedUpdate none{};
    const PreResidual<T> plain{};
    dispatch_twisted<T>(c, c->pat_m1, c->pat_m2, mode, L, g, w, mode ? staged : work, sc, fu ? *fu : none,
                        pr ? *pr : plain);
    LAUNCH_OK();
}
template void smooth_patches<double>(tgms_ctx*, const double*, const double*, const FusedUpdate*,
                                     const PreResidual<double>*);
template void smooth_patches<float>(tgms_ctx*, const float*, const double*, const FusedUpdate*,
                                    const PreResidual<float>*);

}  // namespace tgms
