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

namespace {

// ------------------------------------------------------------------ factorisation
// One workgroup of four waves per patch (the elimination is a chain of pivot steps per
// block row, so the patch's latency falls with the threads sharing each step).  LDS:
// the scaled stencil (c, e, n, ne, nw per vertex), the scale S, and three m x m work
// matrices.
constexpr int FAC_NT = 256;
constexpr int FAC_MAXE = 1024 / FAC_NT;  // m*m <= 1024 entries

// In-place Gauss-Jordan inversion of the SPD matrix W (m x m, row-major) by one
// workgroup; the pivots are Schur-complement diagonals, positive for SPD input.
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
            const int e = lane + FAC_NT * t;
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
            const int e = lane + FAC_NT * t;
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

__global__ void __launch_bounds__(FAC_NT) k_patch_factor(const Rect* __restrict__ rects, const double* __restrict__ a,
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
        double* Bout = F + tw_links(m, mh);
        double* Sout = F + tw_scale(m, mh);
        const int trip = tw_trip(m), b3 = tw_b3(m);
        // stencil couplings of each interior vertex with its east, north, north-east
        // and north-west neighbours (zero where the neighbour is not a patch vertex)
        for (int r = lane; r < n; r += FAC_NT) {
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
        for (int r = lane; r < n; r += FAC_NT) {
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
        // the coupling blocks (three rows of m words per link, zero-padded to b3)
        for (int e = lane; e < (mh - 1) * b3; e += FAC_NT) {
            const int l = e / b3, q = e - l * b3, which = q / m, sidx = q - which * m;
            const double* src = which == 0 ? kn : which == 1 ? kne : knw;
            Bout[e] = which < 3 ? src[l * m + sidx] : 0.0;
        }
        const PatchStencil P{kc, ke, kn, kne, knw, m};
        for (int e = lane; e < mm; e += FAC_NT) Mid[e] = P.A(k, e / m, e % m);
        auto store_pivot = [&](int j) {
            for (int e = lane; e < mm; e += FAC_NT) {
                const int r = e / m, s = e - r * m;
                if (r >= s) Pout[(long long)j * trip + tw_offP(s, m) + (r - s)] = W[e];
            }
            for (int e = tw_tri(m) + lane; e < trip; e += FAC_NT) Pout[(long long)j * trip + e] = 0.0;
        };
        // top sweep: rows 0..k-1
        if (k >= 1)
            for (int e = lane; e < mm; e += FAC_NT) W[e] = P.A(0, e / m, e % m);
        __syncthreads();
        for (int j = 0; j < k; ++j) {
            gj_invert(W, m, fail);
            store_pivot(j);
            // G = B_j T_j^{-1}; B_j[r][s] = kn(s) (r = s), kne(s) (r = s+1), knw(s) (r = s-1) at row j
            const int o = j * m;
            for (int e = lane; e < mm; e += FAC_NT) {
                const int r = e / m, s = e - r * m;
                double g = kn[o + r] * W[r * m + s];
                if (r >= 1) g += kne[o + r - 1] * W[(r - 1) * m + s];
                if (r + 1 < m) g += knw[o + r + 1] * W[(r + 1) * m + s];
                G[e] = g;
            }
            __syncthreads();
            // G B_j^T, subtracted from the next diagonal block (or from the middle one)
            for (int e = lane; e < mm; e += FAC_NT) {
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
            for (int e = lane; e < mm; e += FAC_NT) W[e] = P.A(mh - 1, e / m, e % m);
        __syncthreads();
        for (int j = mh - 1; j > k; --j) {
            gj_invert(W, m, fail);
            store_pivot(j);
            // H = B_{j-1}^T U_j^{-1}
            const int o = (j - 1) * m;
            for (int e = lane; e < mm; e += FAC_NT) {
                const int r = e / m, s = e - r * m;
                double h = kn[o + r] * W[r * m + s];
                if (r + 1 < m) h += kne[o + r] * W[(r + 1) * m + s];
                if (r >= 1) h += knw[o + r] * W[(r - 1) * m + s];
                G[e] = h;
            }
            __syncthreads();
            // H B_{j-1}
            for (int e = lane; e < mm; e += FAC_NT) {
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
        for (int e = lane; e < mm; e += FAC_NT) W[e] = Mid[e];
        __syncthreads();
        gj_invert(W, m, fail);
        store_pivot(k);
        __syncthreads();  // LDS is reused by the next patch
    }
}

// ------------------------------------------------------------------ application
// Per patch: psi = S K~^{-1} S g on the patch's interior vertices, by the chains of
// patch.h.  Wave 0 runs the top chains and wave 1 the bottom ones; lane a holds entry
// a of the current block vector.  A dense symmetric product P v broadcasts the
// entries of v with readlane; a tridiagonal product with B_l takes the neighbouring
// lanes' entries by wave shifts (DPP).  Every step's pivot and coupling blocks are
// staged in LDS by the wave that uses them, with 16-byte loads over all 64 lanes (the
// loads of the next two steps in flight while a step computes), and each lane reads
// its row there: few, full-width memory instructions instead of one narrow load per
// row entry.

// v of lane a-1 (0 on lane 0) and of lane a+1 (0 on lane 63)
__device__ inline int dpp_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ inline int dpp_shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ inline float shr1(float v) { return __int_as_float(dpp_shr1(__float_as_int(v))); }
__device__ inline float shl1(float v) { return __int_as_float(dpp_shl1(__float_as_int(v))); }
__device__ inline double shr1(double v) {
    return __hiloint2double(dpp_shr1(__double2hiint(v)), dpp_shr1(__double2loint(v)));
}
__device__ inline double shl1(double v) {
    return __hiloint2double(dpp_shl1(__double2hiint(v)), dpp_shl1(__double2loint(v)));
}

// (B v)_a and (B^T v)_a from the coupling rows n, e, w of lane a (v zero beyond the
// patch row, so that the shifts bring zeros in)
template <typename T>
__device__ inline T b_apply(T n, T e, T w, T v) { return n * v + shr1(e * v) + shl1(w * v); }
template <typename T>
__device__ inline T bt_apply(T n, T e, T w, T v) { return n * v + e * shl1(v) + w * shr1(v); }

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

// 16 bytes as a native vector (kept in registers where a HIP vector struct array
// is not)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The blocks of one chain step of a patch with rows of M vertices: the pivot block
// P_j (packed, padded to TRIP words) and the coupling block B_l (B3 words), staged
// together in one LDS slot of SW words.
template <typename T, int M>
struct Blocks {
    static constexpr int TRIP = (M * (M + 1) / 2 + 3) & ~3, B3 = (3 * M + 3) & ~3, SW = TRIP + B3;
    static constexpr int VW = 16 / (int)sizeof(T);  // words per 16-byte vector
    static constexpr int NVP = TRIP / VW, NV = SW / VW, PER = (NV + 63) / 64;
    using V = u32x4;
    const T* P;   // the patch's pivot blocks (global memory)
    const T* Bq;  // its coupling blocks
    int lane;
    // every lane loads (lanes past the blocks re-read the last vector): no branch, so
    // the loaded registers are only waited for where they are stored
    __device__ void load(V (&r)[PER], int prow, int link) const {
        const V* gp = reinterpret_cast<const V*>(P + (long long)prow * TRIP);
        const V* gb = reinterpret_cast<const V*>(Bq + (long long)link * B3);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int v = lane + 64 * q, vb = v - NVP;
            r[q] = v < NVP ? gp[v] : gb[vb < NV - NVP ? vb : NV - NVP - 1];
        }
    }
    __device__ void store(const V (&r)[PER], T* slot) const {
        V* d = reinterpret_cast<V*>(slot);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int v = lane + 64 * q;
            if (v < NV) d[v] = r[q];
        }
    }
};

// Row a of a staged step: the pivot row and the three coupling entries
template <typename T, int M>
struct StepRow {
    T pr[M];
    T n, e, w;
};

// P[a][c] of a packed symmetric block: (c, a) below the diagonal for c <= a, (a, c)
// otherwise; offa = offP(a) - a (formed once per lane)
template <int M>
__device__ inline int packed_at(int a, int offa, int c) {
    return c <= a ? tw_offP(c, M) - c + a : offa + c;
}

template <typename T, int M>
__device__ inline void read_row(StepRow<T, M>& R, const T* slot, int offa, int a, bool act) {
#pragma unroll
    for (int c = 0; c < M; ++c) R.pr[c] = slot[packed_at<M>(a, offa, c)];
    const T* b = slot + Blocks<T, M>::TRIP;
    R.n = act ? b[a] : T(0);
    R.e = act ? b[M + a] : T(0);
    R.w = act ? b[2 * M + a] : T(0);
}

// `steps` chain steps of one wave; step t uses the pivot block of row prow(t) and the
// coupling block of link lnk(t), in LDS slot slot(t).  FILL: the wave stages them
// there itself (the loads of steps t+1 and t+2 in flight in registers while step t
// computes); otherwise they are in their slots already.  body(t, row) forms the step.
template <typename T, int M, bool FILL, typename ProwOf, typename LinkOf, typename SlotOf, typename Body>
__device__ inline void staged_steps(const Blocks<T, M>& bk, int steps, ProwOf prow, LinkOf lnk, SlotOf slot,
                                    int offa, int a, bool act, Body body) {
    if (steps <= 0) return;
    using V = u32x4;
    constexpr int PER = Blocks<T, M>::PER;
    // two register buffers named apart (constant indices only, so that they stay in
    // registers): at step t, `next` holds step t+1 and the other one step t+2
    V ra[PER], rb[PER];
    if constexpr (FILL) {
        bk.load(ra, prow(0), lnk(0));
        if (steps > 1) bk.load(rb, prow(1), lnk(1));
        bk.store(ra, slot(0));
        if (steps > 2) bk.load(ra, prow(2), lnk(2));
    }
    auto step = [&](int t, V (&next)[PER]) __attribute__((always_inline)) {
        StepRow<T, M> row;
        read_row<T, M>(row, slot(t), offa, a, act);
        if constexpr (FILL) {
            // step t+1 into its slot (the slot of step t-1, whose rows are read), then
            // the registers take step t+3
            if (t + 1 < steps) bk.store(next, slot(t + 1));
            if (t + 3 < steps) bk.load(next, prow(t + 3), lnk(t + 3));
        }
        body(t, row);
    };
    for (int t0 = 0; t0 < steps; t0 += 2) {
        step(t0, rb);
        if (t0 + 1 < steps) step(t0 + 1, ra);
    }
}

// One patch (fixed row width M).  LDS: vec (b, then the forward chains' w), u, mid
// (the two chains' last products), the middle row's pivot block and the chain slots:
// KEEP: one slot per forward step and wave (the backward chains read them again
// without touching global memory); otherwise two per wave, refilled by the backward
// chains.
template <typename T, int M, bool KEEP>
__device__ inline void solve_patch(int mh, const T* Fg, T* vec, T* u, T* mid, const T* midP, T* slots,
                                   const PatchOut<T>& out) {
    using Bk = Blocks<T, M>;
    constexpr int SW = Bk::SW;
    const int k = mh / 2, top = k, bot = mh - 1 - k;
    // the wave index in a scalar register: the branches on it are taken by whole waves
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const bool act = lane < M;
    const int a = act ? lane : M - 1;
    const T* S = Fg + tw_scale(M, mh);
    const Bk bk{Fg, Fg + tw_links(M, mh), lane};
    const int offa = tw_offP(a, M) - a;
    T* my = slots + (KEEP ? wave * k : wave * 2) * SW;  // this wave's slots
    auto sl = [=](int t) { return my + (KEEP ? t : (t & 1)) * SW; };
    if (wave == 0) {
        // u_t = P_t w_t; w_{t+1} = b_{t+1} - B_t u_t, the last product into mid
        T v = vec[a];
        staged_steps<T, M, true>(bk, top, [](int t) { return t; }, [](int t) { return t; }, sl, offa, a, act,
                                 [&](int t, const StepRow<T, M>& r) {
                                     const T ut = dot_lanes<T, M>(r.pr, v);
                                     if (act) u[t * M + a] = ut;
                                     const T z = b_apply(r.n, r.e, r.w, act ? ut : T(0));
                                     if (t + 1 < top)
                                         v = vec[(t + 1) * M + a] - z;
                                     else if (act)
                                         mid[a] = z;
                                 });
        if (top == 0 && act) mid[a] = T(0);
    } else {
        // u_r = P_r w_r; w_{r-1} = b_{r-1} - B_{r-1}^T u_r from r = mh-1 down, the last into mid + 64
        T v = vec[(mh - 1) * M + a];
        staged_steps<T, M, true>(
            bk, bot, [=](int i) { return mh - 1 - i; }, [=](int i) { return mh - 2 - i; }, sl, offa, a, act,
            [&](int i, const StepRow<T, M>& r) {
                const int row = mh - 1 - i;
                const T ur = dot_lanes<T, M>(r.pr, v);
                if (act) u[row * M + a] = ur;
                const T z = bt_apply(r.n, r.e, r.w, act ? ur : T(0));
                if (row - 1 > k)
                    v = vec[(row - 1) * M + a] - z;
                else if (act)
                    mid[64 + a] = z;
            });
        if (bot == 0 && act) mid[64 + a] = T(0);
    }
    __syncthreads();
    if (wave == 0) {
        // the middle row: x_k = P_k (b_k - B_{k-1} u_{k-1} - B_k^T u_{k+1})
        T pr[M];
#pragma unroll
        for (int c = 0; c < M; ++c) pr[c] = midP[packed_at<M>(a, offa, c)];
        const T xk = dot_lanes<T, M>(pr, vec[k * M + a] - mid[a] - mid[64 + a]);
        if (act) {
            u[k * M + a] = xk;
            out.put(k, a, S[k * M + a] * xk);
        }
    }
    __syncthreads();
    T x = u[k * M + a];
    if (wave == 0) {
        // x_l = u_l - P_l B_l^T x_{l+1}, l = k-1 .. 0
        staged_steps<T, M, !KEEP>(bk, top, [=](int t) { return k - 1 - t; }, [=](int t) { return k - 1 - t; },
                                  [=](int t) { return KEEP ? my + (k - 1 - t) * SW : my + (t & 1) * SW; }, offa, a,
                                  act, [&](int t, const StepRow<T, M>& r) {
                                      const int l = k - 1 - t;
                                      const T y = bt_apply(r.n, r.e, r.w, act ? x : T(0));
                                      x = u[l * M + a] - dot_lanes<T, M>(r.pr, y);
                                      if (act) out.put(l, a, S[l * M + a] * x);
                                  });
    } else {
        // x_{l+1} = u_{l+1} - P_{l+1} B_l x_l, l = k .. mh-2 (forward slot mh-2-l)
        staged_steps<T, M, !KEEP>(bk, bot, [=](int t) { return k + 1 + t; }, [=](int t) { return k + t; },
                                  [=](int t) { return KEEP ? my + (bot - 1 - t) * SW : my + (t & 1) * SW; }, offa,
                                  a, act, [&](int t, const StepRow<T, M>& r) {
                                      const int l = k + t;
                                      const T y = b_apply(r.n, r.e, r.w, act ? x : T(0));
                                      x = u[(l + 1) * M + a] - dot_lanes<T, M>(r.pr, y);
                                      if (act) out.put(l + 1, a, S[(l + 1) * M + a] * x);
                                  });
    }
}

// Any row width m <= 64: the same chains with runtime loops over the columns, the
// blocks read from global memory directly.  Used for widths without a fixed-width
// instantiation.
template <typename T>
__device__ inline void solve_patch_any(int m, int mh, const T* Fg, T* vec, T* u, T* mid, const PatchOut<T>& out) {
    const int k = mh / 2, top = k, bot = mh - 1 - k, trip = tw_trip(m), b3 = tw_b3(m);
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const bool act = lane < m;
    const int a = act ? lane : 0;
    const T* P = Fg;
    const T* Bq = Fg + tw_links(m, mh);
    const T* S = Fg + tw_scale(m, mh);
    auto pdot = [&](int j, T v) {  // (P_j v)_a
        const T* Pj = P + (long long)j * trip;
        T s = T(0);
        for (int c = 0; c < m; ++c) {
            const T pac = c <= a ? Pj[tw_offP(c, m) + a - c] : Pj[tw_offP(a, m) + c - a];
            s += pac * readlane(v, c);
        }
        return s;
    };
    auto cpl = [&](int l, T& n, T& e, T& w) {
        const T* b = Bq + (long long)l * b3;
        n = act ? b[a] : T(0);
        e = act ? b[m + a] : T(0);
        w = act ? b[2 * m + a] : T(0);
    };
    if (wave == 0) {
        T v = vec[a];
        for (int t = 0; t < top; ++t) {
            T n, e, w;
            cpl(t, n, e, w);
            const T ut = pdot(t, v);
            if (act) u[t * m + a] = ut;
            const T z = b_apply(n, e, w, act ? ut : T(0));
            if (t + 1 < top)
                v = vec[(t + 1) * m + a] - z;
            else if (act)
                mid[a] = z;
        }
        if (top == 0 && act) mid[a] = T(0);
    } else if (wave == 1) {
        T v = vec[(mh - 1) * m + a];
        for (int row = mh - 1; row > k; --row) {
            T n, e, w;
            cpl(row - 1, n, e, w);
            const T ur = pdot(row, v);
            if (act) u[row * m + a] = ur;
            const T z = bt_apply(n, e, w, act ? ur : T(0));
            if (row - 1 > k)
                v = vec[(row - 1) * m + a] - z;
            else if (act)
                mid[64 + a] = z;
        }
        if (bot == 0 && act) mid[64 + a] = T(0);
    }
    __syncthreads();
    if (wave == 0) {
        const T xk = pdot(k, vec[k * m + a] - mid[a] - mid[64 + a]);
        if (act) {
            u[k * m + a] = xk;
            out.put(k, a, S[k * m + a] * xk);
        }
    }
    __syncthreads();
    T x = u[k * m + a];
    if (wave == 0) {
        for (int l = k - 1; l >= 0; --l) {
            T n, e, w;
            cpl(l, n, e, w);
            const T y = bt_apply(n, e, w, act ? x : T(0));
            x = u[l * m + a] - pdot(l, y);
            if (act) out.put(l, a, S[l * m + a] * x);
        }
    } else if (wave == 1) {
        for (int l = k; l <= mh - 2; ++l) {
            T n, e, w;
            cpl(l, n, e, w);
            const T y = b_apply(n, e, w, act ? x : T(0));
            x = u[(l + 1) * m + a] - pdot(l + 1, y);
            if (act) out.put(l + 1, a, S[(l + 1) * m + a] * x);
        }
    }
}

// LDS words of one workgroup beyond the input vectors: mid, the middle pivot block and
// the chain slots of a patch with rows of M vertices and at most mh rows
template <typename T, int M>
__host__ __device__ constexpr long long patch_lds_words(bool keep, int mh) {
    return 128 + Blocks<T, M>::TRIP + (keep ? 2LL * (mh / 2) : 4LL) * Blocks<T, M>::SW;
}

// One workgroup (two waves) per patch.  GENERIC: every patch takes the runtime-width
// path (m <= M1 unused); otherwise every patch has width M1 or M2.  KEEP: the chain
// slots hold every forward step (see solve_patch).
template <typename T, int M1, int M2, bool GENERIC, bool KEEP>
__global__ void __launch_bounds__(128) k_smooth_twisted(const Rect* __restrict__ rects, const T* __restrict__ Fpool,
                                                        const T* __restrict__ g, int nx, int ny, T* __restrict__ wout,
                                                        T* __restrict__ w4, int bx, int by, int Nx,
                                                        const double* __restrict__ sc) {
    constexpr int NW = 2, NT = NW * 64;
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;  // PCG already converged
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const Rect R = rects[blockIdx.x];
    const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
    const int n = m * mh;
    const T* Fg = Fpool + R.off;
    const int tid = threadIdx.x;
    T* vec = sm;
    T* u = vec + ((n + 3) & ~3);
    T* mid = u + ((n + 3) & ~3);  // 2 * 64
    T* midP = mid + 128;           // the middle row's pivot block (fixed widths)
    const int MW = GENERIC ? 0 : (m == M1 ? M1 : M2);
    const int trip = tw_trip(m), sw = trip + tw_b3(m);
    T* slots = midP + (GENERIC ? 0 : trip);
    (void)MW;
    (void)sw;
    if (!GENERIC) {
        // stage P_k (16-byte copies)
        using V = float4;
        constexpr int VW = 16 / (int)sizeof(T);
        const V* src = reinterpret_cast<const V*>(Fg + (long long)(mh / 2) * trip);
        V* dst = reinterpret_cast<V*>(midP);
        for (int e = tid; e < trip / VW; e += NT) dst[e] = src[e];
    }
    const T* Sg = Fg + tw_scale(m, mh);
    const int I = blockIdx.x % Nx, J = blockIdx.x / Nx;
    for (int r = tid; r < n; r += NT) {
        const int aa = r % m, bb = r / m;
        vec[r] = Sg[r] * g[(long long)(R.j0 + 1 + bb) * nx + R.i0 + 1 + aa];
    }
    __syncthreads();
    const long long plane = (long long)nx * ny;
    const PatchOut<T> out{wout + R.voff, w4, plane, m, nx, R.i0, R.j0, I * bx, (I + 1) * bx, J * by, (J + 1) * by};
    if constexpr (GENERIC)
        solve_patch_any<T>(m, mh, Fg, vec, u, mid, out);
    else if (m == M1)
        solve_patch<T, M1, KEEP>(mh, Fg, vec, u, mid, midP, slots, out);
    else
        solve_patch<T, M2, KEEP>(mh, Fg, vec, u, mid, midP, slots, out);
}

// Fixed-width pairs (interior width, boundary-clipped width) with an overlap of
// two cells for blocks of 4, 6, 8, 12, 16, 20, 24 and 28 cells; other widths take
// the runtime-width path.
#define TGMS_TW_PAIRS(X) X(7, 5) X(9, 7) X(11, 9) X(15, 13) X(19, 17) X(23, 21) X(27, 25) X(31, 29)

template <typename T, int M1, int M2, bool GENERIC, bool KEEP>
void launch_tw(tgms_ctx* c, const T* L, const T* g, T* w, size_t lds, const double* sc) {
    T* w4 = nullptr;
    if (c->slots) w4 = sizeof(T) == 8 ? (T*)c->patW4 : (T*)c->patW4_32;
    if (c->prof) {
        // events recorded by the dispatch itself (kernel execution only)
        hipEvent_t e1 = tgms::take_event(c), e2 = tgms::take_event(c);
        hipExtLaunchKernelGGL((k_smooth_twisted<T, M1, M2, GENERIC, KEEP>), dim3(c->nblk), dim3(128), lds,
                              c->stream, e1, e2, 0, c->patch, L, g, c->nx, c->ny, w, w4, c->bx, c->by, c->Nx, sc);
        c->prof_rec.push_back({tgms::PK_SMOOTH, c->prof_iter, e1, e2});
    } else {
        hipLaunchKernelGGL((k_smooth_twisted<T, M1, M2, GENERIC, KEEP>), dim3(c->nblk), dim3(128), lds, c->stream,
                           c->patch, L, g, c->nx, c->ny, w, w4, c->bx, c->by, c->Nx, sc);
    }
}

// LDS bytes of the smoother launch: the input vectors, mid, the middle pivot block and
// the chain slots (the widest patch and the tallest)
template <typename T>
size_t smooth_lds(const tgms_ctx* c, bool keep, int mw) {
    const long long trip = tw_trip(mw), sw = trip + tw_b3(mw);
    const long long words = 2 * ((c->pat_nmax + 3) & ~3LL) + 128 + trip + (keep ? 2LL * (c->pat_hmax / 2) : 4LL) * sw;
    return (size_t)words * sizeof(T);
}

// m1 >= m2: the two row widths present among the patches (equal when all
// patches have one width, -1 when there are more than two)
template <typename T, bool KEEP>
bool dispatch_keep(tgms_ctx* c, int m1, int m2, const T* L, const T* g, T* w, const double* sc) {
#define TGMS_TW_CASE(A, B)                                 \
    if (m1 == A && (m2 == B || m2 == A)) {                 \
        const size_t lds = smooth_lds<T>(c, KEEP, A);      \
        if (lds + 64 > (size_t)c->lds_max) return false;   \
        launch_tw<T, A, B, false, KEEP>(c, L, g, w, lds, sc); \
        return true;                                       \
    }
    TGMS_TW_PAIRS(TGMS_TW_CASE)
#undef TGMS_TW_CASE
    launch_tw<T, 0, 0, true, false>(c, L, g, w, smooth_lds<T>(c, false, 0), sc);
    return true;
}

template <typename T>
void allow_lds(int lds_max) {
    auto set = [&](const void* f) { (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max); };
#define TGMS_TW_ATTR(A, B)                                 \
    set((const void*)k_smooth_twisted<T, A, B, false, false>); \
    set((const void*)k_smooth_twisted<T, A, B, false, true>);
    TGMS_TW_PAIRS(TGMS_TW_ATTR)
#undef TGMS_TW_ATTR
    set((const void*)k_smooth_twisted<T, 0, 0, true, false>);
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
    hipLaunchKernelGGL(k_patch_factor, dim3(groups), dim3(FAC_NT), lds, c->stream, c->patch, c->a, c->nx,
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
void smooth_patches(tgms_ctx* c, const T* g, const double* sc) {
    const T* L;
    T* w;
    if constexpr (sizeof(T) == 8) {
        L = (const T*)c->patL;
        w = (T*)c->patW;
    } else {
        L = (const T*)c->patL32;
        w = (T*)c->patW32;
    }
    // 1: the forward chains' blocks kept in LDS for the backward chains (where they
    // fit); 0 (and -1): staged twice, two slots per wave
    if (c->smooth_staged == 1 && dispatch_keep<T, true>(c, c->pat_m1, c->pat_m2, L, g, w, sc)) {
        LAUNCH_OK();
        return;
    }
    if (!dispatch_keep<T, false>(c, c->pat_m1, c->pat_m2, L, g, w, sc))
        throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patch too large for LDS"};
    LAUNCH_OK();
}
template void smooth_patches<double>(tgms_ctx*, const double*, const double*);
template void smooth_patches<float>(tgms_ctx*, const float*, const double*);

}  // namespace tgms
