// The smoother S r = eta * sum_i ext((L_i^+)^{-1} R_i^+ r) (paper section 5,
// eq. smooth) on the oversampled blocks K_i^+ = K_i enlarged by the overlap.
//
// On K_i^+ with zero normal flux on its boundary, the local saddle solve has the
// divergence-free solution v = C psi with psi = (C^T A C)^{-1} C^T r on the
// patch's interior vertices (the 9-point stencil of the stream-function
// operator restricted to them).  The local matrices are factorised once per
// setup in the twisted block form described in patch.h; every smoother
// application is one launch over all patches followed by a gather.
#include "common.h"
#include "patch.h"

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
                                                     int* __restrict__ fail) {
    extern __shared__ double sm[];
    const Rect R = rects[blockIdx.x];
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
}

// ------------------------------------------------------------------ application
// Row r of a link (or, with stride m, its column) for lane `a`; entries beyond m
// are zero so that a fixed-width loop covers every patch width up to MM.
template <typename T, int MM>
__device__ inline void load_line(T (&v)[MM], const T* p, int stride, int m) {
#pragma unroll
    for (int c = 0; c < MM; ++c) {
        const int cc = c < m ? c : m - 1;
        const T x = p[cc * stride];
        v[c] = c < m ? x : T(0);
    }
}

// sum_c v[c] * (value of x held by lane c)
template <typename T, int MM>
__device__ inline T dot_lanes(const T (&v)[MM], T x) {
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
    for (int c = 0; c < MM; c += 4) {
        s0 += v[c] * readlane(x, c);
        if (c + 1 < MM) s1 += v[c + 1] * readlane(x, c + 1);
        if (c + 2 < MM) s2 += v[c + 2] * readlane(x, c + 2);
        if (c + 3 < MM) s3 += v[c + 3] * readlane(x, c + 3);
    }
    return (s0 + s1) + (s2 + s3);
}

// One dependent chain run by one wavefront: for t = 0..steps-1,
//   s = line(t) . x;  x = (t + 1 < steps or !last_to_mid) ? base[row(t)] - s : x
// where line(t) is row or column `a` of link lk(t).  Lane a (< m) holds entry a
// of the current vector.  Link lines are double-buffered in registers so that the
// LDS reads for step t+1 are in flight during step t.
template <typename T, int MM, typename LinkOf, typename Step>
__device__ inline void run_chain(int steps, const T* links, int m, int a, int stride, int elem, LinkOf lk, Step step) {
    if (steps <= 0) return;
    T ra[MM], rb[MM];
    const long long mm = (long long)m * m;
    load_line<T, MM>(ra, links + lk(0) * mm + (long long)a * elem, stride, m);
    int t = 0;
    while (true) {
        if (t + 1 < steps) load_line<T, MM>(rb, links + lk(t + 1) * mm + (long long)a * elem, stride, m);
        step(t, ra);
        if (++t >= steps) break;
        if (t + 1 < steps) load_line<T, MM>(ra, links + lk(t + 1) * mm + (long long)a * elem, stride, m);
        step(t, rb);
        if (++t >= steps) break;
    }
}

// Per patch: psi = S K~^{-1} S g on the patch's interior vertices.  Waves 0 and 1
// run the top and bottom chains, all four waves share the staging and the
// independent pivot products.  STAGED: the patch's factor is copied to LDS with
// 16-byte loads first; otherwise the chains read it from global memory.
template <typename T, int MM, bool STAGED>
__global__ void __launch_bounds__(256) k_smooth_twisted(const Rect* __restrict__ rects, const T* __restrict__ Fpool,
                                                        const T* __restrict__ g, int nx, T* __restrict__ wout) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const Rect R = rects[blockIdx.x];
    const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
    const int n = m * mh, k = mh / 2, tri = tw_tri(m);
    const long long fs = tw_size(m, mh);
    const T* Fg = Fpool + R.off;
    const int tid = threadIdx.x;
    const T* F;
    T* vec;
    if constexpr (STAGED) {
        using V = float4;
        constexpr int PER = 16 / sizeof(T);
        const V* src = reinterpret_cast<const V*>(Fg);
        V* dst = reinterpret_cast<V*>(sm);
        const int nvec = (int)((fs + PER - 1) / PER);
        int e = tid;
        for (; e + 3 * 256 < nvec; e += 4 * 256) {
            const V v0 = src[e], v1 = src[e + 256], v2 = src[e + 512], v3 = src[e + 768];
            dst[e] = v0;
            dst[e + 256] = v1;
            dst[e + 512] = v2;
            dst[e + 768] = v3;
        }
        for (; e < nvec; e += 256) dst[e] = src[e];
        F = sm;
        vec = sm + ((fs + 3) & ~3LL);
    } else {
        F = Fg;
        vec = sm;
    }
    T* u = vec + ((n + 3) & ~3);
    T* mid = u + ((n + 3) & ~3);  // 2 * MM
    const T* Pv = F;
    const T* Lk = F + tw_links(m, mh);
    const T* Sg = Fg + tw_scale(m, mh);
    for (int r = tid; r < n; r += 256) {
        const int aa = r % m, bb = r / m;
        vec[r] = Sg[r] * g[(long long)(R.j0 + 1 + bb) * nx + R.i0 + 1 + aa];
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const bool act = lane < m;
    const int a = act ? lane : 0;
    if (wave == 0) {
        // w_{l+1} = b_{l+1} - G_l w_l (l < k-1); the last product G_{k-1} w_{k-1} goes to the middle row
        T w = act ? vec[a] : T(0);
        run_chain<T, MM>(k, Lk, m, a, 1, m, [](int t) { return (long long)t; }, [&](int t, const T(&line)[MM]) {
            const T s = dot_lanes<T, MM>(line, w);
            if (t + 1 < k) {
                w = act ? vec[(t + 1) * m + a] - s : T(0);
                if (act) vec[(t + 1) * m + a] = w;
            } else if (act) {
                mid[a] = s;
            }
        });
        if (k == 0 && act) mid[a] = T(0);
    } else if (wave == 1) {
        // w_l = b_l - H_l w_{l+1} (l = mh-2 .. k+1); the last product H_k w_{k+1} goes to the middle row
        const int steps = mh - 1 - k;
        T w = act ? vec[(mh - 1) * m + a] : T(0);
        run_chain<T, MM>(steps, Lk, m, a, 1, m, [=](int t) { return (long long)(mh - 2 - t); },
                         [&](int t, const T(&line)[MM]) {
                             const int l = mh - 2 - t;
                             const T s = dot_lanes<T, MM>(line, w);
                             if (l > k) {
                                 w = act ? vec[l * m + a] - s : T(0);
                                 if (act) vec[l * m + a] = w;
                             } else if (act) {
                                 mid[MM + a] = s;
                             }
                         });
        if (steps == 0 && act) mid[MM + a] = T(0);
    }
    __syncthreads();
    if (tid < m) vec[k * m + tid] -= mid[tid] + mid[MM + tid];
    __syncthreads();
    // u_j = P_j w_j for every row (P_j symmetric, lower triangle packed by columns)
    for (int r = tid; r < n; r += 256) {
        const int j = r / m, aa = r - j * m;
        const T* Pj = Pv + (long long)j * tri;
        const T* wj = vec + j * m;
        T acc0 = T(0), acc1 = T(0);
        int c = 0;
        for (; c < aa; ++c) acc0 += Pj[tw_offP(c, m) + (aa - c)] * wj[c];
        const T* col = Pj + tw_offP(aa, m) - aa;
        for (; c < m; ++c) acc1 += col[c] * wj[c];
        u[r] = acc0 + acc1;
    }
    __syncthreads();
    const T* S = F + tw_scale(m, mh);
    T* out = wout + R.voff;
    if (wave == 0) {
        // x_k = u_k; x_l = u_l - G_l^T x_{l+1}, l = k-1 .. 0
        T x = act ? u[k * m + a] : T(0);
        if (act) out[k * m + a] = S[k * m + a] * x;
        run_chain<T, MM>(k, Lk, m, a, m, 1, [=](int t) { return (long long)(k - 1 - t); },
                         [&](int t, const T(&line)[MM]) {
                             const int l = k - 1 - t;
                             const T s = dot_lanes<T, MM>(line, x);
                             x = act ? u[l * m + a] - s : T(0);
                             if (act) out[l * m + a] = S[l * m + a] * x;
                         });
    } else if (wave == 1) {
        // x_{l+1} = u_{l+1} - H_l^T x_l, l = k .. mh-2
        T x = act ? u[k * m + a] : T(0);
        run_chain<T, MM>(mh - 1 - k, Lk, m, a, m, 1, [=](int t) { return (long long)(k + t); },
                         [&](int t, const T(&line)[MM]) {
                             const int l = k + t;
                             const T s = dot_lanes<T, MM>(line, x);
                             x = act ? u[(l + 1) * m + a] - s : T(0);
                             if (act) out[(l + 1) * m + a] = S[(l + 1) * m + a] * x;
                         });
    }
}

// z(v) = [z(v)] + eta * sum of the patch solutions covering v (fixed patch
// order, so the sum is deterministic; no atomics).
template <typename T>
__global__ void k_smooth_gather(const Rect* __restrict__ rects, const T* __restrict__ w, int nx, int ny, int bx,
                                int by, int Nx, int Ny, T eta, T* __restrict__ z, int accumulate) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const long long v = (long long)j * nx + i;
    T s = T(0);
    if (i > 0 && j > 0) {
        const int I0 = i / bx, J0 = j / by;
        for (int J = J0 - 1; J <= J0 + 1; ++J) {
            if (J < 0 || J >= Ny) continue;
            for (int I = I0 - 1; I <= I0 + 1; ++I) {
                if (I < 0 || I >= Nx) continue;
                const Rect R = rects[J * Nx + I];
                if (i > R.i0 && i < R.i1 && j > R.j0 && j < R.j1) {
                    const int m = R.i1 - R.i0 - 1;
                    s += w[R.voff + (long long)(j - R.j0 - 1) * m + (i - R.i0 - 1)];
                }
            }
        }
    }
    s *= eta;
    z[v] = accumulate ? z[v] + s : s;
}

template <typename T, int MM, bool STAGED>
void launch_twisted(tgms_ctx* c, const T* L, const T* g, T* w, size_t lds) {
    hipLaunchKernelGGL((k_smooth_twisted<T, MM, STAGED>), dim3(c->nblk), dim3(256), lds, c->stream, c->patch, L, g,
                       c->nx, w);
}

template <typename T, bool STAGED>
void dispatch_twisted(tgms_ctx* c, int mmax, const T* L, const T* g, T* w, size_t lds) {
    if (mmax <= 8)
        launch_twisted<T, 8, STAGED>(c, L, g, w, lds);
    else if (mmax <= 12)
        launch_twisted<T, 12, STAGED>(c, L, g, w, lds);
    else if (mmax <= 16)
        launch_twisted<T, 16, STAGED>(c, L, g, w, lds);
    else if (mmax <= 20)
        launch_twisted<T, 20, STAGED>(c, L, g, w, lds);
    else if (mmax <= 24)
        launch_twisted<T, 24, STAGED>(c, L, g, w, lds);
    else
        launch_twisted<T, 32, STAGED>(c, L, g, w, lds);
}

template <typename T>
void allow_lds(int lds_max) {
    (void)hipFuncSetAttribute((const void*)k_smooth_twisted<T, 8, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_twisted<T, 12, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_twisted<T, 16, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_twisted<T, 20, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_twisted<T, 24, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_twisted<T, 32, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
}

}  // namespace

namespace tgms {

long long patch_factor_size(int m, int mh) { return tw_size(m, mh); }

void factor_patches(tgms_ctx* c) {
    const int m = c->pat_bmax - 1;
    if (m > 32) throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patch wider than 33 cells"};
    const size_t lds = (size_t)(6 * c->pat_nmax + 3 * m * m) * sizeof(double);
    if (lds > (size_t)c->lds_max) throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patch too large for LDS"};
    (void)hipFuncSetAttribute((const void*)k_patch_factor, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    allow_lds<double>(c->lds_max);
    allow_lds<float>(c->lds_max);
    (void)hipGetLastError();
    int* fail = c->alloc<int>(1);
    HIP_OK(hipMemsetAsync(fail, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_patch_factor, dim3(c->nblk), dim3(64), lds, c->stream, c->patch, c->a, c->nx,
                       c->sx * c->sx, c->sy * c->sy, c->patL, fail);
    LAUNCH_OK();
    if (c->patL32) cast_d2f(c, c->pat_pool, c->patL, c->patL32);
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (h) throw TgmsError{TGMS_E_INVAL, "smoother patch matrix is not positive definite"};
}

template <typename T>
void smooth(tgms_ctx* c, const T* g, T* z, bool accumulate) {
    const T* L;
    T* w;
    if constexpr (sizeof(T) == 8) {
        L = (const T*)c->patL;
        w = (T*)c->patW;
    } else {
        L = (const T*)c->patL32;
        w = (T*)c->patW32;
    }
    const int mmax = c->pat_bmax - 1;
    const size_t work = (size_t)(2 * ((c->pat_nmax + 3) & ~3) + 2 * 32) * sizeof(T);
    const size_t staged = (size_t)((c->pat_fmax + 3) & ~3LL) * sizeof(T) + work;
    {
        ProfScope ps(c, PK_SMOOTH);
        if (staged <= (size_t)c->lds_max)
            dispatch_twisted<T, true>(c, mmax, L, g, w, staged);
        else
            dispatch_twisted<T, false>(c, mmax, L, g, w, work);
        LAUNCH_OK();
    }
    dim3 grid((c->nx + 63) / 64, (c->ny + 3) / 4);
    hipLaunchKernelGGL((k_smooth_gather<T>), grid, dim3(64, 4), 0, c->stream, c->patch, (const T*)w, c->nx, c->ny,
                       c->bx, c->by, c->Nx, c->Ny, T(c->eta), z, accumulate ? 1 : 0);
    LAUNCH_OK();
}
template void smooth<double>(tgms_ctx*, const double*, double*, bool);
template void smooth<float>(tgms_ctx*, const float*, float*, bool);

}  // namespace tgms
