// Local direct solvers on cell rectangles: coarse blocks K_i (preprocessing
// and snapshots, paper sections 3 and 4.1) and oversampled blocks K_i^+ (the
// smoother, eq. smooth).
//
// On a rectangle with zero normal flux on its boundary the local saddle
// problem R L R^T [v; p] = [r; 0] has the divergence-free solution
// v = C psi, psi = (C^T A C)^{-1} C^T r, with psi on the rectangle's interior
// vertices.  C^T A C is the global 9-point stencil restricted to those
// vertices: SPD and banded with lower bandwidth b = (interior vertices per
// row) + 1.  It is diagonally equilibrated, factorised by a band Cholesky in
// FP64 and then regrouped by vertex rows (block-row form of band.h).
#include "common.h"
#include "band.h"

namespace {

// One wavefront per rectangle; band matrix in LDS (n * (b+1) doubles).
template <bool WRITE32>
__global__ void k_band_factor(const Rect* __restrict__ rects, const double* __restrict__ a, int nx, double sx2,
                              double sy2, double* __restrict__ Lpool, double* __restrict__ Spool,
                              float* __restrict__ L32, int* __restrict__ fail) {
    extern __shared__ double M[];
    const Rect R = rects[blockIdx.x];
    const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
    const int n = m * mh, b = m + 1, ld = b + 1;
    const int lane = threadIdx.x;
    // assemble the column band of the 9-point stencil restricted to interior vertices
    for (int r = lane; r < n; r += TGMS_WAVE) {
        const int aa = r % m, bb = r / m;
        const int i = R.i0 + 1 + aa, j = R.j0 + 1 + bb;
        const long long v = (long long)j * nx + i;
        const Stencil9 k = stencil9(a[v - nx - 1], a[v - nx], a[v - 1], a[v], sx2, sy2);
        double* col = M + (long long)r * ld;
        for (int t = 0; t < ld; ++t) col[t] = 0.0;
        col[0] = k.c;
        if (aa + 1 < m) col[1] = k.e;
        if (bb + 1 < mh) {
            if (aa >= 1) col[m - 1] = k.nw;
            col[m] = k.n;
            if (aa + 1 < m) col[m + 1] = k.ne;
        }
    }
    __syncthreads();
    // equilibration: M' = S M S with S = diag(M)^{-1/2}
    for (int r = lane; r < n; r += TGMS_WAVE) Spool[R.voff + r] = 1.0 / sqrt(M[(long long)r * ld]);
    __syncthreads();
    for (int r = lane; r < n; r += TGMS_WAVE) {
        const double sr = Spool[R.voff + r];
        double* col = M + (long long)r * ld;
        for (int t = 0; t < ld && r + t < n; ++t) col[t] *= sr * Spool[R.voff + r + t];
    }
    __syncthreads();
    // right-looking band Cholesky
    const int npair = b * (b + 1) / 2;
    for (int cidx = 0; cidx < n; ++cidx) {
        double* col = M + (long long)cidx * ld;
        const double d = col[0];
        if (!(d > 0.0)) {
            if (lane == 0) atomicOr(fail, 1);
            return;
        }
        const double inv = 1.0 / sqrt(d);
        __syncthreads();
        if (lane >= 1 && lane <= b && cidx + lane < n) col[lane] *= inv;
        __syncthreads();
        for (int p = lane; p < npair; p += TGMS_WAVE) {
            // p -> (u, t'): u = 1..b, t' = 0..b-u, enumerated column by column
            int u = 1, rem = p;
            while (rem > b - u) {
                rem -= b - u + 1;
                ++u;
            }
            const int tp = rem;
            if (cidx + u + tp < n) M[(long long)(cidx + u) * ld + tp] -= col[u] * col[u + tp];
        }
        __syncthreads();
        if (lane == 0) col[0] = inv;
        __syncthreads();
    }
    // repack by vertex rows: D_j = L_jj^{-1} (lower, by columns), E_j = L_{j+1,j} (Hessenberg, by columns)
    const int tri = btri_tri(m), bs = tri + btri_hes(m);
    double* out = Lpool + R.off;
    for (int j = 0; j < mh; ++j) {
        double* D = out + (long long)j * bs;
        if (lane < m) {
            const int cc = lane;  // column of L_jj^{-1}: solve L_jj x = e_cc, rows cc..m-1
            for (int r = cc; r < m; ++r) {
                double acc = (r == cc) ? 1.0 : 0.0;
                for (int k = cc; k < r; ++k)
                    acc -= M[(long long)(j * m + k) * ld + (r - k)] * D[btri_offD(cc, m) + (k - cc)];
                // diagonal of L stored as its reciprocal
                D[btri_offD(cc, m) + (r - cc)] = acc * M[(long long)(j * m + r) * ld];
            }
        }
        if (j + 1 < mh) {
            double* E = D + tri;
            for (int e = lane; e < btri_hes(m); e += TGMS_WAVE) {
                int cc = 0;
                while (btri_offE(cc + 1) <= e && cc + 1 < m) ++cc;
                const int a = e - btri_offE(cc);  // row of E_j, a <= cc + 1
                E[e] = M[(long long)(j * m + cc) * ld + (m + a - cc)];
            }
        }
    }
    double* Sout = out + (long long)mh * bs;
    for (int r = lane; r < n; r += TGMS_WAVE) Sout[r] = Spool[R.voff + r];
    __syncthreads();
    if (WRITE32) {
        const long long tot = btri_size(m, mh);
        for (long long e = lane; e < tot; e += TGMS_WAVE) L32[R.off + e] = (float)out[e];
    }
}

// Smoother, phase 1: per patch, w = (C^T A C)^{-1} g on its interior vertices.
template <typename T, int MW>
__global__ void __launch_bounds__(64) k_smooth_patches(const Rect* __restrict__ rects, const T* __restrict__ L, const T* __restrict__ g,
                                 int nx, T* __restrict__ wout) {
    extern __shared__ unsigned char smem_raw[];
    T* tb = reinterpret_cast<T*>(smem_raw);
    T* xb = tb + 64;
    T* vec = xb + 64;
    const Rect R = rects[blockIdx.x];
    const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
    const int n = m * mh;
    const int lane = threadIdx.x;
    for (int r = lane; r < n; r += TGMS_WAVE) {
        const int aa = r % m, bb = r / m;
        vec[r] = g[(long long)(R.j0 + 1 + bb) * nx + R.i0 + 1 + aa];
    }
    __syncthreads();
    btri_solve_wave<T, MW>(L + R.off, m, mh, vec, tb, xb);
    __syncthreads();
    for (int r = lane; r < n; r += TGMS_WAVE) wout[R.voff + r] = vec[r];
}

// Smoother, phase 1 with the patch factor staged in LDS: the workgroup (4 waves) copies
// the whole factor with 16-byte loads, all in flight together; the block sweeps then
// read only LDS.  Factors start at 16-byte-aligned offsets (multiples of 4 words).
// Patches whose row width is M1 or M2 (the interior and the boundary-clipped widths)
// use the barrier-free compile-time-width solve; any other width the generic one.
template <typename T, int M1, int M2>
__global__ void __launch_bounds__(256) k_smooth_patches_lds(const Rect* __restrict__ rects, const T* __restrict__ L,
                                                            const T* __restrict__ g, int nx, T* __restrict__ wout) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tb = reinterpret_cast<T*>(smem_raw);
    T* xb = tb + 64;
    const Rect R = rects[blockIdx.x];
    const int m = R.i1 - R.i0 - 1, mh = R.j1 - R.j0 - 1;
    const int n = m * mh;
    T* vec = xb + 64;
    T* F = vec + ((n + 3) & ~3);
    const long long fs = btri_size(m, mh);
    const int tid = threadIdx.x;
    using V = float4;  // 16 bytes
    constexpr int PER = 16 / sizeof(T);
    const V* src = reinterpret_cast<const V*>(L + R.off);
    V* dst = reinterpret_cast<V*>(F);
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
    const bool fixed = (m == M1 || m == M2);
    for (int r = tid; r < n; r += 256) {
        const int aa = r % m, bb = r / m;
        const T gv = g[(long long)(R.j0 + 1 + bb) * nx + R.i0 + 1 + aa];
        vec[r] = fixed ? gv * L[R.off + fs - n + r] : gv;  // the fixed-width solve expects S g
    }
    __syncthreads();
    if (fixed) {
        if (tid < 64) {  // one wavefront solves; the others wait at the barrier below
            if (m == M1)
                btri_solve_rl<T, M1>(F, mh, vec);
            else
                btri_solve_rl<T, M2>(F, mh, vec);
        }
    } else {
        btri_solve_lds<T>(F, m, mh, vec, tb, xb);
    }
    __syncthreads();
    for (int r = tid; r < n; r += 256) wout[R.voff + r] = vec[r];
}

// Smoother, phase 2: z(v) = [z(v)] + eta * sum of the patch solutions covering v
// (fixed patch order, so the sum is deterministic; no atomics).
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

}  // namespace

namespace tgms {

static void factor_rects(tgms_ctx* c, Rect* rects, int count, int max_n, int max_b, double* L, double* S,
                         float* L32) {
    size_t lds = (size_t)max_n * (max_b + 1) * sizeof(double);
    if (lds > 65536) throw TgmsError{TGMS_E_UNSUPPORTED, "local band factor exceeds 64 KiB of LDS"};
    int* fail = c->alloc<int>(1);
    if (max_b - 1 > TGMS_MMAX) throw TgmsError{TGMS_E_UNSUPPORTED, "local rectangle wider than 33 cells"};
    if (L32)
        hipLaunchKernelGGL((k_band_factor<true>), dim3(count), dim3(TGMS_WAVE), lds, c->stream, rects, c->a, c->nx,
                           c->sx * c->sx, c->sy * c->sy, L, S, L32, fail);
    else
        hipLaunchKernelGGL((k_band_factor<false>), dim3(count), dim3(TGMS_WAVE), lds, c->stream, rects, c->a,
                           c->nx, c->sx * c->sx, c->sy * c->sy, L, S, L32, fail);
    LAUNCH_OK();
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (h) throw TgmsError{TGMS_E_INVAL, "local stream-function matrix is not positive definite"};
}

void factor_blocks(tgms_ctx* c) {
    std::vector<Rect> r(c->nblk);
    for (int J = 0; J < c->Ny; ++J)
        for (int I = 0; I < c->Nx; ++I) {
            Rect& q = r[J * c->Nx + I];
            q.i0 = I * c->bx;
            q.i1 = (I + 1) * c->bx;
            q.j0 = J * c->by;
            q.j1 = (J + 1) * c->by;
            q.off = (long long)(J * c->Nx + I) * btri_size(c->bx - 1, c->by - 1);
            q.voff = (long long)(J * c->Nx + I) * c->blk_n;
        }
    Rect* d = c->alloc<Rect>(c->nblk);
    HIP_OK(hipMemcpyAsync(d, r.data(), sizeof(Rect) * c->nblk, hipMemcpyHostToDevice, c->stream));
    factor_rects(c, d, c->nblk, c->blk_n, c->blk_b, c->blkL, c->blkS, nullptr);
}

void enable_large_lds(tgms_ctx* c) {
    // allow the staged smoother kernels to use the device's full per-workgroup LDS
    (void)hipFuncSetAttribute((const void*)k_smooth_patches_lds<double, 19, 17>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_patches_lds<double, 11, 9>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_patches_lds<double, 1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_patches_lds<float, 19, 17>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_patches_lds<float, 11, 9>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    (void)hipFuncSetAttribute((const void*)k_smooth_patches_lds<float, 1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max);
    (void)hipGetLastError();
}

void factor_patches(tgms_ctx* c) {
    enable_large_lds(c);
    factor_rects(c, c->patch, c->nblk, c->pat_nmax, c->pat_bmax, c->patL, c->patS, c->precision ? c->patL32 : nullptr);
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
    size_t lds = (size_t)(c->pat_nmax + 128) * sizeof(T);
    const size_t lds_staged = (size_t)(((c->pat_nmax + 3) & ~3) + 128 + c->pat_fmax + 4) * sizeof(T);
    const bool staged = lds_staged <= (size_t)c->lds_max;
    {
        ProfScope ps(c, PK_SMOOTH);
        const int mw = btri_width(c->pat_bmax - 1);
        if (staged) {
            const int mi = c->pat_bmax - 1;  // interior patch row width
            if (mi == 19)
                hipLaunchKernelGGL((k_smooth_patches_lds<T, 19, 17>), dim3(c->nblk), dim3(256), lds_staged, c->stream,
                                   c->patch, L, g, c->nx, w);
            else if (mi == 11)
                hipLaunchKernelGGL((k_smooth_patches_lds<T, 11, 9>), dim3(c->nblk), dim3(256), lds_staged, c->stream,
                                   c->patch, L, g, c->nx, w);
            else
                hipLaunchKernelGGL((k_smooth_patches_lds<T, 1, 1>), dim3(c->nblk), dim3(256), lds_staged, c->stream,
                                   c->patch, L, g, c->nx, w);
        } else if (mw == 16)
            hipLaunchKernelGGL((k_smooth_patches<T, 16>), dim3(c->nblk), dim3(TGMS_WAVE), lds, c->stream, c->patch, L, g,
                               c->nx, w);
        else if (mw == 24)
            hipLaunchKernelGGL((k_smooth_patches<T, 24>), dim3(c->nblk), dim3(TGMS_WAVE), lds, c->stream, c->patch, L, g,
                               c->nx, w);
        else
            hipLaunchKernelGGL((k_smooth_patches<T, 32>), dim3(c->nblk), dim3(TGMS_WAVE), lds, c->stream, c->patch, L, g,
                               c->nx, w);
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
