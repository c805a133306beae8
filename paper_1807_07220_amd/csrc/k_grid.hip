// Vertex/face operators and Krylov vector kernels.
//
// The H(div) operator of the reduced problem (paper section 3, eq.
// reduced_fine_system) acts on divergence-free RT0 fields with zero flux on
// dD.  On the unit square these are exactly the discrete curls C psi of
// vertex stream functions, so the operator is applied as K psi = C^T A C psi:
// a matrix-free 9-point stencil that reads psi (3x3) and the four cell weights
// around each vertex.  Face-space A (eq. fine_system) is used by the
// preprocessing and for the initial residual.
#include "common.h"

namespace {

constexpr int TX = 64, TY = 4;

__global__ void k_cell_weights(const double* __restrict__ kappa, double* __restrict__ kinv,
                               double* __restrict__ a, float* __restrict__ a32, long long n, double area,
                               int* __restrict__ bad) {
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= n) return;
    double k = kappa[c];
    if (!(k > 0.0) || !(k < INFINITY)) {
        atomicOr(bad, 1);
        k = 1.0;
    }
    double ki = 1.0 / k;
    kinv[c] = ki;
    a[c] = area * ki;
    a32[c] = (float)(area * ki);
}

// out = K psi  (mode 0) or out = g - K psi (mode 1), interior vertices; boundary entries 0.
template <typename T, int MODE>
__global__ void k_apply_K(const T* __restrict__ psi, const T* __restrict__ g, T* __restrict__ out,
                          const T* __restrict__ a, int nx, int ny, T sx2, T sy2) {
    int i = blockIdx.x * TX + threadIdx.x;
    int j = blockIdx.y * TY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    long long v = (long long)j * nx + i;
    if (i == 0 || j == 0) {
        out[v] = T(0);
        return;
    }
    const T A00 = a[v - nx - 1], A10 = a[v - nx], A01 = a[v - 1], A11 = a[v];
    const T s = sx2 + sy2;
    const bool hasE = i + 1 < nx, hasN = j + 1 < ny;
    const T pc = psi[v];
    const T pw = psi[v - 1], ps = psi[v - nx], psw = psi[v - nx - 1];
    const T pe = hasE ? psi[v + 1] : T(0);
    const T pse = hasE ? psi[v - nx + 1] : T(0);
    const T pn = hasN ? psi[v + nx] : T(0);
    const T pnw = hasN ? psi[v + nx - 1] : T(0);
    const T pne = (hasE && hasN) ? psi[v + nx + 1] : T(0);
    const T c6 = T(1.0 / 6.0), c3 = T(1.0 / 3.0);
    const T kx = sx2 * c6 - sy2 * c3;  // E/W weight per adjacent cell
    const T ky = sy2 * c6 - sx2 * c3;  // N/S weight per adjacent cell
    T r = s * c3 * (A00 + A10 + A01 + A11) * pc;
    r += kx * ((A10 + A11) * pe + (A00 + A01) * pw);
    r += ky * ((A01 + A11) * pn + (A00 + A10) * ps);
    r -= s * c6 * (A11 * pne + A01 * pnw + A10 * pse + A00 * psw);
    out[v] = MODE == 0 ? r : g[v] - r;
}

// A u on interior faces (full numbering); boundary outputs 0.  use_bnd = 0
// ignores the boundary entries of u (probe semantics), 1 includes them.
__global__ void k_faces_A(const double* __restrict__ u, double* __restrict__ out, const double* __restrict__ a,
                          int nx, int ny, int use_bnd) {
    long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nfx = (long long)(nx + 1) * ny, nf = nfx + (long long)nx * (ny + 1);
    if (f >= nf) return;
    const double c3 = 1.0 / 3.0, c6 = 1.0 / 6.0;
    if (f < nfx) {
        int j = (int)(f / (nx + 1)), i = (int)(f % (nx + 1));
        if (i == 0 || i == nx) {
            out[f] = 0.0;
            return;
        }
        double ul = u[f - 1], ur = u[f + 1];
        if (!use_bnd) {
            if (i - 1 == 0) ul = 0.0;
            if (i + 1 == nx) ur = 0.0;
        }
        const double aL = a[(long long)j * nx + i - 1], aR = a[(long long)j * nx + i];
        out[f] = aL * (u[f] * c3 + ul * c6) + aR * (u[f] * c3 + ur * c6);
    } else {
        long long g = f - nfx;
        int j = (int)(g / nx), i = (int)(g % nx);
        if (j == 0 || j == ny) {
            out[f] = 0.0;
            return;
        }
        double ub = u[f - nx], ut = u[f + nx];
        if (!use_bnd) {
            if (j - 1 == 0) ub = 0.0;
            if (j + 1 == ny) ut = 0.0;
        }
        const double aB = a[(long long)(j - 1) * nx + i], aT = a[(long long)j * nx + i];
        out[f] = aB * (u[f] * c3 + ub * c6) + aT * (u[f] * c3 + ut * c6);
    }
}

// g = scale * C^T w for a full face array w (only interior faces enter).
__global__ void k_curlT(const double* __restrict__ w, double* __restrict__ g, int nx, int ny, double sx,
                        double sy, double scale) {
    int i = blockIdx.x * TX + threadIdx.x;
    int j = blockIdx.y * TY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    long long v = (long long)j * nx + i;
    if (i == 0 || j == 0) {
        g[v] = 0.0;
        return;
    }
    const long long nfx = (long long)(nx + 1) * ny;
    const double wx_s = w[(long long)(j - 1) * (nx + 1) + i], wx_n = w[(long long)j * (nx + 1) + i];
    const double wy_w = w[nfx + (long long)j * nx + i - 1], wy_e = w[nfx + (long long)j * nx + i];
    g[v] = scale * (sx * (wx_s - wx_n) + sy * (wy_e - wy_w));
}

// u = base + C psi on all faces (boundary faces: u = base).
__global__ void k_curl_add(const double* __restrict__ psi, const double* __restrict__ base,
                           double* __restrict__ u, int nx, int ny, double sx, double sy) {
    long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nfx = (long long)(nx + 1) * ny, nf = nfx + (long long)nx * (ny + 1);
    if (f >= nf) return;
    double c = 0.0;
    if (f < nfx) {
        int j = (int)(f / (nx + 1)), i = (int)(f % (nx + 1));
        if (i > 0 && i < nx) {
            double top = (j + 1 < ny) ? psi[(long long)(j + 1) * nx + i] : 0.0;
            double bot = psi[(long long)j * nx + i];
            c = (top - bot) * sx;
        }
    } else {
        long long g = f - nfx;
        int j = (int)(g / nx), i = (int)(g % nx);
        if (j > 0 && j < ny) {
            double rgt = (i + 1 < nx) ? psi[(long long)j * nx + i + 1] : 0.0;
            double lft = psi[(long long)j * nx + i];
            c = -(rgt - lft) * sy;
        }
    }
    u[f] = (base ? base[f] : 0.0) + c;
}

// ---- deterministic reductions: fixed grid, one partial per block, then one block sums them.
constexpr int RED_BLOCKS = 512, RED_THREADS = 256;

template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double* __restrict__ part) {
    __shared__ double sh[NV][RED_THREADS / TGMS_WAVE];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < RED_THREADS / TGMS_WAVE; ++w) s += sh[k][w];
            part[k * RED_BLOCKS + blockIdx.x] = s;
        }
    }
}

template <int NV>
__global__ void k_multidot(const double* __restrict__ x0, const double* __restrict__ y0,
                           const double* __restrict__ x1, const double* __restrict__ y1,
                           const double* __restrict__ x2, const double* __restrict__ y2, long long n,
                           double* __restrict__ part) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (long long t = blockIdx.x * (long long)RED_THREADS + threadIdx.x; t < n;
         t += (long long)RED_BLOCKS * RED_THREADS) {
        v[0] += x0[t] * y0[t];
        if (NV > 1) v[1] += x1[t] * y1[t];
        if (NV > 2) v[2] += x2[t] * y2[t];
    }
    block_reduce_store<NV>(v, part);
}

// sum over faces of (C psi)^2, psi a vertex array
__global__ void k_curl_norm2(const double* __restrict__ psi, int nx, int ny, double sx, double sy,
                             double* __restrict__ part) {
    double v[1] = {0.0};
    const long long n = (long long)nx * ny;
    for (long long t = blockIdx.x * (long long)RED_THREADS + threadIdx.x; t < n;
         t += (long long)RED_BLOCKS * RED_THREADS) {
        int j = (int)(t / nx), i = (int)(t % nx);
        // x-face (i, j) for 1 <= i <= nx-1 and y-face (i, j) for 1 <= j <= ny-1 keyed by vertex (i, j)
        double pc = psi[t];
        if (i > 0) {
            double top = (j + 1 < ny) ? psi[t + nx] : 0.0;
            double d = (top - pc) * sx;
            v[0] += d * d;
        }
        if (j > 0) {
            double rgt = (i + 1 < nx) ? psi[t + 1] : 0.0;
            double d = (rgt - pc) * sy;
            v[0] += d * d;
        }
    }
    block_reduce_store<1>(v, part);
}

__global__ void k_reduce_final(const double* __restrict__ part, int nv, double* __restrict__ out) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __shared__ double sh[RED_THREADS / TGMS_WAVE];
    for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < RED_BLOCKS; b += RED_THREADS) s += part[k * RED_BLOCKS + b];
        s = wave_sum(s);
        if (lane == 0) sh[wid] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < RED_THREADS / TGMS_WAVE; ++w) t += sh[w];
            out[k] = t;
        }
        __syncthreads();
    }
}

__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}
__global__ void k_xpay(long long n, const double* __restrict__ x, double b, double* __restrict__ y) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t] + b * y[t];
}
__global__ void k_d2f(long long n, const double* __restrict__ x, float* __restrict__ y) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = (float)x[t];
}
__global__ void k_f2d(long long n, const float* __restrict__ x, double* __restrict__ y) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = (double)x[t];
}
__global__ void k_fill0(long long n, double* __restrict__ y) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = 0.0;
}

// ---- PCG with its scalars on the device (no host round trip inside an iteration) ----
// sc: [0] rho, [1] p^T q, [2] alpha, [3] beta, [4] |z|^2, [5] |z|^2/|z0|^2, [6] |z0|^2,
//     [7] breakdown flag, [8] iteration counter; hist holds alpha_k, beta_k pairs.
enum { SC_RHO = 0, SC_PQ, SC_ALPHA, SC_BETA, SC_ZN2, SC_REL2, SC_Z02, SC_FLAG, SC_IT };

__device__ inline double block_total(const double* __restrict__ part, int k) {
    __shared__ double sh[RED_THREADS / TGMS_WAVE];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double s = 0.0;
    for (int b = threadIdx.x; b < RED_BLOCKS; b += RED_THREADS) s += part[k * RED_BLOCKS + b];
    s = wave_sum(s);
    if (lane == 0) sh[wid] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < RED_THREADS / TGMS_WAVE; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// after the p^T q partials: alpha = rho / p^T q
__global__ void k_pcg_alpha(const double* __restrict__ part, double* __restrict__ sc, double* __restrict__ hist) {
    const double pq = block_total(part, 0);
    if (threadIdx.x == 0) {
        const int it = (int)sc[SC_IT];
        sc[SC_PQ] = pq;
        if (!(pq > 0.0) || !(pq < INFINITY)) sc[SC_FLAG] = 1.0;
        const double a = sc[SC_RHO] / pq;
        sc[SC_ALPHA] = a;
        hist[2 * it] = a;
    }
}

// after the (g.z, z.gold, |Cz|^2) partials: rho, beta, relative residual; counts the iteration
__global__ void k_pcg_beta(const double* __restrict__ part, double* __restrict__ sc, double* __restrict__ hist,
                           int flexible, int first) {
    const double gz = block_total(part, 0);
    const double zgold = block_total(part, 1);
    const double zn2 = block_total(part, 2);
    if (threadIdx.x == 0) {
        if (first) {
            sc[SC_RHO] = gz;
            sc[SC_Z02] = zn2;
            sc[SC_ZN2] = zn2;
            sc[SC_REL2] = 1.0;
            sc[SC_IT] = 0.0;
            sc[SC_FLAG] = 0.0;
            return;
        }
        const int it = (int)sc[SC_IT];
        const double rho = sc[SC_RHO];
        const double beta = flexible ? (gz - zgold) / rho : gz / rho;
        sc[SC_BETA] = beta;
        sc[SC_RHO] = gz;
        sc[SC_ZN2] = zn2;
        sc[SC_REL2] = zn2 / sc[SC_Z02];
        hist[2 * it + 1] = beta;
        sc[SC_IT] = it + 1;
    }
}

// x += alpha p ; gold = g (flexible) ; g -= alpha q
__global__ void k_pcg_update(long long n, const double* __restrict__ sc, const double* __restrict__ p,
                             const double* __restrict__ q, double* __restrict__ x, double* __restrict__ g,
                             double* __restrict__ gold) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double a = sc[SC_ALPHA];
    x[t] += a * p[t];
    const double gv = g[t];
    if (gold) gold[t] = gv;
    g[t] = gv - a * q[t];
}

// p = z + beta p
__global__ void k_pcg_dir(long long n, const double* __restrict__ sc, const double* __restrict__ z,
                          double* __restrict__ p) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    p[t] = z[t] + sc[SC_BETA] * p[t];
}

__global__ void k_copy(long long n, const double* __restrict__ x, double* __restrict__ y) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t];
}

inline unsigned nb(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

double finish_reduce(tgms_ctx* c, int nv, double* out) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, c->stream, c->red, nv,
                       c->red + 3 * RED_BLOCKS);
    LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(c->red_h, c->red + 3 * RED_BLOCKS, nv * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < nv; ++k) out[k] = c->red_h[k];
    return out[0];
}

}  // namespace

namespace tgms {

void cell_weights(tgms_ctx* c, const double* kappa, int* bad) {
    long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_cell_weights, dim3(nb(n)), dim3(256), 0, c->stream, kappa, c->kinv, c->a, c->a32, n,
                       c->hx * c->hy, bad);
    LAUNCH_OK();
}

template <typename T>
void apply_K(tgms_ctx* c, const T* psi, T* out, const T* a) {
    dim3 grid((c->nx + TX - 1) / TX, (c->ny + TY - 1) / TY);
    ProfScope ps(c, PK_APPLYK);
    hipLaunchKernelGGL((k_apply_K<T, 0>), grid, dim3(TX, TY), 0, c->stream, psi, (const T*)nullptr, out, a, c->nx,
                       c->ny, T(c->sx * c->sx), T(c->sy * c->sy));
    LAUNCH_OK();
}
template <typename T>
void residual_K(tgms_ctx* c, const T* g, const T* psi, T* out, const T* a) {
    dim3 grid((c->nx + TX - 1) / TX, (c->ny + TY - 1) / TY);
    ProfScope ps(c, PK_APPLYK);
    hipLaunchKernelGGL((k_apply_K<T, 1>), grid, dim3(TX, TY), 0, c->stream, psi, g, out, a, c->nx, c->ny,
                       T(c->sx * c->sx), T(c->sy * c->sy));
    LAUNCH_OK();
}
template void apply_K<double>(tgms_ctx*, const double*, double*, const double*);
template void apply_K<float>(tgms_ctx*, const float*, float*, const float*);
template void residual_K<double>(tgms_ctx*, const double*, const double*, double*, const double*);
template void residual_K<float>(tgms_ctx*, const float*, const float*, float*, const float*);

void faces_A(tgms_ctx* c, const double* u, double* out) {
    hipLaunchKernelGGL(k_faces_A, dim3(nb(c->nf)), dim3(256), 0, c->stream, u, out, c->a, c->nx, c->ny, 1);
    LAUNCH_OK();
}

void faces_A_probe(tgms_ctx* c, const double* u, double* out) {
    hipLaunchKernelGGL(k_faces_A, dim3(nb(c->nf)), dim3(256), 0, c->stream, u, out, c->a, c->nx, c->ny, 0);
    LAUNCH_OK();
}

void curlT_A_faces(tgms_ctx* c, const double* u, double* g, double scale) {
    faces_A(c, u, c->fu);
    dim3 grid((c->nx + TX - 1) / TX, (c->ny + TY - 1) / TY);
    hipLaunchKernelGGL(k_curlT, grid, dim3(TX, TY), 0, c->stream, c->fu, g, c->nx, c->ny, c->sx, c->sy, scale);
    LAUNCH_OK();
}

void curlT(tgms_ctx* c, const double* u, double* g) {
    dim3 grid((c->nx + TX - 1) / TX, (c->ny + TY - 1) / TY);
    hipLaunchKernelGGL(k_curlT, grid, dim3(TX, TY), 0, c->stream, u, g, c->nx, c->ny, c->sx, c->sy, 1.0);
    LAUNCH_OK();
}

void curl_add(tgms_ctx* c, const double* psi, const double* base, double* u) {
    hipLaunchKernelGGL(k_curl_add, dim3(nb(c->nf)), dim3(256), 0, c->stream, psi, base, u, c->nx, c->ny, c->sx,
                       c->sy);
    LAUNCH_OK();
}

double dot(tgms_ctx* c, const double* x, const double* y, long long n) {
    hipLaunchKernelGGL((k_multidot<1>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, x, y, nullptr, nullptr,
                       nullptr, nullptr, n, c->red);
    LAUNCH_OK();
    double out[1];
    return finish_reduce(c, 1, out);
}

void dot3(tgms_ctx* c, const double* g, const double* z, const double* gold, double out[3]) {
    long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL((k_multidot<2>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, g, z, gold ? gold : g,
                       z, nullptr, nullptr, n, c->red);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_curl_norm2, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, z, c->nx, c->ny, c->sx,
                       c->sy, c->red + 2 * RED_BLOCKS);
    LAUNCH_OK();
    finish_reduce(c, 3, out);
}

double curl_norm2(tgms_ctx* c, const double* psi) {
    hipLaunchKernelGGL(k_curl_norm2, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, psi, c->nx, c->ny, c->sx,
                       c->sy, c->red);
    LAUNCH_OK();
    double out[1];
    return finish_reduce(c, 1, out);
}

// partial sums of p.q into red, then alpha on the device
void pcg_alpha(tgms_ctx* c, const double* p, const double* q, double* sc, double* hist) {
    const long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL((k_multidot<1>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, p, q, nullptr, nullptr,
                       nullptr, nullptr, n, c->red);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(RED_THREADS), 0, c->stream, (const double*)c->red, sc, hist);
    LAUNCH_OK();
}

void pcg_beta(tgms_ctx* c, const double* g, const double* z, const double* gold, double* sc, double* hist,
              bool flexible, bool first) {
    const long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL((k_multidot<2>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, g, z, gold ? gold : g, z,
                       nullptr, nullptr, n, c->red);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_curl_norm2, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, c->stream, z, c->nx, c->ny, c->sx, c->sy,
                       c->red + 2 * RED_BLOCKS);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(RED_THREADS), 0, c->stream, (const double*)c->red, sc, hist,
                       flexible ? 1 : 0, first ? 1 : 0);
    LAUNCH_OK();
}

void pcg_update(tgms_ctx* c, const double* sc, const double* p, const double* q, double* x, double* g, double* gold) {
    const long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_pcg_update, dim3(nb(n)), dim3(256), 0, c->stream, n, sc, p, q, x, g, gold);
    LAUNCH_OK();
}

void pcg_dir(tgms_ctx* c, const double* sc, const double* z, double* p) {
    const long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_pcg_dir, dim3(nb(n)), dim3(256), 0, c->stream, n, sc, z, p);
    LAUNCH_OK();
}

void copy(tgms_ctx* c, long long n, const double* x, double* y) {
    hipLaunchKernelGGL(k_copy, dim3(nb(n)), dim3(256), 0, c->stream, n, x, y);
    LAUNCH_OK();
}

void axpy(tgms_ctx* c, long long n, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_axpy, dim3(nb(n)), dim3(256), 0, c->stream, n, a, x, y);
    LAUNCH_OK();
}
void xpay(tgms_ctx* c, long long n, const double* x, double b, double* y) {
    hipLaunchKernelGGL(k_xpay, dim3(nb(n)), dim3(256), 0, c->stream, n, x, b, y);
    LAUNCH_OK();
}
void cast_d2f(tgms_ctx* c, long long n, const double* x, float* y) {
    hipLaunchKernelGGL(k_d2f, dim3(nb(n)), dim3(256), 0, c->stream, n, x, y);
    LAUNCH_OK();
}
void cast_f2d(tgms_ctx* c, long long n, const float* x, double* y) {
    hipLaunchKernelGGL(k_f2d, dim3(nb(n)), dim3(256), 0, c->stream, n, x, y);
    LAUNCH_OK();
}
void zero(tgms_ctx* c, void* p, size_t bytes) {
    long long n = (long long)(bytes / sizeof(double));
    hipLaunchKernelGGL(k_fill0, dim3(nb(n)), dim3(256), 0, c->stream, n, (double*)p);
    LAUNCH_OK();
}

}  // namespace tgms
