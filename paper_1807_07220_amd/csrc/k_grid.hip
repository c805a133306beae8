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
                               double* __restrict__ a, long long n, double area, int* __restrict__ bad) {
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
}

// cell weights from a given kappa^{-1} (a restored context): the same product as above
__global__ void k_weights_from_kinv(const double* __restrict__ kinv, double* __restrict__ a, long long n,
                                    double area) {
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= n) return;
    a[c] = area * kinv[c];
}

// cell weights under a mobility field: a = |c| kappa^{-1} / lambda (kinv kept from setup)
__global__ void k_mobility_weights(const double* __restrict__ lambda, const double* __restrict__ kinv,
                                   double* __restrict__ a, long long n, double area, int* __restrict__ bad) {
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= n) return;
    double l = lambda[c];
    if (!(l > 0.0) || !(l < INFINITY)) {
        atomicOr(bad, 1);
        l = 1.0;
    }
    const double w = area * kinv[c] / l;
    a[c] = w;
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

__global__ void k_axpy(long long n, double a, const double* __restrict__ x, double* __restrict__ y) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
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

__global__ void k_copy(long long n, const double* __restrict__ x, double* __restrict__ y) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t];
}

inline unsigned nb(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

namespace tgms {

void cell_weights(tgms_ctx* c, const double* kappa, int* bad) {
    long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_cell_weights, dim3(nb(n)), dim3(256), 0, c->stream, kappa, c->kinv, c->a, n,
                       c->hx * c->hy, bad);
    LAUNCH_OK();
}

void mobility_weights(tgms_ctx* c, const double* lambda, int* bad, double* out) {
    long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_mobility_weights, dim3(nb(n)), dim3(256), 0, c->stream, lambda, (const double*)c->kinv, out,
                       n, c->hx * c->hy, bad);
    LAUNCH_OK();
}

void weights_from_kinv(tgms_ctx* c) {
    long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_weights_from_kinv, dim3(nb(n)), dim3(256), 0, c->stream, (const double*)c->kinv, c->a, n,
                       c->hx * c->hy);
    LAUNCH_OK();
}

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

void copy(tgms_ctx* c, long long n, const double* x, double* y) {
    hipLaunchKernelGGL(k_copy, dim3(nb(n)), dim3(256), 0, c->stream, n, x, y);
    LAUNCH_OK();
}

void axpy(tgms_ctx* c, long long n, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_axpy, dim3(nb(n)), dim3(256), 0, c->stream, n, a, x, y);
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
