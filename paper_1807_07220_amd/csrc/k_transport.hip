// Two-phase transport of section 6.2 (eqs. satEq, fraction, mobility, DisSatEq_Implicit,
// integralFlux): the backward-Euler upwind finite-volume step for the water saturation and
// the total mobility that the next pressure solve uses.
//
// Per cell i with sides k (four on the square, six on the cube) and out_k the total flux
// out of i through side k,
// c = dt / (phi |Omega_i|), the step's equation reads
//   R_i(s) = s_i + a_i f_w(s_i) - b_i(s) = 0,
//   a_i = c (sum_{out_k >= 0} out_k - q_i^-),
//   b_i = s_i^n + c q_i^+ + c sum_{out_k < 0} |out_k| f_w(s_nb(k)),
// the upwind cell of a side being the one the flux leaves.  Cell i's equation depends on
// its own saturation and on those upstream of it only; for a potential flow the upwind
// graph has no cycles, so the system is triangular in flow order and its unique solution
// is reached by nonlinear Gauss-Seidel in that order.  The GPU does this by tiles: a
// workgroup owns 16 x 16 cells (8 x 8 x 4 on the cube), takes the saturations outside the tile from the previous
// outer step, and sweeps its cells in LDS (each sweep solves every cell's scalar equation
// by bracketed Newton, monotone g(s) = s + a f_w(s) - b on [0, 1] with g(0) <= 0 <= g(1))
// until no value changes; the outer steps repeat until max_i |R_i| <= newton_tol.  Outer
// steps grow with the tiles along the longest upwind path, not with the cells.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

constexpr int TT = 256;

__device__ inline void frac_flow(double s, double rmw, double rmo, double& f, double& df) {
    const double a = s * s * rmw, b = (1.0 - s) * (1.0 - s) * rmo;
    const double lam = a + b;
    const double da = 2.0 * s * rmw, db = -2.0 * (1.0 - s) * rmo;
    f = a / lam;
    df = (da * lam - a * (da + db)) / (lam * lam);
}

// the grid of the square (nz = 1, hz = 1: face lengths and cell areas) or of the cube
struct TGeom {
    int nx, ny, nz;
    double hx, hy, hz;
    long long nfx, nfy;
};

// total flux out of cell (i, j, k) through side sd (x-, x+, y-, y+, z-, z+) and the
// neighbour there (-1 on dD, flux 0)
__device__ inline double side_out(const double* __restrict__ u, const TGeom& G, int i, int j, int k, int sd,
                                  long long c, long long& nb) {
    const long long row = (long long)k * G.ny + j;
    const long long plane = (long long)G.nx * G.ny;
    switch (sd) {
        case 0:
            nb = i > 0 ? c - 1 : -1;
            return nb >= 0 ? -u[row * (G.nx + 1) + i] * G.hy * G.hz : 0.0;
        case 1:
            nb = i < G.nx - 1 ? c + 1 : -1;
            return nb >= 0 ? u[row * (G.nx + 1) + i + 1] * G.hy * G.hz : 0.0;
        case 2:
            nb = j > 0 ? c - G.nx : -1;
            return nb >= 0 ? -u[G.nfx + ((long long)k * (G.ny + 1) + j) * G.nx + i] * G.hx * G.hz : 0.0;
        case 3:
            nb = j < G.ny - 1 ? c + G.nx : -1;
            return nb >= 0 ? u[G.nfx + ((long long)k * (G.ny + 1) + j + 1) * G.nx + i] * G.hx * G.hz : 0.0;
        case 4:
            nb = k > 0 ? c - plane : -1;
            return nb >= 0 ? -u[G.nfx + G.nfy + row * G.nx + i] * G.hx * G.hy : 0.0;
        default:
            nb = k < G.nz - 1 ? c + plane : -1;
            return nb >= 0 ? u[G.nfx + G.nfy + (row + G.ny) * G.nx + i] * G.hx * G.hy : 0.0;
    }
}

__device__ inline double block_max(double v) {
    __shared__ double sh[TT / 64];
    v = fabs(v);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = 0.0;
#pragma unroll
    for (int w = 0; w < TT / 64; ++w) m = fmax(m, sh[w]);
    return m;
}

// R_i (the step's residual) and the workgroup's largest |R_i| to part
__global__ void __launch_bounds__(TT) k_tr_residual(const double* __restrict__ u, const double* __restrict__ q,
                                                    const double* __restrict__ s, const double* __restrict__ s_old,
                                                    TGeom G, double coef, double rmw, double rmo,
                                                    double* __restrict__ part) {
    const long long c = blockIdx.x * (long long)TT + threadIdx.x;
    const long long n = (long long)G.nx * G.ny * G.nz;
    double r = 0.0;
    if (c < n) {
        const int i = (int)(c % G.nx), j = (int)((c / G.nx) % G.ny), k = (int)(c / ((long long)G.nx * G.ny));
        double fi, dfi;
        frac_flow(s[c], rmw, rmo, fi, dfi);
        double flux = 0.0;
        for (int sd = 0; sd < 6; ++sd) {
            long long nb;
            const double o = side_out(u, G, i, j, k, sd, c, nb);
            if (o >= 0.0) {
                flux += fi * o;
            } else {
                double fn, dfn;
                frac_flow(s[nb], rmw, rmo, fn, dfn);
                flux += fn * o;
            }
        }
        r = s[c] - s_old[c] - coef * (fmax(q[c], 0.0) - flux + fi * fmin(q[c], 0.0));
    }
    const double m = block_max(r);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// root of s + a f_w(s) = b in [0, 1] (a >= 0, 0 <= b <= 1 + a) by Newton inside a
// bracket, from the guess x
__device__ inline double cell_solve(double a, double b, double x, double rmw, double rmo) {
    double lo = 0.0, hi = 1.0;
    x = fmin(fmax(x, 0.0), 1.0);
    for (int it = 0; it < 60; ++it) {
        double f, df;
        frac_flow(x, rmw, rmo, f, df);
        const double g = x + a * f - b;
        if (g == 0.0) break;
        if (g > 0.0)
            hi = x;
        else
            lo = x;
        double xn = x - g / (1.0 + a * df);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 4e-16 || hi - lo <= 4e-16) {
            x = xn;
            break;
        }
        x = xn;
    }
    return x;
}

// One outer step of tile-wise nonlinear Gauss-Seidel: saturations outside the tile from
// s_in, the tile's own swept in LDS until none changes (at most MAX_LOCAL sweeps).
// Tiles of 16 x 16 cells on the square, 8 x 8 x 4 on the cube (256 threads either way).
constexpr int MAX_LOCAL = 64;

template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX* TY* TZ) k_tr_tile_solve(const double* __restrict__ u,
                                                              const double* __restrict__ q,
                                                              const double* __restrict__ s_old,
                                                              const double* __restrict__ s_in, TGeom G, double coef,
                                                              double rmw, double rmo, double* __restrict__ s_out) {
    constexpr int NTL = TX * TY * TZ;
    __shared__ double buf[2][NTL];
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int i = blockIdx.x * TX + tx, j = blockIdx.y * TY + ty, k = blockIdx.z * TZ + tz;
    const bool act = i < G.nx && j < G.ny && k < G.nz;
    const long long c = ((long long)k * G.ny + j) * G.nx + i;
    // a, the part of b fixed during the sweeps, and per inflow side inside the tile its
    // weight c |out| and LDS slot
    double a = 0.0, b0 = 0.0, w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, x = 0.0;
    int loc[6] = {-1, -1, -1, -1, -1, -1};
    if (act) {
        double outsum = 0.0;
        b0 = s_old[c] + coef * fmax(q[c], 0.0);
        for (int sd = 0; sd < 6; ++sd) {
            long long nb;
            const double o = side_out(u, G, i, j, k, sd, c, nb);
            if (o >= 0.0) {
                outsum += o;
            } else {
                const int ni = (int)(nb % G.nx) - (int)blockIdx.x * TX;
                const int nj = (int)((nb / G.nx) % G.ny) - (int)blockIdx.y * TY;
                const int nk = (int)(nb / ((long long)G.nx * G.ny)) - (int)blockIdx.z * TZ;
                if (ni >= 0 && ni < TX && nj >= 0 && nj < TY && nk >= 0 && nk < TZ) {
                    w[sd] = -coef * o;
                    loc[sd] = (nk * TY + nj) * TX + ni;
                } else {
                    double fn, dfn;
                    frac_flow(s_in[nb], rmw, rmo, fn, dfn);
                    b0 -= coef * o * fn;
                }
            }
        }
        a = coef * (outsum - fmin(q[c], 0.0));
        x = s_in[c];
    }
    double* cur = buf[0];
    double* nxt = buf[1];
    cur[threadIdx.x] = x;
    __syncthreads();
    for (int sw = 0; sw < MAX_LOCAL; ++sw) {
        int changed = 0;
        if (act) {
            double b = b0;
            for (int sd = 0; sd < 6; ++sd)
                if (loc[sd] >= 0) {
                    double fn, dfn;
                    frac_flow(cur[loc[sd]], rmw, rmo, fn, dfn);
                    b += w[sd] * fn;
                }
            const double xn = cell_solve(a, b, x, rmw, rmo);
            changed = xn != x;
            x = xn;
        }
        nxt[threadIdx.x] = x;
        double* t = cur;
        cur = nxt;
        nxt = t;
        if (!__syncthreads_or(changed)) break;
    }
    if (act) s_out[c] = x;
}

__global__ void k_total_mobility(const double* __restrict__ s, long long n, double rmw, double rmo,
                                 double* __restrict__ lam) {
    const long long c = blockIdx.x * (long long)TT + threadIdx.x;
    if (c >= n) return;
    const double v = s[c];
    lam[c] = v * v * rmw + (1.0 - v) * (1.0 - v) * rmo;
}

}  // namespace

namespace tgms {

void total_mobility(hipStream_t st, const double* s, long long n, double mu_w, double mu_o, double* lam) {
    hipLaunchKernelGGL(k_total_mobility, dim3((unsigned)((n + TT - 1) / TT)), dim3(TT), 0, st, s, n, 1.0 / mu_w,
                       1.0 / mu_o, lam);
    LAUNCH_OK();
}

// One transport step; the workspace (2 n + partials doubles) comes from the device cache.
// The result is in s; TransportResult.sweeps counts the outer (tile) launches.
TransportResult transport_step(hipStream_t st, int nx, int ny, int nz, const double* u, const double* q, double* s,
                               double phi, double dt, double mu_w, double mu_o, double newton_tol, int max_outer) {
    const bool cube = nz > 1;
    if (!cube) nz = 1;
    const long long n = (long long)nx * ny * nz;
    const unsigned nbk = (unsigned)((n + TT - 1) / TT);
    size_t got = 0;
    const size_t bytes = sizeof(double) * (2 * (size_t)n + nbk);
    double* w = (double*)dev_alloc(bytes, &got);
    struct Free {
        double* p;
        size_t b;
        hipStream_t st;
        ~Free() {
            (void)hipStreamSynchronize(st);
            dev_free(p, b);
        }
    } fr{w, got, st};
    double *s_old = w, *tmp = w + n, *part = w + 2 * n;
    std::vector<double> ph(nbk);
    const TGeom G{nx, ny, nz, 1.0 / nx, 1.0 / ny, cube ? 1.0 / nz : 1.0, (long long)(nx + 1) * ny * nz,
                  (long long)nx * (ny + 1) * nz};
    const double coef = dt / (phi * G.hx * G.hy * G.hz), rmw = 1.0 / mu_w, rmo = 1.0 / mu_o;
    const dim3 tiles = cube ? dim3((unsigned)((nx + 7) / 8), (unsigned)((ny + 7) / 8), (unsigned)((nz + 3) / 4))
                            : dim3((unsigned)((nx + 15) / 16), (unsigned)((ny + 15) / 16), 1);
    auto tile_step = [&](const double* sin, double* sout) {
        if (cube)
            hipLaunchKernelGGL((k_tr_tile_solve<8, 8, 4>), tiles, dim3(256), 0, st, u, q, (const double*)s_old, sin, G,
                               coef, rmw, rmo, sout);
        else
            hipLaunchKernelGGL((k_tr_tile_solve<16, 16, 1>), tiles, dim3(256), 0, st, u, q, (const double*)s_old, sin,
                               G, coef, rmw, rmo, sout);
    };
    auto residual = [&](const double* x) {
        hipLaunchKernelGGL(k_tr_residual, dim3(nbk), dim3(TT), 0, st, u, q, x, (const double*)s_old, G, coef, rmw,
                           rmo, part);
        LAUNCH_OK();
        HIP_OK(hipMemcpyAsync(ph.data(), part, sizeof(double) * nbk, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        double m = 0.0;
        for (double v : ph) m = std::max(m, v);
        return m;
    };
    HIP_OK(hipMemcpyAsync(s_old, s, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    TransportResult res;
    res.residual = residual(s);
    // outer steps in pairs (s -> tmp -> s), the residual read after every pair
    while (res.residual > newton_tol && res.sweeps < max_outer) {
        tile_step(s, tmp);
        tile_step(tmp, s);
        LAUNCH_OK();
        res.sweeps += 2;
        res.residual = residual(s);
    }
    res.converged = res.residual <= newton_tol;
    return res;
}

}  // namespace tgms
