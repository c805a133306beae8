// Fused kernels of the PCG iteration (paper section 5, Step 3) and of the
// two-grid preconditioner around the smoother and coarse solves.
//
// One PCG iteration in stream-function coordinates is
//   p = z + beta p;  q = K p;  alpha = rho / p.q           (k_dir_apply)
//   x += alpha p;  g -= alpha q                            (k_update)
//   z = B_TG g                                             (smoother, k_gather_res, coarse, residual,
//                                                            smoother, k_gather_final)
//   rho' = g.z, beta = rho'/rho (or (g.z - gold.z)/rho), |C z|^2  (k_gather_final)
// The kernels that form inner products run on a fixed grid of nred <= NRED
// workgroups (chosen by the autotuner) that loop over the tiles, and write one
// partial sum per workgroup; the next kernel sums those partials in a fixed order (so results do not depend on
// scheduling, and the kernel boundary makes the partials visible without device
// fences).  Every kernel first checks the done flag in sc and returns when it is
// set, so iterations queued after convergence cost only their launches.
#include "common.h"

namespace {

constexpr int TX = 64, TY = 4, NT = TX * TY;

__device__ inline bool finished(const double* __restrict__ sc) { return sc != nullptr && sc[SC_DONE] != 0.0; }

// Sum of NV values over the workgroup; the totals are returned to every thread.
template <int NV>
__device__ inline void group_sum(double (&v)[NV]) {
    __shared__ double sh[NV][NT / 64];
    const int tid = threadIdx.y * TX + threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += sh[k][w];
        v[k] = t;
    }
    __syncthreads();
}

constexpr int NRED = 256;  // most workgroups of a reducing kernel (stride of the partial arrays)

// Sum of the nred partials of array k, in fixed order, returned to every thread.
__device__ inline double sum_partials(const double* __restrict__ part, int k, int nred) {
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    double v[1] = {tid < nred ? part[k * NRED + tid] : 0.0};
    group_sum<1>(v);
    return v[0];
}

// 9-point stencil K at tile position (ty+1, tx+1) of an LDS tile with a one-vertex halo
template <typename T>
__device__ inline T stencil_tile(const T (&P)[TY + 2][TX + 2], int tx, int ty, const T* __restrict__ a, long long v,
                                 int nx, T sx2, T sy2) {
    const T A00 = a[v - nx - 1], A10 = a[v - nx], A01 = a[v - 1], A11 = a[v];
    const T s = sx2 + sy2;
    const T c6 = T(1.0 / 6.0), c3 = T(1.0 / 3.0);
    const T kx = sx2 * c6 - sy2 * c3, ky = sy2 * c6 - sx2 * c3;
    const int x = tx + 1, y = ty + 1;
    T r = s * c3 * (A00 + A10 + A01 + A11) * P[y][x];
    r += kx * ((A10 + A11) * P[y][x + 1] + (A00 + A01) * P[y][x - 1]);
    r += ky * ((A01 + A11) * P[y + 1][x] + (A00 + A10) * P[y - 1][x]);
    r -= s * c6 * (A11 * P[y + 1][x + 1] + A01 * P[y + 1][x - 1] + A10 * P[y - 1][x + 1] + A00 * P[y - 1][x - 1]);
    return r;
}

// p_out = z + beta p_in (beta = 0 on the first iteration), q = K p_out, and the
// workgroup's partial sum of p_out . q.  The workgroups loop over the tiles.
__global__ void __launch_bounds__(NT) k_dir_apply(const double* __restrict__ z, const double* __restrict__ pin,
                                                  double* __restrict__ pout, double* __restrict__ q,
                                                  const double* __restrict__ a, int nx, int ny, double sx2,
                                                  double sy2, const double* __restrict__ sc,
                                                  double* __restrict__ part) {
    if (finished(sc)) return;
    __shared__ double P[TY + 2][TX + 2];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int ntx = (nx + TX - 1) / TX, ntiles = ntx * ((ny + TY - 1) / TY);
    const double beta = sc[SC_BETA];
    double v[1] = {0.0};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
        __syncthreads();
        for (int e = tid; e < (TX + 2) * (TY + 2); e += NT) {
            const int ii = i0 - 1 + e % (TX + 2), jj = j0 - 1 + e / (TX + 2);
            double val = 0.0;
            if (ii >= 1 && ii < nx && jj >= 1 && jj < ny) {
                const long long vv = (long long)jj * nx + ii;
                val = z[vv] + beta * pin[vv];
            }
            P[e / (TX + 2)][e % (TX + 2)] = val;
        }
        __syncthreads();
        const int i = i0 + tx, j = j0 + ty;
        if (i < nx && j < ny) {
            const long long vv = (long long)j * nx + i;
            const double pc = P[ty + 1][tx + 1];
            pout[vv] = pc;
            double r = 0.0;
            if (i > 0 && j > 0) r = stencil_tile<double>(P, tx, ty, a, vv, nx, sx2, sy2);
            q[vv] = r;
            v[0] += pc * r;
        }
    }
    group_sum<1>(v);
    if (tid == 0) part[blockIdx.x] = v[0];
}

// alpha = rho / (p . q) from the partials of k_dir_apply (every workgroup forms it;
// workgroup 0 records it), then x += alpha p ; gold = g (flexible) ; g -= alpha q ;
// g32 = (float) g (mixed precision).  A non-positive p . q stops the iteration.
__global__ void __launch_bounds__(NT) k_update(long long n, double* __restrict__ sc, double* __restrict__ hist,
                                               const double* __restrict__ part, int nred, const double* __restrict__ p,
                                               const double* __restrict__ q, double* __restrict__ x,
                                               double* __restrict__ g, double* __restrict__ gold,
                                               float* __restrict__ g32) {
    if (finished(sc)) return;
    const double pq = sum_partials(part, 0, nred);
    const double al = sc[SC_RHO] / pq;
    const bool bad = !(pq > 0.0) || !(pq < INFINITY);
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) {
        sc[SC_PQ] = pq;
        sc[SC_ALPHA] = al;
        hist[2 * (int)sc[SC_IT]] = al;
        if (bad) {
            sc[SC_FLAG] = 1.0;
            sc[SC_DONE] = 1.0;
        }
    }
    if (bad) return;
    for (long long t = blockIdx.x * (long long)NT + tid; t < n; t += (long long)gridDim.x * NT) {
        x[t] += al * p[t];
        const double gv = g[t];
        if (gold) gold[t] = gv;
        const double gn = gv - al * q[t];
        g[t] = gn;
        if (g32) g32[t] = (float)gn;
    }
}

// eta * (sum of the patch solutions covering vertex (i, j)), in fixed patch order
template <typename T>
__device__ inline T gather_w(const Rect* __restrict__ rects, const T* __restrict__ w, int i, int j, int bx, int by,
                             int Nx, int Ny) {
    T s = T(0);
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
    return s;
}

struct GatherGeom {
    int nx, ny, bx, by, Nx, Ny;
};

// the sum of the patch solutions at vertex (i, j): the four slots when present
template <typename T>
__device__ inline T patch_sum(const Rect* __restrict__ rects, const T* __restrict__ w, const T* __restrict__ w4,
                              const GatherGeom& G, int i, int j) {
    if (w4) {
        const T* q = w4 + ((long long)j * G.nx + i) * 4;
        return (q[0] + q[1]) + (q[2] + q[3]);
    }
    return gather_w<T>(rects, w, i, j, G.bx, G.by, G.Nx, G.Ny);
}

// First smoothing of the two-grid cycle: z = eta * sum_i ext(w_i), t = g - K z.
template <typename T>
__global__ void __launch_bounds__(NT) k_gather_res(const Rect* __restrict__ rects, const T* __restrict__ w,
                                                   const T* __restrict__ w4, GatherGeom G, T eta,
                                                   const double* __restrict__ g, const double* __restrict__ a,
                                                   double sx2, double sy2, T* __restrict__ z, T* __restrict__ t,
                                                   const double* __restrict__ sc) {
    if (finished(sc)) return;
    // the tile holds z exactly as stored (in T); the residual is formed in FP64 and
    // rounded once, so an FP32 z does not lose the small residual to cancellation
    __shared__ double Z[TY + 2][TX + 2];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    for (int e = tid; e < (TX + 2) * (TY + 2); e += NT) {
        const int ii = i0 - 1 + e % (TX + 2), jj = j0 - 1 + e / (TX + 2);
        T val = T(0);
        if (ii >= 1 && ii < G.nx && jj >= 1 && jj < G.ny) val = eta * patch_sum<T>(rects, w, w4, G, ii, jj);
        Z[e / (TX + 2)][e % (TX + 2)] = double(val);
    }
    __syncthreads();
    const int i = i0 + tx, j = j0 + ty;
    if (i >= G.nx || j >= G.ny) return;
    const long long v = (long long)j * G.nx + i;
    z[v] = T(Z[ty + 1][tx + 1]);
    t[v] = (i > 0 && j > 0) ? T(g[v] - stencil_tile<double>(Z, tx, ty, a, v, G.nx, sx2, sy2)) : T(0);
}

// Last smoothing of the two-grid cycle: z = zin + eta * sum_i ext(w_i) (zin may be
// null), written as FP64.  With part: the workgroup's partial sums of g.z, gold.z
// and |C z|^2 (the workgroups loop over the tiles).
template <typename T>
__global__ void __launch_bounds__(NT) k_gather_final(const Rect* __restrict__ rects, const T* __restrict__ w,
                                                     const T* __restrict__ w4, GatherGeom G, T eta, const T* __restrict__ zin,
                                                     double* __restrict__ zout, double sx, double sy,
                                                     const double* __restrict__ g, const double* __restrict__ gold,
                                                     const double* __restrict__ sc, double* __restrict__ part) {
    if (finished(sc)) return;
    __shared__ double Z[TY + 1][TX + 1];  // the tile and one vertex beyond it in +x and +y
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int ntx = (G.nx + TX - 1) / TX, ntiles = ntx * ((G.ny + TY - 1) / TY);
    double v[3] = {0.0, 0.0, 0.0};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
        __syncthreads();
        for (int e = tid; e < (TX + 1) * (TY + 1); e += NT) {
            const int ii = i0 + e % (TX + 1), jj = j0 + e / (TX + 1);
            double val = 0.0;
            if (ii >= 1 && ii < G.nx && jj >= 1 && jj < G.ny) {
                T s = eta * patch_sum<T>(rects, w, w4, G, ii, jj);
                if (zin) s += zin[(long long)jj * G.nx + ii];
                val = (double)s;
            }
            Z[e / (TX + 1)][e % (TX + 1)] = val;
        }
        __syncthreads();
        const int i = i0 + tx, j = j0 + ty;
        if (i < G.nx && j < G.ny) {
            const long long vv = (long long)j * G.nx + i;
            const double pc = Z[ty][tx];
            zout[vv] = pc;
            if (part) {
                v[0] += g[vv] * pc;
                if (gold) v[1] += gold[vv] * pc;
                // faces keyed by vertex (i, j): x-face (i, j) for i >= 1, y-face (i, j) for j >= 1
                if (i > 0) {
                    const double d = (Z[ty + 1][tx] - pc) * sx;
                    v[2] += d * d;
                }
                if (j > 0) {
                    const double d = (Z[ty][tx + 1] - pc) * sy;
                    v[2] += d * d;
                }
            }
        }
    }
    if (!part) return;
    group_sum<3>(v);
    if (tid == 0) {
        part[blockIdx.x] = v[0];
        part[NRED + blockIdx.x] = v[1];
        part[2 * NRED + blockIdx.x] = v[2];
    }
}

// rho, beta, the relative residual, the iteration count and the done flag from the
// partials of k_gather_final (first: rho_0 and |z_0|^2).  One workgroup.
__global__ void __launch_bounds__(NT) k_finalize(double* __restrict__ sc, double* __restrict__ hist,
                                                 const double* __restrict__ part, int nred, int first) {
    if (finished(sc)) return;
    const double gz = sum_partials(part, 0, nred), zgold = sum_partials(part, 1, nred),
                 zn2 = sum_partials(part, 2, nred);
    if (threadIdx.x != 0 || threadIdx.y != 0) return;
    if (first) {
        sc[SC_RHO] = gz;
        sc[SC_Z02] = zn2;
        sc[SC_ZN2] = zn2;
        sc[SC_REL2] = 1.0;
        sc[SC_IT] = 0.0;
        sc[SC_FLAG] = 0.0;
        sc[SC_BETA] = 0.0;
        sc[SC_DONE] = (zn2 > 0.0 && sc[SC_MAXIT] > 0.0) ? 0.0 : 1.0;
        return;
    }
    const int it = (int)sc[SC_IT];
    const double rho = sc[SC_RHO];
    const double beta = (sc[SC_FLEX] != 0.0) ? (gz - zgold) / rho : gz / rho;
    sc[SC_BETA] = beta;
    sc[SC_RHO] = gz;
    sc[SC_ZN2] = zn2;
    const double rel2 = zn2 / sc[SC_Z02];
    sc[SC_REL2] = rel2;
    hist[2 * it + 1] = beta;
    sc[SC_IT] = it + 1;
    if (!(rel2 < INFINITY) || !(beta == beta)) sc[SC_FLAG] = 1.0;
    if (sc[SC_FLAG] != 0.0 || rel2 <= sc[SC_RTOL2] || it + 1 >= (int)sc[SC_MAXIT]) sc[SC_DONE] = 1.0;
}

// t = g - K z
template <typename T>
__global__ void __launch_bounds__(NT) k_residual(const T* __restrict__ z, const double* __restrict__ g,
                                                 T* __restrict__ t, const double* __restrict__ a, int nx, int ny,
                                                 double sx2, double sy2, const double* __restrict__ sc) {
    if (finished(sc)) return;
    __shared__ double P[TY + 2][TX + 2];  // z as stored, widened; FP64 residual rounded once to T
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    for (int e = tid; e < (TX + 2) * (TY + 2); e += NT) {
        const int ii = i0 - 1 + e % (TX + 2), jj = j0 - 1 + e / (TX + 2);
        P[e / (TX + 2)][e % (TX + 2)] =
            (ii >= 1 && ii < nx && jj >= 1 && jj < ny) ? double(z[(long long)jj * nx + ii]) : 0.0;
    }
    __syncthreads();
    const int i = i0 + tx, j = j0 + ty;
    if (i >= nx || j >= ny) return;
    const long long v = (long long)j * nx + i;
    t[v] = (i > 0 && j > 0) ? T(g[v] - stencil_tile<double>(P, tx, ty, a, v, nx, sx2, sy2)) : T(0);
}

inline dim3 tiles(tgms_ctx* c) { return dim3((c->nx + TX - 1) / TX, (c->ny + TY - 1) / TY); }
inline GatherGeom ggeom(tgms_ctx* c) { return GatherGeom{c->nx, c->ny, c->bx, c->by, c->Nx, c->Ny}; }
template <typename T>
inline const T* slots(tgms_ctx* c) {
    if (!c->slots) return nullptr;
    return sizeof(T) == 8 ? (const T*)c->patW4 : (const T*)c->patW4_32;
}

}  // namespace

namespace tgms {

unsigned pcg_tiles(tgms_ctx*) { return NRED; }
int nred_max() { return NRED; }

void dir_apply(tgms_ctx* c, const double* z, const double* pin, double* pout, double* q) {
    ProfScope ps(c, PK_APPLYK);
    hipLaunchKernelGGL(k_dir_apply, dim3(c->nred), dim3(TX, TY), 0, c->stream, z, pin, pout, q, (const double*)c->a,
                       c->nx, c->ny, c->sx * c->sx, c->sy * c->sy, (const double*)c->sc, c->part);
    LAUNCH_OK();
}

void update(tgms_ctx* c, const double* p, const double* q, double* x, double* g, double* gold, float* g32) {
    const long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_update, dim3(c->nred), dim3(TX, TY), 0, c->stream, n, c->sc, c->hist, (const double*)c->part,
                       c->nred, p, q, x, g, gold, g32);
    LAUNCH_OK();
}

template <typename T>
void gather_res(tgms_ctx* c, const T* w, const double* g, T* z, T* t, const double* sc) {
    hipLaunchKernelGGL((k_gather_res<T>), tiles(c), dim3(TX, TY), 0, c->stream, c->patch, w, slots<T>(c), ggeom(c),
                       T(c->eta), g, (const double*)c->a, c->sx * c->sx, c->sy * c->sy, z, t, sc);
    LAUNCH_OK();
}
template void gather_res<double>(tgms_ctx*, const double*, const double*, double*, double*, const double*);
template void gather_res<float>(tgms_ctx*, const float*, const double*, float*, float*, const double*);

template <typename T>
void gather_final(tgms_ctx* c, const T* w, const T* zin, double* zout, const double* g, const double* gold,
                  bool with_dots, bool first) {
    const double* sc = with_dots ? c->sc : nullptr;
    if (with_dots)
        hipLaunchKernelGGL((k_gather_final<T>), dim3(c->nred), dim3(TX, TY), 0, c->stream, c->patch, w, slots<T>(c),
                           ggeom(c), T(c->eta), zin, zout, c->sx, c->sy, g, gold, sc, c->part);
    else
        hipLaunchKernelGGL((k_gather_final<T>), dim3(tiles(c).x * tiles(c).y), dim3(TX, TY), 0, c->stream, c->patch,
                           w, slots<T>(c), ggeom(c), T(c->eta), zin, zout, c->sx, c->sy, g, gold, sc, (double*)nullptr);
    LAUNCH_OK();
    if (with_dots) {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TX, TY), 0, c->stream, c->sc, c->hist, (const double*)c->part,
                           c->nred, first ? 1 : 0);
        LAUNCH_OK();
    }
}
template void gather_final<double>(tgms_ctx*, const double*, const double*, double*, const double*, const double*,
                                   bool, bool);
template void gather_final<float>(tgms_ctx*, const float*, const float*, double*, const double*, const double*, bool,
                                  bool);

template <typename T>
void residual(tgms_ctx* c, const T* z, const double* g, T* t, const double* sc) {
    ProfScope ps(c, PK_APPLYK);
    hipLaunchKernelGGL((k_residual<T>), tiles(c), dim3(TX, TY), 0, c->stream, z, g, t, (const double*)c->a, c->nx,
                       c->ny, c->sx * c->sx, c->sy * c->sy, sc);
    LAUNCH_OK();
}
template void residual<double>(tgms_ctx*, const double*, const double*, double*, const double*);
template void residual<float>(tgms_ctx*, const float*, const double*, float*, const double*);

}  // namespace tgms
