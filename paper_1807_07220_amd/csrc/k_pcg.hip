// Fused kernels of the PCG iteration (paper section 5, Step 3) and of the
// two-grid preconditioner around the smoother and coarse solves.
//
// One PCG iteration in stream-function coordinates is these kernels (the coarse
// solve one product with an explicit inverse, or the levels of the cyclic reduction):
//   [finalise the last iteration: rho' = g.z, beta, |C z|^2 test]
//   p = z + beta p;  q = K p;  partial p.q                        (k_dir_apply)
//   alpha = rho / p.q, x += alpha p and g -= alpha q             (k_pcg_update)
//   z = B_TG g: the first smoothing; z1 = eta sum ext(w), t = g - K z1 and the
//   block restriction W_b^T t (k_gather_res_restrict); coarse accumulation and
//   the two triangular products, or one product with the explicit inverse
//   (k_dense.hip); z1' = z1 + W c and the second smoothing's right-hand side
//   g - K z1' (k_prolong_residual); the second smoothing (k_smooth.hip);
//   z = z1' + eta sum ext(w) with the partials of g.z, gold.z and |C z|^2
//   (k_gather_final).
// The partials of k_gather_final are finalised by the next iteration's
// k_dir_apply (every workgroup forms the same sums; workgroup 0 records them),
// or by k_finalize where the host needs the scalars (after the first
// preconditioning and at the end of each group of queued iterations).  A
// "pending" flag in sc tells which: set by k_gather_final, cleared by k_finalize
// or by k_pcg_update (the kernel after the one that finalised), so that no
// workgroup reads a scalar another workgroup of the same kernel writes.
// The reducing kernels run on a fixed grid of nred <= NRED workgroups (chosen by
// the autotuner) that loop over the tiles and write one partial each; the
// consumer sums them in a fixed order (results do not depend on scheduling, and
// the kernel boundary makes them visible without device fences).  Every kernel
// first checks the done flag in sc, so iterations queued after convergence cost
// only their launches.
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

constexpr int NRED = 1024;  // most workgroups of a reducing kernel (stride of the partial arrays)

// Sum of the nred partials of array k, in fixed order (each thread its strided share,
// then the workgroup sum), returned to every thread.
__device__ inline double sum_partials(const double* __restrict__ part, int k, int nred) {
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    for (int j = tid; j < nred; j += NT) v[0] += part[k * NRED + j];
    group_sum<1>(v);
    return v[0];
}

// 9-point stencil K at tile position (y, tx+1) of an LDS tile of H rows with a
// one-vertex halo, with the four cell weights around the vertex (SW, SE, NW, NE)
// already loaded
template <int H>
__device__ inline double stencil_tile4(const double (&P)[H + 2][TX + 2], int tx, int y, const double (&A)[4],
                                       double sx2, double sy2) {
    const double A00 = A[0], A10 = A[1], A01 = A[2], A11 = A[3];
    const double s = sx2 + sy2;
    const double c6 = 1.0 / 6.0, c3 = 1.0 / 3.0;
    const double kx = sx2 * c6 - sy2 * c3, ky = sy2 * c6 - sx2 * c3;
    const int x = tx + 1;
    double r = s * c3 * (A00 + A10 + A01 + A11) * P[y][x];
    r += kx * ((A10 + A11) * P[y][x + 1] + (A00 + A01) * P[y][x - 1]);
    r += ky * ((A01 + A11) * P[y + 1][x] + (A00 + A10) * P[y - 1][x]);
    r -= s * c6 * (A11 * P[y + 1][x + 1] + A01 * P[y + 1][x - 1] + A10 * P[y - 1][x + 1] + A00 * P[y - 1][x - 1]);
    return r;
}

// The scalars after an iteration's last gather, from its partials gpart (g.z, gold.z,
// |C z|^2): beta, rho' and the relative residual; recorded by the calling thread
// when rec.  Returns true when the iteration stops here: converged, a breakdown,
// or (rec only: the other workgroups do not read the iteration count, which rec
// updates) maxit reached.
__device__ inline bool finalise(double* __restrict__ sc, double* __restrict__ hist, const double* __restrict__ gpart,
                                int nred, bool rec, double* beta_out) {
    const double gz = sum_partials(gpart, 0, nred), zgold = sum_partials(gpart, 1, nred),
                 zn2 = sum_partials(gpart, 2, nred);
    const double rho = sc[SC_RHO];
    const double beta = (sc[SC_FLEX] != 0.0) ? (gz - zgold) / rho : gz / rho;
    const double rel2 = zn2 / sc[SC_Z02];
    const bool bad = !(rel2 < INFINITY) || !(beta == beta);
    bool stop = bad || rel2 <= sc[SC_RTOL2];
    if (rec) {
        const int it = (int)sc[SC_IT];
        stop = stop || it + 1 >= (int)sc[SC_MAXIT];
        sc[SC_BETA] = beta;
        sc[SC_RHO_NEW] = gz;
        sc[SC_ZN2] = zn2;
        sc[SC_REL2] = rel2;
        hist[2 * it + 1] = beta;
        sc[SC_IT] = it + 1;
        if (bad) sc[SC_FLAG] = 1.0;
        if (stop) sc[SC_DONE] = 1.0;
    }
    *beta_out = beta;
    return stop;
}

// p_out = z + beta p_in, q = K p_out, and the workgroup's partial sum of p_out . q
// (part).  beta comes from finalising the pending partials gpart, else from sc.  The
// workgroups loop over tiles of 64 x 4 RPT vertices, RPT rows per thread; the loads
// of a tile (cell weights, z and p_in on the tile and its halo) are issued before
// the previous tile's stencil (and the first tile's before the partials are
// finalised), at indices clamped into the grid and zeroed outside it, so that they
// are in flight while the workgroup computes.  Past the last tile the prefetch
// repeats the grid's last tile (an L2 hit: every workgroup ends there).
template <int RPT>
__global__ void __launch_bounds__(NT) k_dir_apply(const double* __restrict__ z, const double* __restrict__ pin,
                                                  double* __restrict__ pout, double* __restrict__ q,
                                                  const double* __restrict__ a, int nx, int ny, double sx2,
                                                  double sy2, double* __restrict__ sc, double* __restrict__ hist,
                                                  const double* __restrict__ gpart, int nred,
                                                  double* __restrict__ part) {
    if (finished(sc)) return;
    constexpr int H = TY * RPT, NE = (TX + 2) * (H + 2), HE = (NE + NT - 1) / NT;
    __shared__ double P[H + 2][TX + 2];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int ntx = (nx + TX - 1) / TX, ntiles = ntx * ((ny + H - 1) / H);
    struct Tile {
        double A[RPT][4];  // cell weights of the thread's vertices
        double Z[HE], Q[HE];  // z and p_in of its halo-tile elements
    };
    auto load = [&](int tile, Tile& T) {
        const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * H, i = i0 + tx;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int j = j0 + ty + TY * r;
            const bool in = i > 0 && j > 0 && i < nx && j < ny;
            const long long vv = in ? (long long)j * nx + i : nx + 1;
            const double w0 = a[vv - nx - 1], w1 = a[vv - nx], w2 = a[vv - 1], w3 = a[vv];
            T.A[r][0] = in ? w0 : 0.0;
            T.A[r][1] = in ? w1 : 0.0;
            T.A[r][2] = in ? w2 : 0.0;
            T.A[r][3] = in ? w3 : 0.0;
        }
#pragma unroll
        for (int h = 0; h < HE; ++h) {
            const int e = tid + h * NT, ii = i0 - 1 + e % (TX + 2), jj = j0 - 1 + e / (TX + 2);
            const bool in = e < NE && ii >= 1 && ii < nx && jj >= 1 && jj < ny;
            const long long ve = in ? (long long)jj * nx + ii : 0;
            const double zv = z[ve], pv = pin[ve];
            T.Z[h] = in ? zv : 0.0;
            T.Q[h] = in ? pv : 0.0;
        }
    };
    Tile cur;
    load(min((int)blockIdx.x, ntiles - 1), cur);
    double beta = sc[SC_BETA];
    if (sc[SC_PENDING] != 0.0) {
        const bool rec = blockIdx.x == 0 && tid == 0;
        if (finalise(sc, hist, gpart, nred, rec, &beta)) return;
    }
    double v[1] = {0.0};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * H;
        const int i = i0 + tx;
#pragma unroll
        for (int h = 0; h < HE; ++h) {
            const int e = tid + h * NT;
            if (e < NE) P[e / (TX + 2)][e % (TX + 2)] = cur.Z[h] + beta * cur.Q[h];
        }
        double A[RPT][4];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k) A[r][k] = cur.A[r][k];
        __syncthreads();
        load(min(tile + (int)gridDim.x, ntiles - 1), cur);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int y = ty + TY * r, j = j0 + y;
            if (i < nx && j < ny) {
                const long long vv = (long long)j * nx + i;
                const double pc = P[y + 1][tx + 1];
                pout[vv] = pc;
                const double qv = (i > 0 && j > 0) ? stencil_tile4<H>(P, tx, y + 1, A[r], sx2, sy2) : 0.0;
                q[vv] = qv;
                v[0] += pc * qv;
            }
        }
        __syncthreads();
    }
    group_sum<1>(v);
    if (tid == 0) part[blockIdx.x] = v[0];
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
        const long long plane = (long long)G.nx * G.ny, v = (long long)j * G.nx + i;
        return (w4[v] + w4[plane + v]) + (w4[2 * plane + v] + w4[3 * plane + v]);
    }
    return gather_w<T>(rects, w, i, j, G.bx, G.by, G.Nx, G.Ny);
}

// Coarse-space data of the two-grid kernels: stream functions W
// [block][owned vertex][slot], per-block unknown ids and counts.
template <typename T>
struct CoarseW {
    const T* W;
    int mu;
    const int* unk;
    const int* nunk;
};

// First gather and restriction, one workgroup per coarse block: z1 = eta * (sum of the
// patch solutions), t = g - K z1 (formed in FP64 from z1 as stored, rounded once) on
// the block's vertices, and cy[b] = W_b^T t.  LDS: the block with a one-vertex halo
// (FP64), t on the block, and the restriction partials.
template <typename T>
__global__ void __launch_bounds__(NT) k_gather_res_restrict(const Rect* __restrict__ rects, const T* __restrict__ w,
                                                            const T* __restrict__ w4, GatherGeom G, T eta,
                                                            const double* __restrict__ g,
                                                            const double* __restrict__ a, double sx2, double sy2,
                                                            T* __restrict__ z, T* __restrict__ t, CoarseW<T> C,
                                                            T* __restrict__ cy, const double* __restrict__ sc) {
    if (finished(sc)) return;
    extern __shared__ double smem[];
    const int bx = G.bx, by = G.by, pw = bx + 2, nown = bx * by;
    double* Z = smem;                                  // (by + 2) x (bx + 2)
    T* tb = reinterpret_cast<T*>(Z + (by + 2) * pw);  // nown
    const int tid = threadIdx.y * TX + threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int blk = blockIdx.x, i0 = (blk % G.Nx) * bx, j0 = (blk / G.Nx) * by;
    // the first owned vertex of this thread: its g and weights load with the tile
    VertexData d0{};
    if (tid < nown) {
        const int i = i0 + tid % bx, j = j0 + tid / bx;
        d0 = vertex_data(g, a, (long long)j * G.nx + i, G.nx, i > 0 && j > 0);
    }
    for (int e = tid; e < (bx + 2) * (by + 2); e += NT) {
        const int ii = i0 - 1 + e % pw, jj = j0 - 1 + e / pw;
        T val = T(0);
        if (ii >= 1 && ii < G.nx && jj >= 1 && jj < G.ny) val = eta * patch_sum<T>(rects, w, w4, G, ii, jj);
        Z[e] = double(val);
    }
    __syncthreads();
    for (int vl = tid; vl < nown; vl += NT) {
        const int aa = vl % bx, bb = vl / bx, i = i0 + aa, j = j0 + bb;
        const long long v = (long long)j * G.nx + i;
        const bool in = i > 0 && j > 0;
        const VertexData d = vl == tid ? d0 : vertex_data(g, a, v, G.nx, in);
        z[v] = T(Z[(bb + 1) * pw + aa + 1]);
        const T tv = in ? T(d.g - stencil_at4(Z, pw, aa + 1, bb + 1, d.A, sx2, sy2)) : T(0);
        t[v] = tv;
        tb[vl] = tv;
    }
    __syncthreads();
    // restriction cy[b][u] = sum_v W[v][u] t[v]: one wavefront per unknown, lanes over v
    const int nu = C.nunk[blk];
    const T* Wb = C.W + (long long)blk * nown * C.mu;
    for (int u = wv; u < nu; u += NT / 64) {
        T acc = T(0);
        for (int vl = lane; vl < nown; vl += 64) acc += Wb[(long long)vl * C.mu + u] * tb[vl];
        acc = wave_sum(acc);
        if (lane == 0) cy[(long long)blk * C.mu + u] = acc;
    }
}

// Last smoothing of the two-grid cycle: z = zin + eta * sum_i ext(w_i) (zin may be
// null), written as FP64.  With part: the workgroup's partial sums of g.z, gold.z
// and |C z|^2 (the workgroups loop over tiles of 64 x 4 RPT vertices), and the
// pending flag set.
template <typename T, int RPT>
__global__ void __launch_bounds__(NT) k_gather_final(const Rect* __restrict__ rects, const T* __restrict__ w,
                                                     const T* __restrict__ w4, GatherGeom G, T eta, const T* __restrict__ zin,
                                                     double* __restrict__ zout, double sx, double sy,
                                                     const double* __restrict__ g, const double* __restrict__ gold,
                                                     const double* __restrict__ sc, double* __restrict__ part,
                                                     double* __restrict__ sc_pending) {
    if (finished(sc)) return;
    constexpr int H = TY * RPT;
    __shared__ double Z[H + 1][TX + 1];  // the tile and one vertex beyond it in +x and +y
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int ntx = (G.nx + TX - 1) / TX, ntiles = ntx * ((G.ny + H - 1) / H);
    double v[3] = {0.0, 0.0, 0.0};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * H;
        const int i = i0 + tx;
        double gv[RPT], gov[RPT];  // loaded with the tile
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int j = j0 + ty + TY * r;
            const long long vv = (long long)j * G.nx + i;
            const bool in = part && i < G.nx && j < G.ny;
            gv[r] = in ? g[vv] : 0.0;
            gov[r] = (in && gold) ? gold[vv] : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < (TX + 1) * (H + 1); e += NT) {
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
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int y = ty + TY * r, j = j0 + y;
            if (i < G.nx && j < G.ny) {
                const long long vv = (long long)j * G.nx + i;
                const double pc = Z[y][tx];
                zout[vv] = pc;
                if (part) {
                    v[0] += gv[r] * pc;
                    if (gold) v[1] += gov[r] * pc;
                    // faces keyed by vertex (i, j): x-face (i, j) for i >= 1, y-face (i, j) for j >= 1
                    if (i > 0) {
                        const double d = (Z[y + 1][tx] - pc) * sx;
                        v[2] += d * d;
                    }
                    if (j > 0) {
                        const double d = (Z[y][tx + 1] - pc) * sy;
                        v[2] += d * d;
                    }
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
        if (blockIdx.x == 0) sc_pending[0] = 1.0;
    }
}

// The scalars from the partials of k_gather_final, one workgroup.  first: rho_0 and
// |z_0|^2 of the initial preconditioning; otherwise finalise the pending partials
// (if any) as k_dir_apply would, and clear the flag.
__global__ void __launch_bounds__(NT) k_finalize(double* __restrict__ sc, double* __restrict__ hist,
                                                 const double* __restrict__ part, int nred, int first) {
    if (finished(sc)) return;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if (first) {
        const double gz = sum_partials(part, 0, nred), zn2 = sum_partials(part, 2, nred);
        if (tid != 0) return;
        sc[SC_RHO] = gz;
        sc[SC_RHO_NEW] = gz;
        sc[SC_Z02] = zn2;
        sc[SC_ZN2] = zn2;
        sc[SC_REL2] = 1.0;
        sc[SC_IT] = 0.0;
        sc[SC_FLAG] = 0.0;
        sc[SC_BETA] = 0.0;
        sc[SC_PENDING] = 0.0;
        // a non-finite preconditioned residual is a breakdown, not convergence
        const bool finite = zn2 < INFINITY && gz == gz;
        sc[SC_FLAG] = finite ? 0.0 : 1.0;
        sc[SC_DONE] = (finite && zn2 > 0.0 && sc[SC_MAXIT] > 0.0) ? 0.0 : 1.0;
        return;
    }
    if (sc[SC_PENDING] == 0.0) return;
    double beta;
    __syncthreads();  // every thread has read the flag before thread 0 clears it
    finalise(sc, hist, part, nred, tid == 0, &beta);
    if (tid == 0) sc[SC_PENDING] = 0.0;
}

inline dim3 tiles(tgms_ctx* c) { return dim3((c->nx + TX - 1) / TX, (c->ny + TY - 1) / TY); }
inline GatherGeom ggeom(tgms_ctx* c) { return GatherGeom{c->nx, c->ny, c->bx, c->by, c->Nx, c->Ny}; }
template <typename T>
inline const T* slots(tgms_ctx* c) {
    if (!c->slots) return nullptr;
    return sizeof(T) == 8 ? (const T*)c->patW4 : (const T*)c->patW4_32;
}

// t = g - K z on the interior vertices (zero elsewhere), FP64: the residual between the
// steps of the unfused two-grid variants (several smoothings, additive coarse correction)
// The PCG update ahead of a preconditioning: alpha = rho' / p.q from the partials of
// k_dir_apply (every workgroup forms the sum, in the order of a 256-thread workgroup;
// workgroup 0 records the scalars), then on the interior vertices g = gin - alpha q
// (FP64, and rounded once to T for the smoother where gT is given) and x += alpha p.
// A p.q that is not positive and finite stops the iteration (breakdown flag).  Each
// thread takes UP vertices, whose vectors are loaded before the partials are summed
// so that both are in flight together.
template <typename T>
__global__ void __launch_bounds__(NT) k_pcg_update(FusedUpdate U, T* __restrict__ gT, int nx, int ny) {
    if (finished(U.sc)) return;
    constexpr int UP = 4;
    const int t = threadIdx.y * TX + threadIdx.x;
    const long long nv = (long long)nx * ny;
    double G[UP], Q[UP], P[UP], X[UP];
    long long vv[UP];
#pragma unroll
    for (int h = 0; h < UP; ++h) {
        vv[h] = (long long)blockIdx.x * (UP * NT) + h * NT + t;
        const long long k = vv[h] < nv ? vv[h] : nv - 1;
        G[h] = U.gin[k];
        Q[h] = U.q[k];
        P[h] = U.p[k];
        X[h] = U.x[k];
    }
    __shared__ double red[NT / 64];
    double v = 0.0;
    for (int j = t; j < U.nred; j += NT) v += U.part[j];
    v = wave_sum(v);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    const double pq = red[0] + red[1] + red[2] + red[3];
    const double rho = U.sc[SC_RHO_NEW];
    const double al = rho / pq;
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
#pragma unroll
    for (int h = 0; h < UP; ++h) {
        const long long k = vv[h];
        if (k >= nv || k % nx == 0 || k < nx) continue;  // past the end, or a boundary vertex
        const double gn = G[h] - al * Q[h];
        U.gout[k] = gn;
        U.x[k] = X[h] + al * P[h];
        if (gT != nullptr) gT[k] = T(gn);
    }
}

// The second smoothing's right-hand side: z1' = z1 + W c on the coarse blocks' vertices
// (written to Pr.z1p) and t = g - K z1' there, formed in FP64 and rounded once to T.
// One workgroup per group of gx x gy coarse blocks (several small blocks share one
// tile); the one-vertex halo of z1' is recomputed from the neighbouring blocks' W and c
// (the same arithmetic as the group's own vertices), so that every vertex of t is a
// function of that vertex alone.  The loads that do not depend on c (z1, the first QB
// entries of each W row, the own vertices' g and cell weights) are issued before the
// coefficients are staged; W rows are read QB entries at a time, the indices past the
// row clamped to its last entry and multiplied by zero coefficients, so that each batch
// is in flight at once and the sum is that of the row's nu entries.
template <typename T>
__global__ void __launch_bounds__(NT) k_prolong_residual(PreResidual<T> Pr, T* __restrict__ t, int nx, int ny,
                                                         int bx, int by, int Nx, int gx, int gy,
                                                         const double* __restrict__ sc) {
    if (finished(sc)) return;
    constexpr int QB = 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Ny = ny / by, ngx = (Nx + gx - 1) / gx;
    const int I0 = (int)(blockIdx.x % ngx) * gx, J0 = (int)(blockIdx.x / ngx) * gy;  // the group's first block
    const int ow = gx * bx, oh = gy * by;            // the group's vertex rectangle
    const int pw = ow + 2, ph = oh + 2, sbx = gx + 2;  // tile with halo; staged blocks per row
    const int mu = Pr.mu, nown = bx * by, ntile = pw * ph, nco = ow * oh;
    const int tid = threadIdx.y * TX + threadIdx.x;
    double* Zt = reinterpret_cast<double*>(smem_raw);
    T* cb = reinterpret_cast<T*>(Zt + ntile);  // [(gx+2)(gy+2)][mu]: the coefficients of the blocks around
    // tile element e: vertex (ii, jj), its block's W row and staged-block index (-1 outside the domain)
    struct Elem {
        long long v;
        const T* Wv;
        int nb;
    };
    auto elem = [&](int e) {
        const int ii = I0 * bx - 1 + e % pw, jj = J0 * by - 1 + e / pw;
        Elem x{(long long)jj * nx + ii, Pr.W, -1};
        if (ii >= 1 && ii < nx && jj >= 1 && jj < ny) {
            const int Ib = ii / bx, Jb = jj / by;
            x.Wv = Pr.W + ((long long)(Jb * Nx + Ib) * nown + (jj % by) * bx + ii % bx) * mu;
            x.nb = (Jb - J0 + 1) * sbx + (Ib - I0 + 1);
        }
        return x;
    };
    auto load_w = [&](const Elem& x, int q0, T (&w)[QB]) {
#pragma unroll
        for (int q = 0; q < QB; ++q) w[q] = x.Wv[min(q0 + q, mu - 1)];
    };
    // prefetch: the first tile element's z1 and W entries, the first own vertex's data
    const Elem x0 = elem(tid < ntile ? tid : 0);
    T w0[QB];
    load_w(x0, 0, w0);
    const T z0 = x0.nb >= 0 ? Pr.z1[x0.v] : T(0);
    const int r0 = tid < nco ? tid : 0, i0v = I0 * bx + r0 % ow, j0v = J0 * by + r0 / ow;
    const bool in0 = i0v > 0 && j0v > 0 && i0v < nx && j0v < ny;
    const VertexData d0 = vertex_data(Pr.g, Pr.a, in0 ? (long long)j0v * nx + i0v : 0, nx, in0);
    for (int e = tid; e < sbx * (gy + 2) * mu; e += NT) {
        const int nb = e / mu, uu = e % mu, Ib = I0 + nb % sbx - 1, Jb = J0 + nb / sbx - 1;
        T val = T(0);
        if (Ib >= 0 && Ib < Nx && Jb >= 0 && Jb < Ny) {
            const int b = Jb * Nx + Ib;
            if (uu < Pr.nunk[b]) val = Pr.c[Pr.unk[(long long)b * mu + uu]];
        }
        cb[e] = val;
    }
    __syncthreads();
    for (int e = tid; e < ntile; e += NT) {
        const bool first = e == tid;
        const Elem x = first ? x0 : elem(e);
        const int ex = e % pw, ey = e / pw;
        const bool own = ex >= 1 && ex <= ow && ey >= 1 && ey <= oh && I0 * bx - 1 + ex < nx && J0 * by - 1 + ey < ny;
        double val = 0.0;
        if (x.nb >= 0) {
            const T* cv = cb + x.nb * mu;
            T s = T(0);
            T w[QB];
            for (int q0 = 0; q0 < mu; q0 += QB) {
                if (first && q0 == 0) {
#pragma unroll
                    for (int q = 0; q < QB; ++q) w[q] = w0[q];
                } else {
                    load_w(x, q0, w);
                }
#pragma unroll
                for (int q = 0; q < QB; ++q) s += w[q] * (q0 + q < mu ? cv[q0 + q] : T(0));
            }
            const T zz = (first ? z0 : Pr.z1[x.v]) + s;
            val = double(zz);
            if (own) Pr.z1p[x.v] = zz;
        } else if (own) {
            Pr.z1p[x.v] = T(0);
        }
        Zt[e] = val;
    }
    __syncthreads();
    for (int r = tid; r < nco; r += NT) {
        const int aa = r % ow, bb = r / ow, i = I0 * bx + aa, j = J0 * by + bb;
        if (i >= nx || j >= ny) continue;  // past the last block of an edge group
        const long long v = (long long)j * nx + i;
        if (i == 0 || j == 0) {
            t[v] = T(0);
            continue;
        }
        const VertexData d = r == tid ? d0 : vertex_data(Pr.g, Pr.a, v, nx, true);
        t[v] = T(d.g - stencil_at4(Zt, pw, aa + 1, bb + 1, d.A, Pr.sx2, Pr.sy2));
    }
}

__global__ void k_vertex_residual(const double* __restrict__ g, const double* __restrict__ z,
                                  const double* __restrict__ a, int nx, int ny, double sx2, double sy2,
                                  double* __restrict__ t) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= (long long)nx * ny) return;
    const int i = (int)(v % nx), j = (int)(v / nx);
    if (i == 0 || j == 0) {
        t[v] = 0.0;
        return;
    }
    auto Z = [&](int ii, int jj) { return (ii >= 1 && ii < nx && jj >= 1 && jj < ny) ? z[(long long)jj * nx + ii] : 0.0; };
    const Stencil9 k = stencil9(a[v - nx - 1], a[v - nx], a[v - 1], a[v], sx2, sy2);
    const double kz = k.c * Z(i, j) + k.e * Z(i + 1, j) + k.w * Z(i - 1, j) + k.n * Z(i, j + 1) + k.s * Z(i, j - 1) +
                      k.ne * Z(i + 1, j + 1) + k.nw * Z(i - 1, j + 1) + k.se * Z(i + 1, j - 1) + k.sw * Z(i - 1, j - 1);
    t[v] = g[v] - kz;
}

}  // namespace

namespace tgms {

void vertex_residual(tgms_ctx* c, const double* g, const double* z, double* t) {
    const long long n = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_vertex_residual, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, g, z,
                       (const double*)c->a, c->nx, c->ny, c->sx * c->sx, c->sy * c->sy, t);
    LAUNCH_OK();
}


unsigned pcg_tiles(tgms_ctx*) { return NRED; }
int nred_max() { return NRED; }

void dir_apply(tgms_ctx* c, const double* z, const double* pin, double* pout, double* q) {
    ProfScope ps(c, PK_APPLYK);
    if (c->rpt == 4)
        hipLaunchKernelGGL(k_dir_apply<4>, dim3(c->nred), dim3(TX, TY), 0, c->stream, z, pin, pout, q,
                           (const double*)c->a, c->nx, c->ny, c->sx * c->sx, c->sy * c->sy, c->sc, c->hist,
                           (const double*)c->part, c->nred, c->part2);
    else
        hipLaunchKernelGGL(k_dir_apply<1>, dim3(c->nred), dim3(TX, TY), 0, c->stream, z, pin, pout, q,
                           (const double*)c->a, c->nx, c->ny, c->sx * c->sx, c->sy * c->sy, c->sc, c->hist,
                           (const double*)c->part, c->nred, c->part2);
    LAUNCH_OK();
}

template <typename T>
void pcg_update(tgms_ctx* c, const FusedUpdate& fu, T* gT) {
    const long long nv = (long long)c->nx * c->ny;
    const unsigned grid = (unsigned)((nv + 4 * NT - 1) / (4 * NT));
    hipLaunchKernelGGL((k_pcg_update<T>), dim3(std::max(grid, 1u)), dim3(TX, TY), 0, c->stream, fu, gT, c->nx, c->ny);
    LAUNCH_OK();
}
template void pcg_update<double>(tgms_ctx*, const FusedUpdate&, double*);
template void pcg_update<float>(tgms_ctx*, const FusedUpdate&, float*);

template <typename T>
void prolong_residual(tgms_ctx* c, const PreResidual<T>& pr, T* t, const double* sc) {
    // blocks of at most 64 vertices go in 2 x 2 groups (one tile of about a workgroup's size)
    const int g = c->bx * c->by <= 64 ? 2 : 1;
    const int ngx = (c->Nx + g - 1) / g, ngy = (c->Ny + g - 1) / g;
    const size_t lds = sizeof(double) * (size_t)(g * c->bx + 2) * (g * c->by + 2) +
                       sizeof(T) * (size_t)(g + 2) * (g + 2) * pr.mu;
    hipLaunchKernelGGL((k_prolong_residual<T>), dim3(ngx * ngy), dim3(TX, TY), lds, c->stream, pr, t, c->nx, c->ny,
                       c->bx, c->by, c->Nx, g, g, sc);
    LAUNCH_OK();
}
template void prolong_residual<double>(tgms_ctx*, const PreResidual<double>&, double*, const double*);
template void prolong_residual<float>(tgms_ctx*, const PreResidual<float>&, float*, const double*);

void finalize(tgms_ctx* c, bool first) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TX, TY), 0, c->stream, c->sc, c->hist, (const double*)c->part,
                       c->nred, first ? 1 : 0);
    LAUNCH_OK();
}

template <typename T>
static CoarseW<T> coarse_w(tgms_ctx* c) {
    CoarseW<T> C;
    C.W = sizeof(T) == 8 ? (const T*)c->W : (const T*)c->W32;
    C.mu = c->mu;
    C.unk = c->blk_unk;
    C.nunk = c->blk_nu;
    return C;
}

template <typename T>
static size_t gather_res_lds(tgms_ctx* c) {
    return sizeof(double) * (c->bx + 2) * (c->by + 2) + sizeof(T) * (size_t)c->bx * c->by;
}

void allow_fused_lds(tgms_ctx* c) {
    const size_t need = gather_res_lds<double>(c);
    if (need <= 65536) return;
    if ((long long)need > c->lds_max) throw TgmsError{TGMS_E_UNSUPPORTED, "coarse blocks too large for the LDS tiles"};
    auto set = [&](const void* f) {
        HIP_OK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
    };
    set((const void*)k_gather_res_restrict<double>);
    set((const void*)k_gather_res_restrict<float>);
}

template <typename T>
void gather_res_restrict(tgms_ctx* c, const T* w, const double* g, T* z, T* t, T* cy, const double* sc) {
    ProfScope ps(c, PK_RESTRICT);
    hipLaunchKernelGGL((k_gather_res_restrict<T>), dim3(c->nblk), dim3(TX, TY), gather_res_lds<T>(c), c->stream,
                       c->patch, w, slots<T>(c), ggeom(c), T(c->eta), g, (const double*)c->a, c->sx * c->sx,
                       c->sy * c->sy, z, t, coarse_w<T>(c), cy, sc);
    LAUNCH_OK();
}
template void gather_res_restrict<double>(tgms_ctx*, const double*, const double*, double*, double*, double*,
                                          const double*);
template void gather_res_restrict<float>(tgms_ctx*, const float*, const double*, float*, float*, float*,
                                         const double*);

template <typename T>
void gather_final(tgms_ctx* c, const T* w, const T* zin, double* zout, const double* g, const double* gold,
                  bool with_dots, bool first) {
    const double* sc = with_dots ? c->sc : nullptr;
    if (with_dots && c->rpt == 4)
        hipLaunchKernelGGL((k_gather_final<T, 4>), dim3(c->nred), dim3(TX, TY), 0, c->stream, c->patch, w,
                           slots<T>(c), ggeom(c), T(c->eta), zin, zout, c->sx, c->sy, g, gold, sc, c->part,
                           c->sc + SC_PENDING);
    else if (with_dots)
        hipLaunchKernelGGL((k_gather_final<T, 1>), dim3(c->nred), dim3(TX, TY), 0, c->stream, c->patch, w,
                           slots<T>(c), ggeom(c), T(c->eta), zin, zout, c->sx, c->sy, g, gold, sc, c->part,
                           c->sc + SC_PENDING);
    else
        hipLaunchKernelGGL((k_gather_final<T, 1>), dim3(tiles(c).x * tiles(c).y), dim3(TX, TY), 0, c->stream,
                           c->patch, w, slots<T>(c), ggeom(c), T(c->eta), zin, zout, c->sx, c->sy, g, gold, sc,
                           (double*)nullptr, (double*)nullptr);
    LAUNCH_OK();
    if (with_dots && first) finalize(c, true);
}
template void gather_final<double>(tgms_ctx*, const double*, const double*, double*, const double*, const double*,
                                   bool, bool);
template void gather_final<float>(tgms_ctx*, const float*, const float*, double*, const double*, const double*, bool,
                                  bool);

}  // namespace tgms
