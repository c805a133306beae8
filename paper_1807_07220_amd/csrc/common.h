// Internal definitions shared by the tgms HIP sources (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tgms.h"

#define TGMS_WAVE 64

// ---------------------------------------------------------------- errors
void tgms_set_error(const std::string& msg);

struct TgmsError {
    tgms_status code;
    std::string msg;
};

#define HIP_OK(expr)                                                                 \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            throw TgmsError{e_ == hipErrorOutOfMemory ? TGMS_E_NOMEM : TGMS_E_DEVICE, \
                            std::string(#expr) + ": " + hipGetErrorString(e_)};      \
    } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

// ---------------------------------------------------------------- wave helpers
__device__ inline double readlane(double v, int l) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ inline float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, TGMS_WAVE);
    return v;
}

// ---------------------------------------------------------------- geometry
// Vertex (i, j) is the lower-left corner of cell (i, j); vertex arrays are
// ny x nx with the i = 0 and j = 0 entries (boundary of D) held at zero.  The
// discrete curl maps a vertex function psi to normal velocities
//   x-face (i, j):  (psi(i, j+1) - psi(i, j)) * sx,   sx = 1/hy,
//   y-face (i, j): -(psi(i+1, j) - psi(i, j)) * sy,   sy = 1/hx,
// so every curl is divergence free with zero flux through dD.  The H(div)
// operator on that space is K = C^T A C, a 9-point vertex stencil whose
// coefficients come from the weights a_c = |c| kappa_c^{-1} of the four cells
// around the vertex (A00 = SW, A10 = SE, A01 = NW, A11 = NE).
struct Stencil9 {
    double c, e, w, n, s, ne, nw, se, sw;
};

__host__ __device__ inline Stencil9 stencil9(double A00, double A10, double A01, double A11, double sx2,
                                             double sy2) {
    const double s = sx2 + sy2;
    Stencil9 k;
    k.c = s * (A00 + A10 + A01 + A11) * (1.0 / 3.0);
    k.e = (A10 + A11) * (sx2 * (1.0 / 6.0) - sy2 * (1.0 / 3.0));
    k.w = (A00 + A01) * (sx2 * (1.0 / 6.0) - sy2 * (1.0 / 3.0));
    k.n = (A01 + A11) * (sy2 * (1.0 / 6.0) - sx2 * (1.0 / 3.0));
    k.s = (A00 + A10) * (sy2 * (1.0 / 6.0) - sx2 * (1.0 / 3.0));
    k.ne = -s * A11 * (1.0 / 6.0);
    k.nw = -s * A01 * (1.0 / 6.0);
    k.se = -s * A10 * (1.0 / 6.0);
    k.sw = -s * A00 * (1.0 / 6.0);
    return k;
}

// 9-point stencil K at (x, y) of an FP64 LDS tile with row pitch pw, with the four
// cell weights around the vertex already loaded
__device__ inline double stencil_at4(const double* __restrict__ P, int pw, int x, int y, const double (&A)[4],
                                     double sx2, double sy2) {
    const double A00 = A[0], A10 = A[1], A01 = A[2], A11 = A[3];
    const double s = sx2 + sy2;
    const double c6 = 1.0 / 6.0, c3 = 1.0 / 3.0;
    const double kx = sx2 * c6 - sy2 * c3, ky = sy2 * c6 - sx2 * c3;
    const double* r0 = P + (y - 1) * pw + x;
    const double* r1 = P + y * pw + x;
    const double* r2 = P + (y + 1) * pw + x;
    double r = s * c3 * (A00 + A10 + A01 + A11) * r1[0];
    r += kx * ((A10 + A11) * r1[1] + (A00 + A01) * r1[-1]);
    r += ky * ((A01 + A11) * r2[0] + (A00 + A10) * r0[0]);
    r -= s * c6 * (A11 * r2[1] + A01 * r2[-1] + A10 * r0[1] + A00 * r0[-1]);
    return r;
}

// g and the four cell weights of interior vertex v (zeros elsewhere): loaded before a
// tile barrier so that their latency overlaps the tile's
struct VertexData {
    double g, A[4];
};
__device__ inline VertexData vertex_data(const double* __restrict__ g, const double* __restrict__ a, long long v,
                                         int nx, bool interior) {
    VertexData d{0.0, {0.0, 0.0, 0.0, 0.0}};
    if (interior) {
        d.g = g[v];
        d.A[0] = a[v - nx - 1];
        d.A[1] = a[v - nx];
        d.A[2] = a[v - 1];
        d.A[3] = a[v];
    }
    return d;
}

// Rectangle of cells [i0, i1) x [j0, j1) with its band-factor location.
struct Rect {
    int i0, i1, j0, j1;
    long long off;   // offset of the factor (column band) in the pool, in elements
    long long voff;  // offset of the local vector (n entries) in a per-problem vector pool
};

// ---------------------------------------------------------------- context
struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Block cyclic reduction Cholesky of a banded SPD matrix (k_dense.hip): n unknowns in nb
// blocks of bs rows (the half-bandwidth is at most bs); per block the inverse of its
// Cholesky factor C and the off-diagonal factors Gm, Gp (bs x bs, row-major, FP64 and,
// for an FP32 preconditioner, FP32 copies); x: the padded right-hand side / solution
// (nb * bs), Y the forward pass's intermediate.
struct Bcr {
    int n = 0, bs = 0, nb = 0;
    double *D = nullptr, *Lc = nullptr, *C = nullptr, *Gm = nullptr, *Gp = nullptr, *Y = nullptr, *x = nullptr;
    // the products the FP64 solve applies (row-major blocks): Gp^T C, Gm^T C (forward),
    // C^T Gm, C^T Gp (backward) and C^T C = D^{-1}
    double *PGP = nullptr, *PGM = nullptr, *QGM = nullptr, *QGP = nullptr, *R = nullptr;
    // the FP32 solve's factors (two-step form): C, its transpose, Gm, Gp and theirs
    double *CT = nullptr, *GmT = nullptr, *GpT = nullptr;
    float *C32 = nullptr, *Gm32 = nullptr, *Gp32 = nullptr, *CT32 = nullptr, *GmT32 = nullptr, *GpT32 = nullptr;
    float *Y32 = nullptr, *x32 = nullptr;
    int* fail = nullptr;
    // truncated reduction: levels s < step only, then the explicit FP64 inverse
    // Minv of the remaining block tridiagonal system (blocks 0, step, 2 step, ...; nr of
    // them); step 0: reduced to block 0
    int step = 0, nr = 0;
    double* Minv = nullptr;
};

namespace tgms {
// Device memory through a per-device cache of freed blocks: setups of the same
// shape allocate the same sizes, and hipMalloc / hipFree of the large dense
// workspaces cost milliseconds each.  dev_alloc returns a block of at least
// `bytes` (its size in *got); dev_free takes it back (the caller has synchronised
// the work that used it).  The cache keeps at most a fixed total per device and
// is emptied when hipMalloc fails.
void* dev_alloc(size_t bytes, size_t* got);
void dev_free(void* p, size_t bytes);
}  // namespace tgms

namespace tgms3 {
struct Ctx3;
}

struct tgms_ctx {
    int dim = 2;
    tgms3::Ctx3* d3 = nullptr;  // the cube's solver (dim 3)
    // grid
    int nx, ny, bx, by, Nx, Ny, nblk, ne, nex, jmax;
    double hx, hy, sx, sy, H, eta, tol;
    int overlap, precision;
    hipStream_t stream = nullptr;       // the library's own stream (graph capture needs a real stream)
    hipStream_t user_stream = nullptr;  // the caller's stream: work starts after what is queued there
    hipEvent_t ev_enter = nullptr;
    int nfx, nfy, nf;  // full-face counts
    // cell data
    double* kinv = nullptr;  // kappa^{-1}
    double* a = nullptr;     // |c| kappa^{-1}
    // block (K_i) stream-function factors
    int blk_m, blk_n, blk_b;  // m = bx-1 columns, n = (bx-1)(by-1), b = bx
    double* blkL = nullptr;   // nblk * n * (b+1)
    double* blkS = nullptr;   // nblk * n
    // smoother patches (K_i^+)
    std::vector<Rect> patch_h;
    Rect* patch = nullptr;
    int pat_bmax = 0, pat_nmax = 0;
    int pat_m1 = 0, pat_m2 = 0;  // the row widths present among the patches (m1 >= m2)
    long long pat_fmax = 0;   // largest patch factor (elements)
    int pat_hmax = 0;         // most vertex rows of a patch
    int lds_max = 65536;      // device limit on LDS per workgroup (bytes)
    long long pat_pool = 0, pat_vpool = 0;
    double* patL = nullptr;
    float* patL32 = nullptr;
    double* patW = nullptr;  // per-patch local solution (vpool)
    float* patW32 = nullptr;
    bool slots = false;        // patch solutions go to four slots per vertex (blocks >= 2 * overlap)
    double* patW4 = nullptr;   // 4 * nx * ny
    float* patW4_32 = nullptr;
    // snapshots and Gram
    int nfk, ncol;            // faces per block (full, incl. block boundary), snapshot columns per block
    double* Psi = nullptr;    // nblk * ncol * nfk  (column major per block)
    double* APsi = nullptr;
    double* G = nullptr;      // nblk * ncol * ncol
    // spectral results per coarse face
    double* eigs = nullptr;   // ne * jmax (ascending lambda)
    int* counts = nullptr;    // ne
    double* Y = nullptr;      // ne * jmax * jmax
    std::vector<int> counts_h;
    // coarse SPD system
    int ncs = 0;              // unknowns
    int mu = 0;               // max unknowns touching one block
    int* blk_unk = nullptr;   // nblk * mu (ids, -1 pad)
    int* blk_nu = nullptr;    // nblk
    double* blk_T = nullptr;  // nblk * ncol * mu : snapshot-column coefficients of each unknown on K
    double* W = nullptr;      // nblk * (bx*by) * mu  stream functions on owned vertices
    float* W32 = nullptr;
    int* unk_ptr = nullptr;   // ncs+1 CSR of (block, slot) touching each unknown
    int* unk_ent = nullptr;
    double* Ac = nullptr;     // ncs * ncs (dense, then its inverse)
    double* Acf = nullptr;    // FP64 with small ncs: the explicit inverse (ncs * ncs, symmetric)
    float* Ac32 = nullptr;
    double* cy = nullptr;     // nblk * mu restricted values
    float* cy32 = nullptr;
    double* cvec = nullptr;   // ncs
    double* cvec2 = nullptr;
    float* cvec32 = nullptr;
    float* cvec2_32 = nullptr;
    // coarse space of the two-grid preconditioner: 0 adaptive GMsFEM (section 4), 1 MsFEM
    // (one basis per face, the sum of its snapshots), 2 coarse RT0 (the paper's comparators)
    int coarse_space = 0;
    int* force = nullptr;     // ne imposed basis counts (device), or null
    int* eig_bad = nullptr;   // faces whose Jacobi solve hit its sweep limit (device counter)
    int eig_unconverged = 0;
    double* YQ = nullptr;     // ne * jmax * jmax kept modes times recombination (the basis; saved by tgms_save)
    double* AH0c = nullptr;   // nblk * 6 coarse RT0 Grams for the RT0 coarse space (main stream)
    int cband = 0;            // half-bandwidth of the coarse SPD matrix in its numbering
    int coarse_factor = 0;    // tgms_options.coarse_factor
    int msteps = 1;           // pre- and post-smoothing steps of the two-grid cycle
    int additive = 0;         // 1: two-level additive Schwarz (no residual recomputed)
    Bcr cb;                   // its cyclic-reduction Cholesky (cb.nb == 0: the dense inverse is used)
    Bcr kb;                   // the same for the coarse RT0 stiffness of the preprocessing
    // coarse RT0 (preprocessing)
    int nv = 0;               // interior coarse vertices
    double* AH0 = nullptr;    // nblk * 6 : WW, WE, EE, SS, SN, NN
    double* KH = nullptr;     // nv * nv inverse of the coarse vertex stiffness
    double* cflux = nullptr;  // coarse velocities: x part Ny*(Nx+1), y part (Ny+1)*Nx
    double* svec = nullptr;   // nv
    double* svec2 = nullptr;
    // pressure
    double* Qx = nullptr;     // nx*nx DCT-II (orthonormal)
    double* Qy = nullptr;
    double* lamx = nullptr;
    double* lamy = nullptr;
    // solve workspaces (vertex arrays nx*ny, face arrays nf)
    double *vx = nullptr, *vg = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr, *vt = nullptr,
           *vt2 = nullptr, *vgold = nullptr;
    float *fg = nullptr, *fz = nullptr, *ft = nullptr, *ft2 = nullptr;
    double *fbar = nullptr, *fu = nullptr, *fF = nullptr, *cellw = nullptr, *cellw2 = nullptr;
    double* blkbuf = nullptr; // 2 * nblk
    double* red_h = nullptr;  // pinned host
    double* sc = nullptr;     // device PCG scalars (SC_* below)
    double* hist = nullptr;   // device alpha/beta history
    int hist_cap = 0;
    double* part = nullptr;   // per-workgroup partial sums of the final gather (3 x NRED)
    double* part2 = nullptr;  // per-workgroup partial sums of p.q (NRED)
    double* vt3 = nullptr;    // z1 after the coarse correction (FP64 preconditioner)
    double* vg2 = nullptr;    // second residual buffer (the PCG update reads one and writes the other)
    int nred = 256;           // workgroups of the reducing PCG kernels (autotuned)
    int rpt = 1;              // vertex rows per thread in the tiled PCG kernels (1 or 4; autotuned)
    int smooth_staged = -1;   // smoother: 1 forward blocks kept in LDS for the backward chains, 0 staged twice
    int snap_cols = 1;        // snapshots: 1 one lane per column where supported, 0 one wave per block
    int tuned = 0;            // 0 defaults, 1 timed at setup, 2 taken from the tuning cache
    double* vp1 = nullptr;    // second search-direction buffer (p alternates between vp and vp1)
    hipGraphExec_t iter_graph = nullptr;  // two captured PCG iterations
    bool graph_failed = false;
    int last_graph = 0;  // how the last solve ran its iterations: 0 direct launches, 1 graph
    // per-kernel event timing (tgms_profile)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    // (kernel, iteration tag, start, stop); tag -1: outside a PCG iteration
    struct ProfRec {
        int id, iter;
        hipEvent_t e1, e2;
    };
    std::vector<ProfRec> prof_rec;
    int prof_iter = -1;  // tag of the launches being recorded
    double prof_acc_ms[8] = {0};
    int prof_acc_n[8] = {0};
    // diagnostics
    std::vector<double> alphas, betas;
    double t_setup_ms = 0, t_snap_ms = 0, t_eig_ms = 0, t_coarse_ms = 0, t_smoother_ms = 0;
    std::vector<DeviceBuf> owned;
    Rect* blk_rects = nullptr;
    double* Td = nullptr;      // coarse basis combination matrices (kept for mobility updates)
    double* clH = nullptr;     // H_K = T_K^T G_K T_K per block (coarse assembly)
    int* zcd = nullptr;
    // warm-started local eigensolves (tgms_options.warm_start)
    int warm = 0;               // 0 dense Jacobi, 1 DCT-II start, 2 network start
    double rq_tol = 1e-6;       // relative Ritz residual for acceptance
    int warm_maxit = 8;         // subspace iterations before the dense fallback
    int* wstat = nullptr;       // per face: accepting iteration, or -1 (fallback)
    std::vector<int> wstat_h;
    int warm_accepted = 0, warm_iters = 0;
    double t_cnn_ms = 0;
    bool mobility_updated = false;
    int* scratch_int = nullptr;
    int* alloc_scratch_int() {
        if (!scratch_int) scratch_int = alloc<int>(4);
        HIP_OK(hipMemsetAsync(scratch_int, 0, 4 * sizeof(int), stream));
        return scratch_int;
    }

    template <typename T>
    T* alloc(size_t n) {
        DeviceBuf b;
        b.p = tgms::dev_alloc(n * sizeof(T) + 256, &b.bytes);
        HIP_OK(hipMemsetAsync(b.p, 0, b.bytes, stream));
        owned.push_back(b);
        return reinterpret_cast<T*>(b.p);
    }
};

// ---------------------------------------------------------------- launchers
// device PCG scalars: rho, p.q, alpha, beta, |z|^2, |z|^2/|z0|^2, |z0|^2, breakdown flag,
// iteration count, done flag, rtol^2, maxit, flexible (1) or Fletcher-Reeves (0), the
// rho of the latest finalisation (moved into rho by the next update), and the flag
// of gather partials not finalised yet
enum { SC_RHO = 0, SC_PQ, SC_ALPHA, SC_BETA, SC_ZN2, SC_REL2, SC_Z02, SC_FLAG, SC_IT, SC_DONE, SC_RTOL2, SC_MAXIT,
       SC_FLEX, SC_RHO_NEW, SC_PENDING, SC_COUNT };

// sum of cy[ent[k]] for k in [k0, k1), added in order; the index and value loads of
// four terms are issued together (two memory round trips per four terms, not eight)
template <typename T>
__device__ inline T gather_sum(const int* __restrict__ ent, const T* __restrict__ cy, int k0, int k1) {
    T v = T(0);
    for (int k = k0; k < k1; k += 4) {
        int e[4];
        T c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = k + q < k1 ? ent[k + q] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = e[q] >= 0 ? cy[e[q]] : T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (k + q < k1) v += c[q];
    }
    return v;
}

// inputs of k_prolong_residual: z1p = z1 + W c and the residual g - K z1p
template <typename T>
struct PreResidual {
    const T* z1 = nullptr;
    T* z1p = nullptr;
    const T* c = nullptr;     // coarse solution
    const T* W = nullptr;     // [block][owned vertex][slot]
    int mu = 0;
    const int* unk = nullptr;
    const int* nunk = nullptr;
    const double* g = nullptr;  // FP64 right-hand side of the cycle
    const double* a = nullptr;  // cell weights
    double sx2 = 0, sy2 = 0;
};

// inputs of k_pcg_update: the p.q partials, the PCG scalars and the vectors
struct FusedUpdate {
    const double* part;
    int nred;
    double* sc;
    double* hist;
    const double* p;
    const double* q;
    double* x;
    const double* gin;
    double* gout;
};

namespace tgms {
enum ProfKernel { PK_SMOOTH = 0, PK_APPLYK = 1, PK_RESTRICT = 2, PK_PROLONG = 3, PK_COUNT = 4 };
// record an event pair around one launch when profiling is on
struct ProfScope {
    tgms_ctx* c;
    int id;
    hipEvent_t e1 = nullptr;
    ProfScope(tgms_ctx* ctx, int kid);
    ~ProfScope();
};
void enter(tgms_ctx* c);
hipEvent_t take_event(tgms_ctx* c);  // from the profiling event pool
// grid / vector kernels (k_grid.hip)
void cell_weights(tgms_ctx* c, const double* kappa, int* bad);
void mobility_weights(tgms_ctx* c, const double* lambda, int* bad, double* out);  // out = |c| kappa^{-1} / lambda
void weights_from_kinv(tgms_ctx* c);  // a = |c| kinv (a restored context)
void faces_A(tgms_ctx* c, const double* u, double* out);                    // A u on interior faces
void faces_A_probe(tgms_ctx* c, const double* u, double* out);              // same, boundary inputs ignored
void curlT_A_faces(tgms_ctx* c, const double* u, double* g, double scale);  // g = scale * C^T A u
void curl_add(tgms_ctx* c, const double* psi, const double* base, double* u); // u = base + C psi
void curlT(tgms_ctx* c, const double* u, double* g);
void copy(tgms_ctx* c, long long n, const double* x, double* y);
void axpy(tgms_ctx* c, long long n, double a, const double* x, double* y);        // y += a x
void cast_d2f(tgms_ctx* c, long long n, const double* x, float* y);
void cast_f2d(tgms_ctx* c, long long n, const float* x, double* y);
void zero(tgms_ctx* c, void* p, size_t bytes);
// band factors and smoother (k_band.hip)
void factor_blocks(tgms_ctx* c, int* fail = nullptr);  // fail: checked later by the caller (null: here)
void factor_patches(tgms_ctx* c);
// the same without waiting: a failed factorisation sets *fail (zero on entry);
// max_groups > 0 bounds the workgroups (each then factors several patches in turn)
void factor_patches_launch(tgms_ctx* c, int* fail, int max_groups);
template <typename T>
void smooth_patches(tgms_ctx* c, const T* g, const double* sc);  // local solves of S g into the patch pool
// fused PCG / two-grid kernels (k_pcg.hip); sc: skip when the done flag is set (may be null)
unsigned pcg_tiles(tgms_ctx* c);
int nred_max();
void autotune(tgms_ctx* c, const char* cache_path);  // picks nred, smoother staging (k_tune.hip)
void twogrid_probe(tgms_ctx* c);  // one two-grid application on the context's zeroed vectors (timing)
void dir_apply(tgms_ctx* c, const double* z, const double* pin, double* pout, double* q);
void vertex_residual(tgms_ctx* c, const double* g, const double* z, double* t);  // t = g - K z (FP64)
template <typename T>
void pcg_update(tgms_ctx* c, const FusedUpdate& fu, T* gT);  // alpha, g = gin - alpha q (and T(g) in gT), x += alpha p
template <typename T>
void prolong_residual(tgms_ctx* c, const PreResidual<T>& pr, T* t, const double* sc);  // z1p = z1 + W c, t = g - K z1p
void finalize(tgms_ctx* c, bool first);  // scalars from pending gather partials (first: rho_0, |z_0|^2)
void allow_fused_lds(tgms_ctx* c);      // LDS limit of the per-block fused kernels (large blocks)
template <typename T>
void gather_res_restrict(tgms_ctx* c, const T* w, const double* g, T* z, T* t, T* cy, const double* sc);
template <typename T>
void gather_final(tgms_ctx* c, const T* w, const T* zin, double* zout, const double* g, const double* gold,
                  bool with_dots, bool first);
// setup (k_setup.hip)
void snapshots(tgms_ctx* c, double* scratch, long long scratch_per_block);  // scratch: a workspace free during the call
void gram(tgms_ctx* c);
inline bool gram_uses_mfma(const tgms_ctx* c) { return c->ncol == 64 || c->ncol == 32; }  // blocks of 16 or 8 cells
void pencil_eig_q(tgms_ctx* c, double* YQ, const float* Y0, float* Vtop);  // YQ: kept modes times recombination
void fill_td(tgms_ctx* c, const int* meta, const double* YQ, double* Td);     // coarse basis combinations
// warm-start network (k_cnn.hip)
int cnn_nparams();
int cnn_kout();
bool cnn_shape_ok(int H, int W);
size_t cnn_train_workspace(long long n, int H, int W);
void cnn_forward(hipStream_t st, const float* prm, const float* X, long long n, int H, int W, float* Y, float* act);
double cnn_train_step(hipStream_t st, float* prm, float* m, float* v, int t, float lr, const float* X, const float* V,
                      long long n, int H, int W, int k, float* work);
void cnn_windows(tgms_ctx* c, float* X);
// inference only, BF16 matrix cores with FP32 accumulation (no saved activations)
void cnn_infer_bf16(hipStream_t st, const float* prm, const float* X, long long n, int H, int W, float* Y);
void coarse_local_run(tgms_ctx* c, const double* Tm, const int* zc);
void coarse_rt0_blocks(tgms_ctx* c, double* AH0);                    // per-block coarse RT0 Grams
void rt0_stiffness(tgms_ctx* c, const double* AH0, double* K);       // coarse vertex stiffness (dense)
void rt0_coarse_W(tgms_ctx* c);  // coarse space = coarse RT0: bilinear vertex stream functions in W
void pencil_probe(tgms_ctx* c, double* D, double* S);  // each face's a-form diagonal and s-form
// coarse apply (k_setup.hip)
template <typename T>
void coarse_apply(tgms_ctx* c, const T* g, T* z, bool accumulate, const double* sc);
template <typename T>
T* coarse_cy(tgms_ctx* c);  // the block restriction buffer of the coarse correction
template <typename T>
const T* coarse_solve(tgms_ctx* c, const double* sc);  // accumulate the restrictions, apply the coarse inverse
// dense (k_dense.hip)
// A -> tril(L^{-1}) + triu(L^{-T}, 1) in place; full (optional): the explicit inverse
void dense_spd_inverse(tgms_ctx* c, double* A, int n, double* full = nullptr);
struct DenseInvWork {
    double* Dinv = nullptr;
    int* fail = nullptr;
    double* X = nullptr;
    double* Tm = nullptr;
    size_t bytes[4] = {0, 0, 0, 0};  // block sizes of Dinv, fail, X, Tm
};
// an inverse queued on a stream without waiting (dense_spd_inverse_begin / _end)
struct DenseInvAsync {
    DenseInvWork w;
    hipStream_t stream = nullptr;
    DenseInvAsync() = default;
    DenseInvAsync(const DenseInvAsync&) = delete;
    DenseInvAsync& operator=(const DenseInvAsync&) = delete;
    ~DenseInvAsync();
    void release();
};
void dense_spd_inverse_begin(tgms_ctx* c, double* A, int n, DenseInvAsync& h);
void dense_spd_inverse_end(DenseInvAsync& h);
int bcr_max_block(const tgms_ctx* c);  // largest block the factor kernel holds in LDS
// factorise the banded SPD A (dense n x n, row-major; zero beyond half-bandwidth bs)
// truncate: stop the reduction where the remaining system has at most symv_acc_max()
// unknowns and invert that explicitly in FP64 (applied in FP64 by both solves;
// synchronises)
void bcr_factor(tgms_ctx* c, const double* A, int n, int bs, Bcr& F, bool fp32, bool truncate = false);
bool bcr_failed(tgms_ctx* c, const Bcr& F);  // a non-positive pivot (synchronises)
template <typename T>
void bcr_solve(tgms_ctx* c, const Bcr& F, T* x, const double* sc);  // x (nb * bs) <- A^{-1} x
template <typename T>
void symv(tgms_ctx* c, const T* A, int n, const T* x, T* y, const double* sc);
template <typename T>
bool symv_acc(tgms_ctx* c, const T* B, int n, const int* ptr, const int* ent, const T* cy, T* y, const double* sc);
// the same with the explicit inverse F (one launch); false when n > symv_acc_max() or F is null
bool symv_full_acc(tgms_ctx* c, const double* F, int n, const int* ptr, const int* ent, const double* cy, double* y,
                   const double* sc);
int symv_acc_max();
void gemm(tgms_ctx* c, int transA, int transB, int M, int N, int K, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc);
// batched GEMM: matrix z of A (and B, C) at A + (z / nin) * outer + (z % nin) * inner
struct Strided {
    long long outer = 0, inner = 0;
    int nin = 1;
};
void gemm_batched(tgms_ctx* c, int transA, int transB, int M, int N, int K, double alpha, const double* A, int lda,
                  Strided sa, const double* B, int ldb, Strided sb, double beta, double* C, int ldc, Strided sc,
                  long long batch, bool lower_only = false);
// each of batch consecutive n x n SPD matrices -> its explicit inverse, in place
void dense_spd_inverse_batched(tgms_ctx* c, double* A, int n, long long batch);
// preprocessing and pressure (k_pre.hip)
void preprocess(tgms_ctx* c, const double* F, const double* g_bnd, double* vbar, double* Fp);
void pressure(tgms_ctx* c, const double* u, double* p);
void dct_matrix(tgms_ctx* c, int n, double* Q, double* lam);  // orthonormal DCT-II and Neumann eigenvalues
// two-phase transport (k_transport.hip)
struct TransportResult {
    long long sweeps = 0;   // outer (tile) launches
    double residual = 0.0;  // max_i |R_i| at return
    bool converged = false;
};
void total_mobility(hipStream_t st, const double* s, long long n, double mu_w, double mu_o, double* lam);
// nz <= 1: the square (16 x 16 tiles); nz > 1: the cube (8 x 8 x 4 tiles)
TransportResult transport_step(hipStream_t st, int nx, int ny, int nz, const double* u, const double* q, double* s,
                               double phi, double dt, double mu_w, double mu_o, double tol, int max_outer);
}  // namespace tgms
