/*
 * tgms: two-grid preconditioned solver with an adaptive GMsFEM coarse space
 * for mixed (RT0 velocity, P0 pressure) Darcy flow on a uniform Cartesian
 * grid of the unit square, on one AMD MI355X (gfx950).
 *
 * Problem (paper section 2, eq. orgional_equation): find v, p with
 *     kappa^{-1} v + grad p = 0,   div v = f   in D = (0,1)^2,
 *     v . n = g on dD  (g = 0 in the paper),
 * discretised by RT0 x P0 (eqs. matrixform, fine_system).  Algorithm
 * (section 5): preprocessing (section 3) gives vbar with B vbar = F; PCG on
 * the divergence-free remainder with a two-grid preconditioner made of an
 * overlapping-patch smoother (eq. smooth) and a coarse correction through
 * the adaptive spectral space (section 4, eqs. snapshot_eqn, spectral_eqn;
 * eq. coarsepre).
 *
 * Conventions shared by every entry point
 *   cells      (i, j), 0 <= i < nx, 0 <= j < ny, index j*nx + i (x fastest);
 *   faces      "full" numbering including the boundary of D:
 *              x-faces (at x = i/nx, row j, 0 <= i <= nx): index j*(nx+1) + i,
 *              y-faces (at y = j/ny, column i, 0 <= j <= ny): index
 *              (nx+1)*ny + j*nx + i;  nfaces = (nx+1)*ny + nx*(ny+1);
 *              a face value is the normal velocity along +x or +y;
 *   sources    cell-integrated, F_c = int_c f;
 *   pressure   physical sign (A v = B^T p, i.e. kappa^{-1} v = -grad p),
 *              zero mean over the cells.
 *
 * Memory: every array argument documented "device" is a pointer to GPU
 * memory owned by the caller (e.g. a PyTorch tensor); the library reads or
 * writes it on the context's stream and keeps no reference after the call
 * returns.  The context owns all of its own workspaces.
 *
 * Errors: every call returns a tgms_status; on failure tgms_last_error()
 * returns a message (thread-local, valid until the next call on that thread).
 * No call aborts the process.
 */
#ifndef TGMS_H
#define TGMS_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tgms_ctx tgms_ctx;

typedef enum {
    TGMS_OK = 0,
    TGMS_E_INVAL = -1,        /* bad argument: sizes, non-positive or non-finite permeability */
    TGMS_E_INCOMPAT = -2,     /* sum of sources differs from the boundary outflow */
    TGMS_E_NOTCONV = -3,      /* PCG reached maxit; the last iterate is returned */
    TGMS_E_BREAKDOWN = -4,    /* PCG breakdown (p^T A p <= 0 or not finite) */
    TGMS_E_DEVICE = -5,       /* HIP runtime error */
    TGMS_E_NOMEM = -6,        /* device allocation failed */
    TGMS_E_UNSUPPORTED = -7   /* a size the kernels do not handle (see tgms_setup) */
} tgms_status;

typedef struct {
    int dim;          /* 2 (the unit square) or 3 (the unit cube, see below) */
    int nx, ny, nz;   /* fine cells per axis (nz: 0 or 1 when dim = 2) */
    int bx, by, bz;   /* coarse block size in fine cells; nx % bx == 0, ny % by == 0 (bz: 0 or 1
                         when dim = 2, nz % bz == 0 when dim = 3) */
} tgms_grid;

typedef struct {
    double eta;        /* smoother weight, eq. smooth (paper: 0.2) */
    int overlap;       /* K_i^+ = K_i enlarged by this many fine cells, clipped to D (paper: 2);
                          at least 1: without oversampling the smoother misses the fluxes
                          across block edges and the preconditioner is singular */
    int precision;     /* 0: FP64 preconditioner and PCG;
                          1: FP32 preconditioner (smoother factors, coarse basis, coarse
                             inverse, inner operator applies) inside a flexible FP64 PCG */
    double s_scale;    /* H in the 1/H prefactor of the s-form (eq. spectral_eqn).  Default 1
                          (a unit prefactor): with the printed 1/H and H the block side, a
                          homogeneous medium keeps about seven modes per face at the
                          tolerance 10 of section 6, whose tables report one (the coarse RT0
                          dimension); the unit prefactor reproduces them.  <= 0 selects the
                          printed |K|^(1/2), the coarse block side */
    void* stream;      /* hipStream_t to run on; NULL = the default stream */
    int graphs;        /* 1: PCG iterations replayed from a captured HIP graph (falls back to
                          direct launches if capture fails); 0: every kernel launched directly */
    int autotune;      /* 1: time the candidate launch configurations (reduction grid, smoother
                          staging) at setup, once per shape and device; 0: fixed defaults */
    const char* tune_cache;  /* file keeping tuned configurations across processes (read and
                                rewritten by setup); NULL: keep them in this process only */
    int warm_start;    /* local spectral problems (section 4.2):
                          0: dense cyclic Jacobi on every face's pencil;
                          1: Rayleigh-Ritz subspace iteration from the DCT-II basis (k = 8
                             vectors, at most 8 iterations), accepted when the selected modes
                             are certified (inertia count of 1/tol - T, Ritz residuals
                             <= rq_tol), else the dense solve for that face;
                          2: as 1, the initial vectors from the warm-start network
                             (tgms_cnn_forward) on the face's permeability; needs square
                             blocks of at most 16 x 16 cells and cnn_weights */
    const float* cnn_weights;  /* device, tgms_cnn_nparams() floats (warm_start 2; read during
                                  setup only) */
    double rq_tol;     /* relative Ritz residual |T u - theta u| / theta for acceptance (1e-6) */
    int smoother_staging;  /* -1: chosen by the autotuner (without it: 0); 0: each chain step's
                              factor blocks are staged in LDS by the forward chains and again by
                              the backward chains; 1: the forward chains' blocks are kept in LDS
                              for the backward chains (falls back to 0 where they do not fit) */
    int rows_per_thread;   /* vertex rows per thread in the tiled PCG kernels: 0 chosen by the
                              autotuner (without it: 1); 1 or 4 */
    const int* force_counts;  /* host, n_coarse_faces ints (face order of tgms_get_counts), or NULL:
                                 impose the basis count l_i of every face (1 <= l_i <= J_i, the
                                 face's fine faces) instead of #{lambda < eig_tol}; the kept modes
                                 are still the l_i smallest eigenvalues' (section 4.2).  For
                                 comparisons with another eigensolver where an eigenvalue lies
                                 at the tolerance.  Needs warm_start 0 and coarse_space 0; read
                                 during tgms_setup only. */
    int coarse_space;  /* coarse space of the two-grid preconditioner (section 5):
                          0: the adaptive GMsFEM space (section 4; the paper's method);
                          1: MsFEM, one basis per face, the sum of its snapshots (eq. msfem);
                          2: the coarse RT0 space (the fine interpolant of the lowest-order
                             Raviart-Thomas functions on the blocks).  1 and 2 are the
                             comparators of section 6; they need warm_start 0. */
    int coarse_factor;  /* factorisation of the coarse SPD systems (the coarse space's and the
                           preprocessing's coarse RT0 one): 0 chosen by size (the dense
                           Cholesky inverse for small FP64 systems, else the cyclic-reduction
                           Cholesky of the band where it fits); 1 always the dense inverse;
                           2 cyclic reduction wherever the band fits */
    int smooth_steps;  /* m1 = m2: smoothing steps before and after the coarse correction (section 5,
                          with the residual recomputed after each; the paper uses 1), 1..16 */
    int additive;      /* 1: the two-level additive Schwarz form z = S r + P r instead of the
                          multiplicative two-grid cycle (section 5 contrasts the two: the
                          residual is not recomputed between the parts); 0 (default): the cycle */
} tgms_options;

typedef struct {
    int n_coarse_faces;   /* N_e: interior coarse faces (one local spectral problem each) */
    int n_blocks;         /* coarse blocks */
    int dim;              /* paper's "Dim": sum of basis counts + n_blocks + 1 */
    int n_coarse_spd;     /* unknowns of the SPD coarse system actually factorised */
    double t_setup_ms;    /* device time of tgms_setup (all phases) */
    double t_snap_ms, t_eig_ms, t_coarse_ms, t_smoother_ms;  /* setup phases */
    int lds_max;          /* LDS bytes per workgroup the device allows (picks the smoother kernel) */
    int pcg_graph;        /* last solve: 0 kernels launched directly, 1 iterations replayed from a
                             HIP graph */
    int tuned;            /* launch configuration: 0 defaults, 1 timed at this setup, 2 from the cache */
    int nred;             /* workgroups of the reducing PCG kernels */
    int smooth_staged;    /* smoother: 1 forward blocks kept in LDS, 0 staged twice */
    int warm_accepted;    /* warm start: faces whose modes were certified without the dense solve */
    int warm_iters;       /* warm start: subspace iterations summed over the accepted faces */
    double t_cnn_ms;      /* warm start 2: network inputs and forward pass (inside t_eig_ms) */
    int rows_per_thread;  /* vertex rows per thread in the tiled PCG kernels (1 or 4) */
    int eig_unconverged;  /* faces whose dense eigensolve (cyclic Jacobi) was still rotating at its
                             sweep limit (60 sweeps); their eigenpairs are the last iterate */
    int coarse_space;     /* as in tgms_options */
    int nx, ny, bx, by;   /* the grid (also of a context restored by tgms_load) */
    int precision;        /* as in tgms_options */
    int coarse_block;     /* block of the cyclic-reduction Cholesky of the coarse system (its
                             half-bandwidth), 0 when the dense inverse is used */
    int rt0_block;        /* the same for the preprocessing's coarse RT0 system */
} tgms_info_t;

/* Paper defaults: eta 0.2, overlap 2, FP64, s_scale = 1 (unit s-form prefactor), default stream,
 * graph replay on, autotuning on without a cache file, dense local eigensolves
 * (warm_start 0, rq_tol 1e-6), smoother staging chosen by the autotuner, no imposed
 * counts, the adaptive coarse space. */
void tgms_default_options(tgms_options* opt);

/*
 * Setup (section 5, Step 2, and the source-independent part of Step 1):
 * snapshot space and local spectral problems for every interior coarse face
 * (section 4), adaptive selection l_i = max(1, #{lambda < eig_tol}), the
 * coarse operator and its FP64 Cholesky factorisation, the smoother patch
 * factorisations (K_i^+), and the coarse RT0 operator used by preprocessing.
 *   kappa  device, nx*ny doubles, permeability per cell (> 0, finite).
 * Returns TGMS_E_INVAL for bad sizes, tolerance, eta, overlap or permeability;
 * TGMS_E_UNSUPPORTED for blocks smaller than 3 x 3 cells, fewer than 2 x 2
 * blocks, an overlap not smaller than the block, blocks wider than 64 cells or
 * smoother patches (block + 2 overlap, clipped to D) wider than 33 cells.
 * On success *out owns all device workspaces until tgms_destroy.
 *
 * The unit cube (dim = 3; the paper's models 2 and 3): cells (i, j, k) index
 * (k ny + j) nx + i; faces x ((k ny + j)(nx + 1) + i), then y ((k (ny + 1) + j) nx
 * + i), then z ((k ny + j) nx + i); kappa and F have nx ny nz entries.  Local
 * problems are solved through their pressure Schur complement (line-tridiagonal
 * A^{-1}, a dense inverse per block and per patch), the coarse problem through a
 * dense solution operator; PCG runs on the face vectors.  Supported: FP64
 * (precision 0), no warm start, one pre- and one post-smoothing (smooth_steps 1,
 * additive 0), no-flow boundary (g_bnd NULL), at least 2 blocks per axis, an
 * overlap of at most the block size, patches of at most 32 cells per axis, at most
 * 64 fine faces per coarse face; coarse_space 0, 1 and 2.  tgms_solve,
 * tgms_update_mobility, tgms_impes, tgms_info, tgms_get_counts, tgms_get_eigs,
 * tgms_last_cond, tgms_apply_A, tgms_preprocess, tgms_apply_precond and
 * tgms_time_smoother (the patch solves) accept such a context; the other calls
 * that take a context return TGMS_E_UNSUPPORTED for it.
 * Coarse faces are ordered x, y, z, each by (K, J, I) of the block on the face's
 * high side; the fine faces of a coarse face with the lower tangential axis fastest.
 */
tgms_status tgms_setup(const tgms_grid* grid, const double* kappa, double eig_tol,
                       const tgms_options* opt, tgms_ctx** out);

/*
 * Solve (section 5, Steps 1, 3, 4): preprocessing, PCG to
 * ||z_k||_2 <= rtol ||z_0||_2 (z = preconditioned residual), v = vbar + vtilde,
 * then the pressure by least squares from A v = B^T p (zero mean).
 *   F      device, nx*ny doubles, cell-integrated source;
 *   g_bnd  device, nfaces doubles (full face numbering), only the boundary
 *          entries are read; NULL means no-flow (the paper's case);
 *   u      device, nfaces doubles, output velocity (boundary entries = g);
 *   p      device, nx*ny doubles, output pressure (may be NULL);
 *   iters, relres  host, outputs (may be NULL).
 * TGMS_E_INCOMPAT if |sum F - boundary outflow| > 1e-12 (sum |F| + sum |g| |e|);
 * TGMS_E_NOTCONV returns the last iterate with *iters = maxit.
 */
tgms_status tgms_solve(tgms_ctx* ctx, const double* F, const double* g_bnd, double rtol,
                       int maxit, double* u, double* p, int* iters, double* relres);

/*
 * The solve of tgms_solve for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid allocation): same arguments, same kernels and,
 * bitwise, the same results as tgms_solve.  The PCG's scalars, the partial sums of
 * its reductions and its alpha / beta history live in a fixed array in device memory
 * of the library (512 KB per device, held until the process ends) instead of the
 * context's buffers; the iterations are launched directly (no HIP graph is
 * instantiated), no history is read back (tgms_last_cond then reports 1), and the
 * call allocates nothing.  Limit: maxit <= 32000 or so (the exact bound is in the
 * message of TGMS_E_INVAL).  Every call on one device shares that device's array:
 * calls that overlap in time on one device (other threads, other contexts) race.
 */
tgms_status tgms_solve_noalloc(tgms_ctx* ctx, const double* F, const double* g_bnd, double rtol, int maxit,
                               double* u, double* p, int* iters, double* relres);

/*
 * Mobility update with the coarse space kept (section 6.2: the multiscale basis
 * of the initial permeability is reused while the total mobility changes).  The
 * operator becomes A(lambda), built from (lambda kappa)^{-1}; the block factors,
 * the coarse operator over the kept basis (Gram matrices of the kept snapshots,
 * its Cholesky inverse), the coarse RT0 operator and the smoother patch factors
 * are rebuilt.  The eigenvalues, basis counts and basis functions are unchanged.
 *   lambda  device, nx*ny doubles, total mobility per cell (> 0, finite).
 * TGMS_E_INVAL for a non-positive or non-finite mobility (the context then holds
 * a partially rebuilt operator: call again with a valid field before solving).
 */
tgms_status tgms_update_mobility(tgms_ctx* ctx, const double* lambda);

/* Sizes and timings of the setup. */
tgms_status tgms_info(const tgms_ctx* ctx, tgms_info_t* info);

/*
 * Checkpoint of the setup (section 6.2 keeps the coarse space of the initial
 * permeability over all pressure solves): tgms_save writes the permeability the
 * setup saw (kappa^{-1} per cell), the current cell weights (after mobility
 * updates), the basis counts, the eigenvalues and each face's kept modes (snapshot
 * coefficients) to `path` (binary, little-endian; overwritten).  tgms_load
 * rebuilds a context from it: the snapshots, coarse operator, factorisations and
 * smoother are formed again from the saved weights, the eigenproblems are not
 * solved again.  eta, overlap, precision, s_scale, coarse_space and the eigenvalue
 * tolerance come from the file; opt (NULL = defaults) gives the stream, graphs,
 * autotuning, tuning cache, smoother staging and rows per thread.  With the same
 * launch configuration (autotune 0, or one tuning cache) a loaded context's solves
 * are bitwise those of the saved one.  TGMS_E_INVAL when the file cannot be opened,
 * read or written, is not a saved context of this version, or holds inconsistent
 * sizes, counts or weights; *out is then NULL.
 */
tgms_status tgms_save(const tgms_ctx* ctx, const char* path);
tgms_status tgms_load(const char* path, const tgms_options* opt, tgms_ctx** out);

/* The pencil of every coarse face's local spectral problem (section 4.2, eqs.
 * spectral_1, spectral_eqn) in the snapshot basis, as the eigensolver forms it:
 * D (device, n_coarse_faces * jmax doubles) the diagonal of a(., .) =
 * |e_l| (kappa^{-1} mean of the two cells at e_l), and S (device, n_coarse_faces *
 * jmax * jmax doubles, row-major per face, symmetrised) s(., .) with its prefactor;
 * jmax = max(bx, by); entries beyond a face's J_i fine faces are 0.  Reflects the
 * current operator (its Gram matrices are rebuilt by tgms_update_mobility).
 * TGMS_E_INVAL for the RT0 coarse space (no snapshots). */
tgms_status tgms_probe_pencil(tgms_ctx* ctx, double* D, double* S);

/* Return the device memory blocks the library keeps for reuse (freed contexts'
 * workspaces, at most 16 GB per device) to the HIP runtime, on the current device.
 * Call with no context of the library in use on that device from another thread. */
void tgms_trim_device_cache(void);

/* Basis counts l_i (host, n_coarse_faces ints) and all eigenvalues lambda of
 * each local spectral problem, ascending (host, n_coarse_faces * jmax doubles,
 * jmax = max(bx, by), on the cube the most fine faces of a coarse face; rows of faces
 * with fewer fine faces are padded with 0).
 * Coarse faces are ordered: x-faces (block row J, I = 1..Nx-1), then y-faces
 * (J = 1..Ny-1, block column I). */
tgms_status tgms_get_counts(const tgms_ctx* ctx, int* counts);
tgms_status tgms_get_eigs(const tgms_ctx* ctx, double* eigs);

/* Condition-number estimate of the preconditioned operator from the last
 * solve's PCG scalars (Lanczos tridiagonal), as the paper reports "Cond". */
tgms_status tgms_last_cond(const tgms_ctx* ctx, double* cond);

/* Per-kernel timing with HIP events on the context's stream (for roofline
 * measurements).  tgms_profile(ctx, 1) starts recording every launch of the
 * instrumented kernels (and clears earlier records); tgms_profile_get
 * returns the number of launches and their summed duration in ms.
 * kernel: 0 = smoother patch solve, 1 = search-direction update with the
 * stream-function operator apply (q = K p, K = C^T A C), 2 = first gather of the
 * patch solutions with the residual and the coarse restriction (and, in the
 * probes, the plain restriction), 3 = the plain coarse prolongation of the
 * coarse-correction probe (in the PCG the second smoothing prolongs the coarse
 * solution itself and is counted as a smoother launch). */
tgms_status tgms_profile(tgms_ctx* ctx, int enable);
tgms_status tgms_profile_get(tgms_ctx* ctx, int kernel, int* launches, double* total_ms);

/* Kernel-only timing of the smoother patch solve: `reps` back-to-back launches
 * (after one untimed launch) on the context's stream over the context's own
 * work vector, bracketed by one HIP event pair; *avg_ms = elapsed / reps.  The
 * launches do the full work whatever the vector holds (the device done flag is
 * not consulted).  Requires a completed setup.  reps in [1, 100000], else
 * TGMS_E_INVAL.  Blocks the host until the launches have finished. */
tgms_status tgms_time_smoother(tgms_ctx* ctx, int reps, double* avg_ms);

/* The same for the search-direction update with the operator apply (p' = z + beta p,
 * q = K p' with K = C^T A C, and the partial sums of p'^T q) over the context's own
 * work vectors; the PCG scalars are overwritten (the next solve sets them again). */
tgms_status tgms_time_dir_apply(tgms_ctx* ctx, int reps, double* avg_ms);

/* Per-face outcome of the warm-started eigensolves of a context set up with
 * warm_start 1 or 2: wstat (host, n_coarse_faces ints) receives the subspace
 * iteration at which the face was accepted (0 = the initial block), or -1 when it
 * fell back to the dense solve.  TGMS_E_INVAL without a warm start. */
tgms_status tgms_get_warm_status(const tgms_ctx* ctx, int* wstat);

/* ---- warm-start network (section 4.2 eigenproblem, learned initial vectors) ----
 * A fully convolutional network on a face's permeability window: input X[h][w] =
 * log10(kappa)/3 on the cells of omega_i = K1 u K2 (rows across the coarse face,
 * H = 2 b; columns along it, W = b, in the pencil's fine-face order); four 3x3
 * convolutions with zero padding, channels 1 -> 16 -> 16 -> 16 -> 8, ReLU after the
 * first three; output: the first 8 DCT-II vectors of length W (unit norm, zero
 * beyond W) plus the mean over the rows, 8 vectors of length W.  Parameters:
 * one flat float array, per layer the weights [cout][cin][3][3] then the biases
 * [cout].  FP32 throughout.  Shapes: 1 <= H, W <= 64, H * W <= 512; n >= 1.
 * Every pointer is device memory owned by the caller; calls run on `stream`
 * (hipStream_t, NULL = the null stream) and return after it has finished them. */
int tgms_cnn_nparams(void);

/* Y [n][8][W] = network(X [n][H][W]). */
tgms_status tgms_cnn_forward(const float* params, const float* X, int n, int H, int W, float* Y, void* stream);

/* The same network for inference on the BF16 matrix cores: weights and activations
 * rounded to BF16 (nearest even), products accumulated in FP32, the first layer and
 * the output in FP32 (relative difference from tgms_cnn_forward about 1e-3 to
 * 1e-2).  The warm start of tgms_setup (warm_start = 2) uses this form. */
tgms_status tgms_cnn_infer(const float* params, const float* X, int n, int H, int W, float* Y, void* stream);

/* Floats of the workspace one training step on n samples needs (0 for bad shapes). */
size_t tgms_cnn_train_workspace(int n, int H, int W);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; t = step number from 1, lr the
 * learning rate) on the batch-mean loss sum_{c<k} |y_c/|y_c| - s_c v_c|^2 with
 * s_c = sign(y_c . v_c): X [n][H][W] inputs, V [n][8][W] unit target vectors (rows
 * c < k read, 1 <= k <= min(8, W)); params, adam_m, adam_v (tgms_cnn_nparams()
 * floats each) are updated in place; work: tgms_cnn_train_workspace(n, H, W)
 * floats; *loss (host, may be NULL) = the batch-mean loss before the step. */
tgms_status tgms_cnn_train_step(float* params, float* adam_m, float* adam_v, int t, float lr, const float* X,
                                const float* V, int n, int H, int W, int k, float* work, double* loss,
                                void* stream);

/* Training samples from a set-up context (square blocks b x b, b <= 16): X
 * [n_coarse_faces][2b][b] network inputs and V [n_coarse_faces][8][b] the unit
 * eigenvectors of T = D^{-1/2} S D^{-1/2} (section 4.2 pencil) for its 8 largest
 * mu (rows beyond b are 0), from the dense solve.  Not available after
 * tgms_update_mobility (TGMS_E_INVAL). */
tgms_status tgms_cnn_samples(tgms_ctx* ctx, float* X, float* V);

/* ---- two-phase flow by IMPES (section 6.2) ----------------------------------
 * Quadratic relative permeabilities (k_rw = s^2, k_ro = (1 - s)^2, eqs. fraction,
 * mobility): total mobility lambda(s) = s^2 / mu_w + (1 - s)^2 / mu_o, fractional
 * flow f_w(s) = (s^2 / mu_w) / lambda(s).  The saturation s is the water
 * saturation per cell (cell numbering above). */
typedef struct {
    double phi;         /* porosity, > 0 (0.2); the step divides by phi |cell| */
    double mu_w, mu_o;  /* viscosities, > 0 (1, 5) */
    double tol;         /* the step ends when max_i |R_i| <= tol (1e-12; R_i below) */
    int max_outer;      /* tile launches per step (0: 8 (nx + ny + nz)) */
} tgms_transport_params;

void tgms_default_transport(tgms_transport_params* prm);

/* lambda = total mobility of s (n cells; device arrays; stream a hipStream_t or
 * NULL).  TGMS_E_INVAL for n < 0 or a null pointer with n > 0. */
tgms_status tgms_total_mobility(const double* s, long long n, const tgms_transport_params* prm, double* lambda,
                                void* stream);

/*
 * One backward-Euler upwind finite-volume step of the saturation equation (eqs.
 * satEq, DisSatEq_Implicit, integralFlux) on the nx x ny grid of the square (nz 0 or
 * 1) or the nx x ny x nz grid of the cube (cell and face numbering of tgms_setup for
 * that dimension): s^{n+1} solves, for every cell i,
 *   R_i = s_i - s_i^n - dt / (phi |c_i|) (q_i^+ - sum_sides f_w(s_up) out_i,side
 *                                         + f_w(s_i) q_i^-) = 0,
 * out_i,side = u_f |f| the total flux out of cell i through that side, s_up the
 * saturation of the cell the flux leaves, q^+ = max(q, 0) injected water, q^- =
 * min(q, 0) produced at the cell's fractional flow.  The system is triangular in
 * flow order for a potential flow; it is solved by nonlinear Gauss-Seidel over 16 x
 * 16 (cube: 8 x 8 x 4) cell tiles (every cell's scalar equation by bracketed Newton on
 * [0, 1]) until max_i |R_i| <= tol.  The solution stays in [0, 1].
 *   u  device, nfaces doubles: total velocity (normal, full numbering; boundary
 *      entries not read, the boundary is no-flow);
 *   q  device, nx*ny doubles: cell-integrated sources (tgms_solve's F);
 *   s  device, nx*ny doubles: s^n on entry, s^{n+1} on return;
 *   outer, residual  host or NULL: tile launches used, max_i |R_i| at return.
 * TGMS_E_INVAL for bad sizes or parameters; TGMS_E_NOTCONV when max_outer launches
 * do not reach tol (s then holds the last iterate; tol below the rounding of the
 * largest a_i = dt / (phi |c_i|) outflow_i cannot be reached).  Synchronises the
 * stream (the convergence test reads the device).
 */
tgms_status tgms_transport_step(int nx, int ny, int nz, const double* u, const double* q, double* s, double dt,
                                const tgms_transport_params* prm, void* stream, long long* outer, double* residual);

/*
 * The IMPES loop of section 6.2 with the context's coarse space kept: for k = 0 ..
 * steps-1, when k % pressure_every == 0 the mobility of the current s is set
 * (tgms_update_mobility) and the pressure equation solved (tgms_solve with F, no-flow
 * boundary, rtol, maxit); then s takes one transport step of length dt with q = F.
 *   F  device, nx*ny doubles (cell-integrated sources, sum 0);
 *   s  device, nx*ny doubles: initial saturation on entry, final on return;
 *   u  device, nfaces doubles, or NULL: the last pressure solve's velocity;
 *   pcg_iters  host, ceil(steps / pressure_every) ints, or NULL.
 * Runs on the context's stream; errors as in the calls it makes.
 */
tgms_status tgms_impes(tgms_ctx* ctx, const double* F, double* s, int steps, double dt, int pressure_every,
                       const tgms_transport_params* prm, double rtol, int maxit, double* u, int* pcg_iters);

void tgms_destroy(tgms_ctx* ctx);
const char* tgms_last_error(void);

/* ---- operator probes (same definitions the solver uses; for testing) ----
 * Vectors are device arrays in the full face numbering; boundary entries of
 * inputs are ignored and of outputs set to 0.                              */

/* y = A_h x restricted to the interior faces (eq. fine_system). */
tgms_status tgms_apply_A(tgms_ctx* ctx, const double* x, double* y);

/* vbar of the preprocessing step (section 3, eq. subproblem): B vbar = F - B_bnd g. */
tgms_status tgms_preprocess(tgms_ctx* ctx, const double* F, const double* g_bnd, double* vbar);

/* z = M r for the residual r of the reduced problem: which = 0 smoother
 * (eq. smooth), 1 coarse correction (eq. coarsepre), 2 two-grid (section 5).
 * Runs in the context's precision. */
tgms_status tgms_apply_precond(tgms_ctx* ctx, int which, const double* r, double* z);

#ifdef __cplusplus
}
#endif
#endif /* TGMS_H */
