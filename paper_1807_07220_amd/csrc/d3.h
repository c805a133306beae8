// The solver on the unit cube (paper section 2 in three dimensions; models 2 and 3 of
// section 6): RT0 x P0 on a uniform grid, the two-grid preconditioner of section 5 with
// the spectral coarse space of section 4, PCG on the face vectors.
//
// Layout in HBM
//   cells (i, j, k)  index (k ny + j) nx + i;
//   faces            full numbering, x-faces ((k ny + j)(nx + 1) + i), then y-faces
//                    ((k (ny + 1) + j) nx + i), then z-faces ((k ny + j) nx + i), each the
//                    normal velocity along +x, +y, +z; boundary entries are zero (no flow);
//   boxes            coarse blocks K (block size b) and oversampled patches K^+ (b plus the
//                    overlap on each side, clipped to D), numbered like the blocks; a box's
//                    cells and its closure faces are numbered like the grid's, inside a
//                    padded box of extents E (the largest box), cells beyond the box's own
//                    extent e inactive.
#pragma once
#include <vector>

#include "common.h"

namespace tgms3 {

constexpr int MAXE = 32;  // largest box extent per axis
constexpr int JM = 64;    // largest number of fine faces on a coarse face

struct G3 {
    int n[3];           // cells per axis
    double h[3];        // cell sizes
    double vol;         // cell volume
    long long foff[3];  // first index of each axis's faces
    long long nf;       // faces
    long long nc;       // cells
};

struct Boxes {
    int b[3], N[3], ov;  // block size, blocks per axis, overlap (0: the blocks themselves)
    int E[3];            // padded extents
    int n;               // padded cells
    int nfc;             // closure faces of the padded box
    int count;           // boxes
};

__host__ __device__ inline long long cell_id(const G3& g, int i, int j, int k) {
    return ((long long)k * g.n[1] + j) * g.n[0] + i;
}

__host__ __device__ inline long long face_id(const G3& g, int a, const int* q) {
    if (a == 0) return ((long long)q[2] * g.n[1] + q[1]) * (g.n[0] + 1) + q[0];
    if (a == 1) return g.foff[1] + ((long long)q[2] * (g.n[1] + 1) + q[1]) * g.n[0] + q[0];
    return g.foff[2] + ((long long)q[2] * g.n[1] + q[1]) * g.n[0] + q[0];
}

// face index -> axis and position (the coordinate along the axis counts faces)
__host__ __device__ inline int face_pos(const G3& g, long long f, int* q) {
    if (f < g.foff[1]) {
        q[0] = (int)(f % (g.n[0] + 1));
        const long long r = f / (g.n[0] + 1);
        q[1] = (int)(r % g.n[1]);
        q[2] = (int)(r / g.n[1]);
        return 0;
    }
    if (f < g.foff[2]) {
        const long long l = f - g.foff[1];
        q[0] = (int)(l % g.n[0]);
        const long long r = l / g.n[0];
        q[1] = (int)(r % (g.n[1] + 1));
        q[2] = (int)(r / (g.n[1] + 1));
        return 1;
    }
    const long long l = f - g.foff[2];
    q[0] = (int)(l % g.n[0]);
    const long long r = l / g.n[0];
    q[1] = (int)(r % g.n[1]);
    q[2] = (int)(r / g.n[1]);
    return 2;
}

__host__ __device__ inline long long cell_stride(const G3& g, int a) {
    return a == 0 ? 1 : a == 1 ? g.n[0] : (long long)g.n[0] * g.n[1];
}

__host__ __device__ inline void box_of(const Boxes& B, const G3& g, int id, int* lo, int* e) {
    const int I[3] = {id % B.N[0], (id / B.N[0]) % B.N[1], id / (B.N[0] * B.N[1])};
    for (int a = 0; a < 3; ++a) {
        lo[a] = I[a] * B.b[a] - B.ov;
        if (lo[a] < 0) lo[a] = 0;
        int hi = (I[a] + 1) * B.b[a] + B.ov;
        if (hi > g.n[a]) hi = g.n[a];
        e[a] = hi - lo[a];
    }
}

// closure face of a box with padded extents E: axis a, local position q (q[a] counts faces)
__host__ __device__ inline int lface(const int* E, int a, const int* q) {
    const int NX = (E[0] + 1) * E[1] * E[2], NY = E[0] * (E[1] + 1) * E[2];
    if (a == 0) return (q[2] * E[1] + q[1]) * (E[0] + 1) + q[0];
    if (a == 1) return NX + (q[2] * (E[1] + 1) + q[1]) * E[0] + q[0];
    return NX + NY + (q[2] * E[1] + q[1]) * E[0] + q[0];
}

// stride of lface along its own axis
__host__ __device__ inline int lface_stride(const int* E, int a) { return a == 0 ? 1 : a == 1 ? E[0] : E[0] * E[1]; }

__host__ __device__ inline int closure_faces(const int* E) {
    return (E[0] + 1) * E[1] * E[2] + E[0] * (E[1] + 1) * E[2] + E[0] * E[1] * (E[2] + 1);
}

struct Ctx3 {
    G3 g;
    Boxes blk, pat;
    int nblk = 0;
    int ne = 0;        // interior coarse faces
    int Jmax = 0;      // fine faces of the widest coarse face
    int Jax[3] = {0, 0, 0};
    int cmax = 0;      // most modes kept on one face
    int nu = 0;        // coarse velocity unknowns (sum of the counts)
    double eta = 0.2, s_scale = 1.0, tol = 0.0;
    int coarse_space = 0;
    // device
    double* w = nullptr;      // |c| kappa^{-1} / lambda per cell
    double* kinv = nullptr;   // kappa^{-1} of the setup
    int* cf = nullptr;        // [ne][4]: axis, I0, I1, I2 (I: the block on the high side)
    int* slot = nullptr;      // [nblk][6]: coarse face of side 2a + (0 low, 1 high), or -1
    int* fnoff = nullptr;     // [ne + 1]: first coarse unknown of each face
    double* Sblk = nullptr;   // [nblk][n][n]: (B A^{-1} B^T + sigma 1 1^T)^{-1} of the blocks
    double* Spat = nullptr;   // the same for the patches
    double* eigs = nullptr;   // [ne][Jmax]
    int* counts = nullptr;    // [ne]
    double* Y = nullptr;      // [ne][Jmax][Jmax]: snapshot coefficients of the kept modes
    double* W = nullptr;      // [nblk][nfc][6 cmax]: the basis on each block's closure faces
    double* PH = nullptr;     // [nu][nu]: the coarse solution operator
    double* BH = nullptr;     // [nblk][nu]
    double* Q0T = nullptr;    // [nblk][ne]: the coarse RT0 preprocessing operator
    double* dctq[3] = {nullptr, nullptr, nullptr};  // orthonormal DCT-II per axis
    // solve workspaces
    double *vbar = nullptr, *vx = nullptr, *vr = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr,
           *vt = nullptr, *vt2 = nullptr, *vrold = nullptr;
    double *patch_out = nullptr, *cbk = nullptr, *cb = nullptr, *cz = nullptr, *cell1 = nullptr, *cell2 = nullptr,
           *part = nullptr, *gK = nullptr, *vH = nullptr;
    std::vector<int> counts_h;
    std::vector<double> eigs_h;
    std::vector<double> hist_alpha, hist_beta;
    double t_snap_ms = 0, t_eig_ms = 0, t_coarse_ms = 0, t_smoother_ms = 0;
};

// entry points used by the C ABI (k3.hip); all run on c->stream
void setup3(tgms_ctx* c, const tgms_grid* grid, const double* kappa, double eig_tol, const tgms_options* opt);
void solve3(tgms_ctx* c, const double* F, double rtol, int maxit, double* u, double* p, int* iters, double* relres,
            tgms_status* st);
void update_mobility3(tgms_ctx* c, const double* lambda);
void apply_A3(tgms_ctx* c, const double* x, double* y);
void preprocess3(tgms_ctx* c, const double* F, double* vbar);
void apply_precond3(tgms_ctx* c, int which, const double* r, double* z);
void destroy3(tgms_ctx* c);
void smooth_patches3(tgms_ctx* c);  // one launch of the patch solves on the solve workspace (timing)

}  // namespace tgms3
