// The solver on the unit cube: kernels and host steps (layout in d3.h).
//
// Local saddle problems (eq. fine_system restricted to a box, zero flux on its boundary,
// the cell sum of the pressure fixed by one multiplier) are solved through the pressure:
// the mass matrix of a box couples only the faces of one grid line (no coupling across
// axes on a box grid with scalar kappa), so A^{-1} is a tridiagonal solve per line, and
//   p = (B A^{-1} B^T + sigma 1 1^T)^{-1} (B A^{-1} f - g + mu 1),  mu = sum(g) / #cells,
//   v = A^{-1} (f - B^T p)
// solves [A B^T 0; B 0 1; 0 1^T 0] [v; p; mu] = [f; g; 0]; the Schur matrix B A^{-1} B^T
// is a sum of dense line blocks, and its inverse (with the rank-one term that fixes the
// constant) is formed once per box by a batched MFMA Cholesky.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "d3.h"
#include "jacobi.h"

namespace tgms3 {
namespace {

constexpr int NT3 = 256;

inline unsigned nblocks(long long n, int t = NT3) { return (unsigned)((n + t - 1) / t); }

__device__ inline double area_of(const G3& g, int a) { return g.vol / g.h[a]; }

// ---------------------------------------------------------------- cell data
__global__ void k3_weights(const double* __restrict__ kappa, long long nc, double vol, double* __restrict__ w,
                           double* __restrict__ kinv, int* __restrict__ bad) {
    const long long c = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (c >= nc) return;
    const double k = kappa[c];
    if (!(k > 0.0) || !isfinite(k)) {
        atomicOr(bad, 1);
        return;
    }
    kinv[c] = 1.0 / k;
    w[c] = vol / k;
}

__global__ void k3_mob_weights(const double* __restrict__ kinv, const double* __restrict__ lam, long long nc,
                               double vol, double* __restrict__ w, int* __restrict__ bad) {
    const long long c = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (c >= nc) return;
    const double l = lam[c];
    if (!(l > 0.0) || !isfinite(l)) {
        atomicOr(bad, 1);
        return;
    }
    w[c] = vol * kinv[c] / l;
}

// ---------------------------------------------------------------- operator
// y = A x on the interior faces (boundary entries of y set to 0): per face of axis a
// between cells L and R, (w_L + w_R)/3 x_f + w_L/6 x_{f-} + w_R/6 x_{f+}
__global__ void k3_apply_A(G3 g, const double* __restrict__ w, const double* __restrict__ x,
                           double* __restrict__ y) {
    const long long f = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (f >= g.nf) return;
    int q[3];
    const int a = face_pos(g, f, q);
    const int pa = q[a];
    if (pa == 0 || pa == g.n[a]) {
        y[f] = 0.0;
        return;
    }
    const long long fs = a == 0 ? 1 : a == 1 ? g.n[0] : (long long)g.n[0] * g.n[1];
    int qc[3] = {q[0], q[1], q[2]};
    const long long R = cell_id(g, qc[0], qc[1], qc[2]);
    const long long L = R - cell_stride(g, a);
    const double wl = w[L], wr = w[R];
    y[f] = (wl + wr) * (1.0 / 3.0) * x[f] + wl * (1.0 / 6.0) * x[f - fs] + wr * (1.0 / 6.0) * x[f + fs];
}

// out_c = (B u)_c = sum over the cell's faces of +-|face| u (the cell-integrated divergence)
__global__ void k3_div(G3 g, const double* __restrict__ u, double* __restrict__ out, const double* __restrict__ sub) {
    const long long c = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (c >= g.nc) return;
    const int i = (int)(c % g.n[0]);
    const long long r = c / g.n[0];
    const int j = (int)(r % g.n[1]), k = (int)(r / g.n[1]);
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        int q[3] = {i, j, k};
        const double ar = g.vol / g.h[a];
        const double lo = u[face_id(g, a, q)];
        q[a] += 1;
        const double hi = u[face_id(g, a, q)];
        s += ar * (hi - lo);
    }
    out[c] = sub ? sub[c] - s : s;
}

// ---------------------------------------------------------------- boxes
// Tridiagonal solve in place along one box line of the closure layout: faces at positions
// 1 .. m-1 (stride fs from base), cells 0 .. m-1 with weights wc(t).
template <typename WF>
__device__ inline void line_solve(double* __restrict__ y, int base, int fs, int m, WF wc) {
    if (m < 2) return;
    double cp[MAXE];
    double wprev = wc(0);
    double den_prev_c = 0.0, dprev = 0.0;
    for (int t = 1; t < m; ++t) {
        const double wt = wc(t);
        const double bdiag = (wprev + wt) * (1.0 / 3.0);
        const double sub = wprev * (1.0 / 6.0), sup = wt * (1.0 / 6.0);
        const double den = bdiag - (t > 1 ? sub * den_prev_c : 0.0);
        const double inv = 1.0 / den;
        const double c_t = (t < m - 1) ? sup * inv : 0.0;
        const double d_t = (y[base + t * fs] - (t > 1 ? sub * dprev : 0.0)) * inv;
        cp[t] = c_t;
        y[base + t * fs] = d_t;
        den_prev_c = c_t;
        dprev = d_t;
        wprev = wt;
    }
    for (int t = m - 2; t >= 1; --t) y[base + t * fs] -= cp[t] * y[base + (t + 1) * fs];
}

// every line of the box (all three axes): lines are independent, one thread each
__device__ inline void box_lines_solve(double* y, const G3& g, const int* E, const int* lo, const int* e,
                                       const double* __restrict__ w) {
    const int nl0 = E[1] * E[2], nl1 = E[0] * E[2], nl2 = E[0] * E[1];
    for (int L = threadIdx.x; L < nl0 + nl1 + nl2; L += blockDim.x) {
        int a, u, v;
        if (L < nl0) {
            a = 0;
            u = L % E[1];
            v = L / E[1];
        } else if (L < nl0 + nl1) {
            a = 1;
            u = (L - nl0) % E[0];
            v = (L - nl0) / E[0];
        } else {
            a = 2;
            u = (L - nl0 - nl1) % E[0];
            v = (L - nl0 - nl1) / E[0];
        }
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        if (u >= e[t1] || v >= e[t2]) continue;
        int q[3];
        q[a] = 0;
        q[t1] = u;
        q[t2] = v;
        const int base = lface(E, a, q);
        int qc[3];
        qc[a] = lo[a];
        qc[t1] = lo[t1] + u;
        qc[t2] = lo[t2] + v;
        const long long c0 = cell_id(g, qc[0], qc[1], qc[2]);
        const long long cs = cell_stride(g, a);
        line_solve(y, base, lface_stride(E, a), e[a], [&](int t) { return w[c0 + t * cs]; });
    }
}

// S = B A^{-1} B^T + sigma 1 1^T on the active cells of each box (identity on inactive
// ones), sigma the mean diagonal of B A^{-1} B^T: any sigma > 0 gives the same mean-zero
// pressure, and this one keeps the constant mode at the scale of the others (with sigma = 1
// the condition number grows like 1 / (kappa |f|^2 / |c|), 1e11 on thin cells of low kappa).
// One workgroup per box; the line blocks T = B_l A_l^{-1} B_l^T are added axis by axis.
__global__ void __launch_bounds__(NT3) k3_schur(Boxes B, G3 g, const double* __restrict__ w, double* __restrict__ S) {
    const int id = blockIdx.x;
    int lo[3], e[3];
    box_of(B, g, id, lo, e);
    const int n = B.n;
    double* Sb = S + (long long)id * n * n;
    for (long long idx = threadIdx.x; idx < (long long)n * n; idx += NT3) {
        const int r = (int)(idx / n), cc = (int)(idx % n);
        const int ri = r % B.E[0], rj = (r / B.E[0]) % B.E[1], rk = r / (B.E[0] * B.E[1]);
        const int ci = cc % B.E[0], cj = (cc / B.E[0]) % B.E[1], ck = cc / (B.E[0] * B.E[1]);
        const bool ra = ri < e[0] && rj < e[1] && rk < e[2], ca = ci < e[0] && cj < e[1] && ck < e[2];
        Sb[idx] = (!ra || !ca) && r == cc ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int a = 0; a < 3; ++a) {
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        const int m = e[a];
        const double ar = area_of(g, a);
        const int lstride = a == 0 ? 1 : a == 1 ? B.E[0] : B.E[0] * B.E[1];  // local cell stride
        const long long cs = cell_stride(g, a);
        for (int L = threadIdx.x; L < e[t1] * e[t2]; L += NT3) {
            const int u = L % e[t1], v = L / e[t1];
            int ql[3];
            ql[a] = 0;
            ql[t1] = u;
            ql[t2] = v;
            const int lc0 = (ql[2] * B.E[1] + ql[1]) * B.E[0] + ql[0];
            int qg[3];
            qg[a] = lo[a];
            qg[t1] = lo[t1] + u;
            qg[t2] = lo[t2] + v;
            const long long c0 = cell_id(g, qg[0], qg[1], qg[2]);
            // W = A_l^{-1} B_l^T e_t column by column, T[s][t] = |f| (W[s+1] - W[s])
            for (int t = 0; t < m; ++t) {
                double y[MAXE + 1];
                for (int f = 0; f <= m; ++f) y[f] = 0.0;
                if (t >= 1) y[t] = -ar;       // the cell's low face
                if (t + 1 <= m - 1) y[t + 1] = ar;  // its high face
                line_solve(y, 0, 1, m, [&](int tt) { return w[c0 + tt * cs]; });
                y[0] = 0.0;
                y[m] = 0.0;
                for (int s2 = 0; s2 < m; ++s2) {
                    const double tv = ar * (y[s2 + 1] - y[s2]);
                    Sb[(long long)(lc0 + s2 * lstride) * n + lc0 + t * lstride] += tv;
                }
            }
        }
        __syncthreads();
    }
    // sigma = mean of the active diagonal, added to every active pair
    __shared__ double red[NT3 / 64];
    double ds = 0.0;
    for (int c = threadIdx.x; c < n; c += NT3) {
        const int ci = c % B.E[0], cj = (c / B.E[0]) % B.E[1], ck = c / (B.E[0] * B.E[1]);
        if (ci < e[0] && cj < e[1] && ck < e[2]) ds += Sb[(long long)c * n + c];
    }
    ds = wave_sum(ds);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ds;
    __syncthreads();
    const double sigma = (red[0] + red[1] + red[2] + red[3]) / (double)(e[0] * e[1] * e[2]);
    for (long long idx = threadIdx.x; idx < (long long)n * n; idx += NT3) {
        const int r = (int)(idx / n), cc = (int)(idx % n);
        const int ri = r % B.E[0], rj = (r / B.E[0]) % B.E[1], rk = r / (B.E[0] * B.E[1]);
        const int ci = cc % B.E[0], cj = (cc / B.E[0]) % B.E[1], ck = cc / (B.E[0] * B.E[1]);
        if (ri < e[0] && rj < e[1] && rk < e[2] && ci < e[0] && cj < e[1] && ck < e[2]) Sb[idx] += sigma;
    }
}

// One local saddle solve per box (single right-hand side):
//   f = scale_f * fglob on the box's interior faces, g = gglob on its cells (or 0);
// the solution v on the interior faces goes to out_box (closure layout, boundary 0) or is
// added to out_glob (boxes with disjoint interiors).  LDS: the closure faces and two cell
// vectors of the padded box.
__global__ void __launch_bounds__(NT3) k3_box_solve(Boxes B, G3 g, const double* __restrict__ w,
                                                    const double* __restrict__ Sinv, const double* __restrict__ fglob,
                                                    double scale_f, const double* __restrict__ gglob,
                                                    double* __restrict__ out_box, double* __restrict__ out_glob) {
    extern __shared__ double lds[];
    const int id = blockIdx.x;
    int lo[3], e[3];
    box_of(B, g, id, lo, e);
    const int n = B.n, nfc = B.nfc;
    double* y = lds;        // nfc
    double* h = y + nfc;    // n
    double* p = h + n;      // n
    __shared__ double red[NT3 / 64];
    // y = f on interior faces
    auto load_f = [&]() {
        for (int lf = threadIdx.x; lf < nfc; lf += NT3) {
            int q[3];
            int a;
            const int NX = (B.E[0] + 1) * B.E[1] * B.E[2], NY = B.E[0] * (B.E[1] + 1) * B.E[2];
            if (lf < NX) {
                a = 0;
                q[0] = lf % (B.E[0] + 1);
                q[1] = (lf / (B.E[0] + 1)) % B.E[1];
                q[2] = lf / ((B.E[0] + 1) * B.E[1]);
            } else if (lf < NX + NY) {
                a = 1;
                const int l = lf - NX;
                q[0] = l % B.E[0];
                q[1] = (l / B.E[0]) % (B.E[1] + 1);
                q[2] = l / (B.E[0] * (B.E[1] + 1));
            } else {
                a = 2;
                const int l = lf - NX - NY;
                q[0] = l % B.E[0];
                q[1] = (l / B.E[0]) % B.E[1];
                q[2] = l / (B.E[0] * B.E[1]);
            }
            bool in = q[a] >= 1 && q[a] <= e[a] - 1;
            for (int d = 0; d < 3; ++d)
                if (d != a && q[d] >= e[d]) in = false;
            double v = 0.0;
            if (in) {
                int qg[3] = {lo[0] + q[0], lo[1] + q[1], lo[2] + q[2]};
                v = scale_f * fglob[face_id(g, a, qg)];
            }
            y[lf] = v;
        }
    };
    load_f();
    __syncthreads();
    box_lines_solve(y, g, B.E, lo, e, w);
    __syncthreads();
    // h = B y - g + mu
    double gs = 0.0;
    for (int c = threadIdx.x; c < n; c += NT3) {
        const int ci = c % B.E[0], cj = (c / B.E[0]) % B.E[1], ck = c / (B.E[0] * B.E[1]);
        double hv = 0.0;
        if (ci < e[0] && cj < e[1] && ck < e[2]) {
            int q[3] = {ci, cj, ck};
            for (int a = 0; a < 3; ++a) {
                const double lo_v = y[lface(B.E, a, q)];
                q[a] += 1;
                const double hi_v = y[lface(B.E, a, q)];
                q[a] -= 1;
                hv += area_of(g, a) * (hi_v - lo_v);
            }
            if (gglob) {
                const double gv = gglob[cell_id(g, lo[0] + ci, lo[1] + cj, lo[2] + ck)];
                hv -= gv;
                gs += gv;
            }
        }
        h[c] = hv;
    }
    if (gglob) {
        gs = wave_sum(gs);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = gs;
        __syncthreads();
        const double mu = (red[0] + red[1] + red[2] + red[3]) / (double)(e[0] * e[1] * e[2]);
        for (int c = threadIdx.x; c < n; c += NT3) {
            const int ci = c % B.E[0], cj = (c / B.E[0]) % B.E[1], ck = c / (B.E[0] * B.E[1]);
            if (ci < e[0] && cj < e[1] && ck < e[2]) h[c] += mu;
        }
    }
    __syncthreads();
    // p = Sinv h (Sinv symmetric: column reads are coalesced across the rows)
    const double* Sb = Sinv + (long long)id * n * n;
    for (int r0 = 0; r0 < n; r0 += NT3) {
        const int r = r0 + threadIdx.x;
        double acc = 0.0;
        if (r < n)
            for (int j = 0; j < n; ++j) acc += Sb[(long long)j * n + r] * h[j];
        if (r < n) p[r] = acc;
    }
    __syncthreads();
    // y = f - B^T p, then v = A^{-1} y
    load_f();
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += NT3) {
        const int ci = c % B.E[0], cj = (c / B.E[0]) % B.E[1], ck = c / (B.E[0] * B.E[1]);
        if (!(ci < e[0] && cj < e[1] && ck < e[2])) continue;
        // each interior face is handled by the cell on its low side: (B^T p)_f = |f| (p_L - p_R)
        int q[3] = {ci, cj, ck};
        for (int a = 0; a < 3; ++a) {
            if (q[a] + 1 > e[a] - 1) continue;
            const int cR = c + (a == 0 ? 1 : a == 1 ? B.E[0] : B.E[0] * B.E[1]);
            q[a] += 1;
            y[lface(B.E, a, q)] -= area_of(g, a) * (p[c] - p[cR]);
            q[a] -= 1;
        }
    }
    __syncthreads();
    box_lines_solve(y, g, B.E, lo, e, w);
    __syncthreads();
    if (out_box) {
        double* ob = out_box + (long long)id * nfc;
        for (int lf = threadIdx.x; lf < nfc; lf += NT3) ob[lf] = y[lf];
    } else {
        // interior faces of the box into the global vector
        for (int a = 0; a < 3; ++a) {
            if (e[a] < 2) continue;
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const int cnt = (e[a] - 1) * e[t1] * e[t2];
            for (int idx = threadIdx.x; idx < cnt; idx += NT3) {
                int q[3];
                q[a] = 1 + idx % (e[a] - 1);
                q[t1] = (idx / (e[a] - 1)) % e[t1];
                q[t2] = idx / ((e[a] - 1) * e[t1]);
                int qg[3] = {lo[0] + q[0], lo[1] + q[1], lo[2] + q[2]};
                out_glob[face_id(g, a, qg)] += y[lface(B.E, a, q)];
            }
        }
    }
}

// z = scale * sum over the patches that hold face f as an interior face of their solution
// (fixed order of the patches: deterministic)
__global__ void k3_gather(G3 g, Boxes P, const double* __restrict__ pout, double scale, double* __restrict__ z) {
    const long long f = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (f >= g.nf) return;
    int q[3];
    const int a = face_pos(g, f, q);
    if (q[a] == 0 || q[a] == g.n[a]) {
        z[f] = 0.0;
        return;
    }
    // candidate blocks per axis
    int cand[3][8], nc[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = 0;
        const int x = q[d];
        int i0 = (x - P.ov) / P.b[d] - 1, i1 = (x + P.ov) / P.b[d] + 1;
        if (i0 < 0) i0 = 0;
        if (i1 > P.N[d] - 1) i1 = P.N[d] - 1;
        for (int I = i0; I <= i1 && nc[d] < 8; ++I) {
            int lo = I * P.b[d] - P.ov, hi = (I + 1) * P.b[d] + P.ov;
            if (lo < 0) lo = 0;
            if (hi > g.n[d]) hi = g.n[d];
            const bool in = (d == a) ? (lo < x && x < hi) : (lo <= x && x < hi);
            if (in) cand[d][nc[d]++] = I;
        }
    }
    double s = 0.0;
    for (int u2 = 0; u2 < nc[2]; ++u2)
        for (int u1 = 0; u1 < nc[1]; ++u1)
            for (int u0 = 0; u0 < nc[0]; ++u0) {
                const int I[3] = {cand[0][u0], cand[1][u1], cand[2][u2]};
                const int id = (I[2] * P.N[1] + I[1]) * P.N[0] + I[0];
                int ql[3];
                for (int d = 0; d < 3; ++d) {
                    int lo = I[d] * P.b[d] - P.ov;
                    if (lo < 0) lo = 0;
                    ql[d] = q[d] - lo;
                }
                s += pout[(long long)id * P.nfc + lface(P.E, a, ql)];
            }
    z[f] = scale * s;
}

// ---------------------------------------------------------------- snapshots (section 4.1)
// Column col = s * Jmax + l of block K: the snapshot of fine face l of the block's side s
// (s = 2a + 0 low, 2a + 1 high; eq. snapshot_eqn): v.n = 1 on that fine face, 0 on the rest
// of dK, divergence alpha = +-|e_l| / |K| in every cell (+ when the face is the block's high
// side, the outward direction of the snapshot's flux).
struct SnapCol {
    bool valid;
    int a, side, t0, t1;
    int q[3];   // local position of the fine face on the closure
    int qc[3];  // local cell inside K next to it
};

__device__ inline SnapCol snap_col(const Boxes& B, const int* __restrict__ slot, int K, int col, int Jmax) {
    SnapCol sc;
    const int s = col / Jmax, l = col % Jmax;
    sc.a = s / 2;
    sc.side = s % 2;
    sc.t0 = sc.a == 0 ? 1 : 0;
    sc.t1 = sc.a == 2 ? 1 : 2;
    const int J = B.b[sc.t0] * B.b[sc.t1];
    sc.valid = s < 6 && slot[K * 6 + s] >= 0 && l < J;
    if (!sc.valid) return sc;
    sc.q[sc.a] = sc.side ? B.b[sc.a] : 0;
    sc.q[sc.t0] = l % B.b[sc.t0];
    sc.q[sc.t1] = l / B.b[sc.t0];
    sc.qc[0] = sc.q[0];
    sc.qc[1] = sc.q[1];
    sc.qc[2] = sc.q[2];
    sc.qc[sc.a] = sc.side ? B.b[sc.a] - 1 : 0;
    return sc;
}

// H[K][c][col] = (B A^{-1} f - g + mu)_c for the snapshot right-hand sides
//   f = -A[interior faces, e_l] (one entry, the face next to e_l on its line),
//   g = alpha |c| - B[:, e_l]
__global__ void k3_snap_rhs(Boxes B, G3 g, const double* __restrict__ w, const int* __restrict__ slot, int Jmax,
                            double* __restrict__ H) {
    const int K = blockIdx.x;
    const int col = blockIdx.y * 64 + threadIdx.x;
    const int ncol = 6 * Jmax;
    if (col >= ncol) return;
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    const int n = B.n;
    double* Hc = H + (long long)K * n * ncol + col;
    const SnapCol sc = snap_col(B, slot, K, col, Jmax);
    if (!sc.valid) {
        for (int c = 0; c < n; ++c) Hc[(long long)c * ncol] = 0.0;
        return;
    }
    const int a = sc.a, m = B.b[a];
    const double ar = area_of(g, a);
    const double volK = g.vol * n;
    const double alpha = (sc.side ? 1.0 : -1.0) * ar / volK;
    const long long cadj = cell_id(g, lo[0] + sc.qc[0], lo[1] + sc.qc[1], lo[2] + sc.qc[2]);
    // y = A^{-1} f on the line through the adjacent cell
    int ql[3] = {sc.qc[0], sc.qc[1], sc.qc[2]};
    ql[a] = 0;
    const long long c0 = cell_id(g, lo[0] + ql[0], lo[1] + ql[1], lo[2] + ql[2]);
    const long long cs = cell_stride(g, a);
    double y[MAXE + 1];
    for (int t = 0; t <= m; ++t) y[t] = 0.0;
    if (m >= 2) {
        y[sc.side ? m - 1 : 1] = -w[cadj] * (1.0 / 6.0);
        line_solve(y, 0, 1, m, [&](int t) { return w[c0 + t * cs]; });
    }
    y[0] = 0.0;
    y[m] = 0.0;
    const double bsign = sc.side ? ar : -ar;  // B[c_adj, e_l]
    const double mu = (alpha * g.vol * n - bsign) / n;
    const int ladj = (sc.qc[2] * B.E[1] + sc.qc[1]) * B.E[0] + sc.qc[0];
    const int lstride = a == 0 ? 1 : a == 1 ? B.E[0] : B.E[0] * B.E[1];
    const int l0 = (ql[2] * B.E[1] + ql[1]) * B.E[0] + ql[0];
    for (int c = 0; c < n; ++c) {
        double hv = -alpha * g.vol + mu;
        if (c == ladj) hv += bsign;
        const int d = c - l0;
        if (d >= 0 && d % lstride == 0 && d / lstride < m) {
            // on the line: check the transverse coordinates
            const int ci = c % B.E[0], cj = (c / B.E[0]) % B.E[1], ck = c / (B.E[0] * B.E[1]);
            const int cq[3] = {ci, cj, ck};
            bool on = true;
            for (int dd = 0; dd < 3; ++dd)
                if (dd != a && cq[dd] != ql[dd]) on = false;
            if (on) {
                const int t = cq[a];
                hv += ar * (y[t + 1] - y[t]);
            }
        }
        Hc[(long long)c * ncol] = hv;
    }
}

// C[K][lf][col] = the snapshot on the block's closure faces: v = A^{-1}(f - B^T p) inside,
// 1 on e_l, 0 on the rest of the boundary (P[K][c][col] = p)
__global__ void k3_snap_finish(Boxes B, G3 g, const double* __restrict__ w, const int* __restrict__ slot, int Jmax,
                               const double* __restrict__ P, double* __restrict__ C) {
    const int K = blockIdx.x;
    const int col = blockIdx.y * 64 + threadIdx.x;
    const int ncol = 6 * Jmax;
    if (col >= ncol) return;
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    const int n = B.n, nfc = B.nfc;
    double* Cc = C + (long long)K * nfc * ncol + col;
    const SnapCol sc = snap_col(B, slot, K, col, Jmax);
    const int lf_el = sc.valid ? lface(B.E, sc.a, sc.q) : -1;
    for (int lf = 0; lf < nfc; ++lf) Cc[(long long)lf * ncol] = (lf == lf_el) ? 1.0 : 0.0;
    if (!sc.valid) return;
    const double* Pc = P + (long long)K * n * ncol + col;
    // interior faces: f - B^T p
    for (int a = 0; a < 3; ++a) {
        const double ar = area_of(g, a);
        const int cstr = a == 0 ? 1 : a == 1 ? B.E[0] : B.E[0] * B.E[1];
        for (int c = 0; c < n; ++c) {
            const int cq[3] = {c % B.E[0], (c / B.E[0]) % B.E[1], c / (B.E[0] * B.E[1])};
            if (cq[a] + 1 > e[a] - 1) continue;
            int q[3] = {cq[0], cq[1], cq[2]};
            q[a] += 1;
            Cc[(long long)lface(B.E, a, q) * ncol] = -ar * (Pc[(long long)c * ncol] - Pc[(long long)(c + cstr) * ncol]);
        }
    }
    {
        const int m = B.b[sc.a];
        if (m >= 2) {
            int q[3] = {sc.q[0], sc.q[1], sc.q[2]};
            q[sc.a] = sc.side ? m - 1 : 1;
            const long long cadj = cell_id(g, lo[0] + sc.qc[0], lo[1] + sc.qc[1], lo[2] + sc.qc[2]);
            Cc[(long long)lface(B.E, sc.a, q) * ncol] += -w[cadj] * (1.0 / 6.0);
        }
    }
    // A^{-1} on every line (this thread's column only)
    for (int a = 0; a < 3; ++a) {
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        for (int v = 0; v < e[t2]; ++v)
            for (int u = 0; u < e[t1]; ++u) {
                int q[3];
                q[a] = 0;
                q[t1] = u;
                q[t2] = v;
                int qc[3];
                qc[a] = lo[a];
                qc[t1] = lo[t1] + u;
                qc[t2] = lo[t2] + v;
                const long long c0 = cell_id(g, qc[0], qc[1], qc[2]);
                const long long cs = cell_stride(g, a);
                line_solve(Cc, lface(B.E, a, q) * ncol, lface_stride(B.E, a) * ncol, e[a],
                           [&](int t) { return w[c0 + t * cs]; });
            }
    }
}

// Z = A^(K) X on the closure faces of every block, A^(K) the mass of the block's own cells
// (ncol columns per face, row-major)
__global__ void k3_closure_A(Boxes B, G3 g, const double* __restrict__ w, const double* __restrict__ X, int ncol,
                             double* __restrict__ Z) {
    const int K = blockIdx.y;
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    const int nfc = B.nfc;
    if (idx >= (long long)nfc * ncol) return;
    const int lf = (int)(idx / ncol), col = (int)(idx % ncol);
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    int q[3], a;
    const int NX = (B.E[0] + 1) * B.E[1] * B.E[2], NY = B.E[0] * (B.E[1] + 1) * B.E[2];
    if (lf < NX) {
        a = 0;
        q[0] = lf % (B.E[0] + 1);
        q[1] = (lf / (B.E[0] + 1)) % B.E[1];
        q[2] = lf / ((B.E[0] + 1) * B.E[1]);
    } else if (lf < NX + NY) {
        a = 1;
        const int l = lf - NX;
        q[0] = l % B.E[0];
        q[1] = (l / B.E[0]) % (B.E[1] + 1);
        q[2] = l / (B.E[0] * (B.E[1] + 1));
    } else {
        a = 2;
        const int l = lf - NX - NY;
        q[0] = l % B.E[0];
        q[1] = (l / B.E[0]) % B.E[1];
        q[2] = l / (B.E[0] * B.E[1]);
    }
    const double* Xb = X + (long long)K * nfc * ncol + col;
    const int fs = lface_stride(B.E, a) * ncol;
    const long long base = (long long)lf * ncol;
    const double x0 = Xb[base];
    double z = 0.0;
    if (q[a] >= 1) {  // the cell below the face
        int qc[3] = {lo[0] + q[0], lo[1] + q[1], lo[2] + q[2]};
        qc[a] -= 1;
        const double wc = w[cell_id(g, qc[0], qc[1], qc[2])];
        z += wc * (1.0 / 3.0) * x0 + wc * (1.0 / 6.0) * Xb[base - fs];
    }
    if (q[a] <= e[a] - 1) {  // the cell above it
        const double wc = w[cell_id(g, lo[0] + q[0], lo[1] + q[1], lo[2] + q[2])];
        z += wc * (1.0 / 3.0) * x0 + wc * (1.0 / 6.0) * Xb[base + fs];
    }
    Z[(long long)K * nfc * ncol + base + col] = z;
}

// ---------------------------------------------------------------- the local spectral problems (section 4.2)
// One wavefront per coarse face E: S = (G_{K1} + G_{K2} + |e|^2 (1/|K1| + 1/|K2|)) / s_scale
// (Gram matrices of the snapshots on the two blocks, plus the divergence term), D_l = |e_l|
// (kappa_L^{-1} + kappa_R^{-1}) / 2; T = D^{-1/2} S D^{-1/2} by cyclic Jacobi, lambda = 1/mu
// ascending, l_E = max(1, #{lambda < tol}) (or forced, or 1 for MsFEM), Y = D^{-1/2} V of the
// kept modes (MsFEM: all coefficients 1).
__global__ void __launch_bounds__(64) k3_pencil_eig(Boxes B, G3 g, const int* __restrict__ cf, int Jmax,
                                                    const double* __restrict__ Gm, const double* __restrict__ kinv,
                                                    double tol, double inv_scale, const int* __restrict__ force,
                                                    int msfem, double* __restrict__ eigs, int* __restrict__ counts,
                                                    double* __restrict__ Y, int* __restrict__ bad) {
    constexpr int LD = JM + 1;
    __shared__ double T[JM][LD];
    __shared__ double V[JM][LD];
    __shared__ double D[JM];
    __shared__ double cs[JM / 2][2];
    __shared__ int pq[JM / 2][2];
    __shared__ int order[JM];
    __shared__ int rot_flag;
    const int E = blockIdx.x, lane = threadIdx.x;
    const int a = cf[E * 4], I[3] = {cf[E * 4 + 1], cf[E * 4 + 2], cf[E * 4 + 3]};
    const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
    const int J = B.b[t0] * B.b[t1];
    int I1[3] = {I[0], I[1], I[2]};
    I1[a] -= 1;
    const int K1 = (I1[2] * B.N[1] + I1[1]) * B.N[0] + I1[0];
    const int K2 = (I[2] * B.N[1] + I[1]) * B.N[0] + I[0];
    const double ar = area_of(g, a);
    const double volK = g.vol * B.n;
    const double* G1 = Gm + ((long long)K1 * 6 + 2 * a + 1) * Jmax * Jmax;
    const double* G2 = Gm + ((long long)K2 * 6 + 2 * a) * Jmax * Jmax;
    for (int l = lane; l < J; l += 64) {
        int q[3];
        q[a] = I[a] * B.b[a];
        q[t0] = I[t0] * B.b[t0] + l % B.b[t0];
        q[t1] = I[t1] * B.b[t1] + l / B.b[t0];
        const long long R = cell_id(g, q[0], q[1], q[2]);
        const long long L = R - cell_stride(g, a);
        D[l] = ar * 0.5 * (kinv[L] + kinv[R]);
    }
    __syncthreads();
    const double divt = ar * ar * (2.0 / volK);
    for (int el = lane; el < J * J; el += 64) {
        const int l = el / J, m = el % J;
        const double s1 = G1[l * Jmax + m] + G2[l * Jmax + m] + divt;
        const double s2 = G1[m * Jmax + l] + G2[m * Jmax + l] + divt;
        T[l][m] = 0.5 * (s1 + s2) * inv_scale / sqrt(D[l] * D[m]);
        V[l][m] = (l == m) ? 1.0 : 0.0;
    }
    __syncthreads();
    const bool conv = jacobi_rr<JM>(&T[0][0], &V[0][0], LD, J, cs, pq, &rot_flag);
    if (!conv && lane == 0) atomicAdd(bad, 1);
    if (lane < J) {
        const double mu = T[lane][lane];
        int rank = 0;
        for (int k = 0; k < J; ++k) {
            const double o = T[k][k];
            rank += (o > mu) || (o == mu && k < lane);
        }
        order[rank] = lane;
    }
    __syncthreads();
    double* ev = eigs + (long long)E * Jmax;
    for (int k = lane; k < Jmax; k += 64) ev[k] = (k < J) ? 1.0 / T[order[k]][order[k]] : 0.0;
    int cnt = 0;
    for (int k = 0; k < J; ++k) cnt += (1.0 / T[order[k]][order[k]] < tol);
    cnt = cnt < 1 ? 1 : cnt;
    if (force) cnt = min(max(force[E], 1), J);
    if (msfem) cnt = 1;
    if (lane == 0) counts[E] = cnt;
    double* Yf = Y + (long long)E * Jmax * Jmax;
    for (int el = lane; el < Jmax * Jmax; el += 64) {
        const int l = el / Jmax, k = el % Jmax;
        Yf[el] = (l < J && k < cnt) ? (msfem ? 1.0 : V[l][order[k]] / sqrt(D[l])) : 0.0;
    }
}

// Ys[K][s][l][k] = Y[face of side s][l][k] (k < cmax), zero for sides on dD
__global__ void k3_gather_Y(const int* __restrict__ slot, const double* __restrict__ Y, int Jmax, int cmax, int nblk,
                            double* __restrict__ Ys) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    const long long tot = (long long)nblk * 6 * Jmax * cmax;
    if (idx >= tot) return;
    const int k = (int)(idx % cmax);
    const int l = (int)((idx / cmax) % Jmax);
    const long long ks = idx / ((long long)cmax * Jmax);
    const int E = slot[ks];
    Ys[idx] = E >= 0 ? Y[((long long)E * Jmax + l) * Jmax + k] : 0.0;
}

// the coarse RT0 functions on the block closures (section 3): the function of the
// block's side s = 2a + side is 1 - x_a / H_a (low side) or x_a / H_a (high side) on the
// faces of axis a, in fine face positions; Y[E][l][0] = 1
__global__ void k3_rt0_basis(Boxes B, const int* __restrict__ slot, double* __restrict__ W) {
    const int K = blockIdx.y;
    const int lf = blockIdx.x * NT3 + threadIdx.x;
    if (lf >= B.nfc) return;
    int q[3], a;
    const int NX = (B.E[0] + 1) * B.E[1] * B.E[2], NY = B.E[0] * (B.E[1] + 1) * B.E[2];
    if (lf < NX) {
        a = 0;
        q[0] = lf % (B.E[0] + 1);
    } else if (lf < NX + NY) {
        a = 1;
        q[1] = ((lf - NX) / B.E[0]) % (B.E[1] + 1);
    } else {
        a = 2;
        q[2] = (lf - NX - NY) / (B.E[0] * B.E[1]);
    }
    double* Wr = W + ((long long)K * B.nfc + lf) * 6;
    for (int s = 0; s < 6; ++s) Wr[s] = 0.0;
    const double t = (double)q[a] / B.b[a];
    if (slot[K * 6 + 2 * a] >= 0) Wr[2 * a] = 1.0 - t;
    if (slot[K * 6 + 2 * a + 1] >= 0) Wr[2 * a + 1] = t;
}

__global__ void k3_unit_Y(const int* __restrict__ cf, const Boxes B, int Jmax, int ne, double* __restrict__ Y,
                          int* __restrict__ counts) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (idx >= (long long)ne * Jmax) return;
    const int E = (int)(idx / Jmax), l = (int)(idx % Jmax);
    const int a = cf[E * 4];
    const int J = B.b[a == 0 ? 1 : 0] * B.b[a == 2 ? 1 : 2];
    Y[((long long)E * Jmax + l) * Jmax] = l < J ? 1.0 : 0.0;
    if (l == 0) counts[E] = 1;
}

// ---------------------------------------------------------------- coarse operator (eq. coarsepre)
// A_H += the block Grams GH[K] (6 cmax x 6 cmax) of the blocks of one parity colour
__global__ void k3_assemble_AH(Boxes B, const int* __restrict__ slot, const int* __restrict__ counts,
                               const int* __restrict__ fnoff, int cmax, const double* __restrict__ GH, int nu,
                               int color, double* __restrict__ AH) {
    const int K = blockIdx.y;
    const int I0 = K % B.N[0], I1 = (K / B.N[0]) % B.N[1], I2 = K / (B.N[0] * B.N[1]);
    if (((I0 & 1) | ((I1 & 1) << 1) | ((I2 & 1) << 2)) != color) return;
    const int m = 6 * cmax;
    const int idx = blockIdx.x * NT3 + threadIdx.x;
    if (idx >= m * m) return;
    const int ra = idx / m, rb = idx % m;
    const int sa = ra / cmax, ka = ra % cmax, sb = rb / cmax, kb = rb % cmax;
    const int Ea = slot[K * 6 + sa], Eb = slot[K * 6 + sb];
    if (Ea < 0 || Eb < 0 || ka >= counts[Ea] || kb >= counts[Eb]) return;
    const long long ga = fnoff[Ea] + ka, gb = fnoff[Eb] + kb;
    AH[ga * nu + gb] += GH[(long long)K * m * m + idx];
}

// B_H[K][gid] = +-|e| sum_l Y[E][l][k]: the flux of the basis function out of K
__global__ void k3_BH(G3 g, const int* __restrict__ slot, const int* __restrict__ counts, const int* __restrict__ fnoff,
                      const double* __restrict__ Y, int Jmax, int cmax, int nblk, int nu, double* __restrict__ BH) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (idx >= (long long)nblk * 6 * cmax) return;
    const int k = (int)(idx % cmax), s = (int)((idx / cmax) % 6);
    const int K = (int)(idx / (6 * cmax));
    const int E = slot[K * 6 + s];
    if (E < 0 || k >= counts[E]) return;
    const int a = s / 2;
    double sum = 0.0;
    for (int l = 0; l < Jmax; ++l) sum += Y[((long long)E * Jmax + l) * Jmax + k];
    BH[(long long)K * nu + fnoff[E] + k] = ((s & 1) ? 1.0 : -1.0) * (g.vol / g.h[a]) * sum;
}

// out = mean of the diagonal of the n x n matrix A (one workgroup)
__global__ void __launch_bounds__(NT3) k3_diag_mean(const double* __restrict__ A, int n, double* __restrict__ out) {
    __shared__ double red[NT3 / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NT3) s += A[(long long)i * n + i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1] + red[2] + red[3]) / n;
}

__global__ void k3_add_const(double* __restrict__ A, long long n, double v) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (idx < n) A[idx] += v;
}

// the coarse RT0 mass matrix (R^T A R over the block's cells) for the blocks of one colour
__global__ void __launch_bounds__(64) k3_rt0_AH0(Boxes B, G3 g, const double* __restrict__ w,
                                                 const int* __restrict__ slot, int ne, int color,
                                                 double* __restrict__ AH0) {
    const int K = blockIdx.x;
    const int I0 = K % B.N[0], I1 = (K / B.N[0]) % B.N[1], I2 = K / (B.N[0] * B.N[1]);
    if (((I0 & 1) | ((I1 & 1) << 1) | ((I2 & 1) << 2)) != color) return;
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    for (int a = 0; a < 3; ++a) {
        const double bb = B.b[a];
        double sll = 0.0, slh = 0.0, shh = 0.0;
        for (int c = threadIdx.x; c < B.n; c += 64) {
            const int cq[3] = {c % B.E[0], (c / B.E[0]) % B.E[1], c / (B.E[0] * B.E[1])};
            const double wc = w[cell_id(g, lo[0] + cq[0], lo[1] + cq[1], lo[2] + cq[2])];
            const int t = cq[a];
            const double l0 = 1.0 - t / bb, l1 = 1.0 - (t + 1) / bb, h0 = t / bb, h1 = (t + 1) / bb;
            sll += wc * ((l0 * l0 + l1 * l1) / 3.0 + (l0 * l1) / 3.0);
            shh += wc * ((h0 * h0 + h1 * h1) / 3.0 + (h0 * h1) / 3.0);
            slh += wc * ((l0 * h0 + l1 * h1) / 3.0 + (l0 * h1 + l1 * h0) / 6.0);
        }
        sll = wave_sum(sll);
        shh = wave_sum(shh);
        slh = wave_sum(slh);
        if (threadIdx.x == 0) {
            const int El = slot[K * 6 + 2 * a], Eh = slot[K * 6 + 2 * a + 1];
            if (El >= 0) AH0[(long long)El * ne + El] += sll;
            if (Eh >= 0) AH0[(long long)Eh * ne + Eh] += shh;
            if (El >= 0 && Eh >= 0) {
                AH0[(long long)El * ne + Eh] += slh;
                AH0[(long long)Eh * ne + El] += slh;
            }
        }
    }
}

__global__ void k3_rt0_BH0(G3 g, Boxes B, const int* __restrict__ slot, int nblk, int ne, double* __restrict__ BH0) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (idx >= (long long)nblk * 6) return;
    const int K = (int)(idx / 6), s = (int)(idx % 6);
    const int E = slot[K * 6 + s];
    if (E < 0) return;
    const int a = s / 2;
    const double J = (double)B.b[a == 0 ? 1 : 0] * B.b[a == 2 ? 1 : 2];
    BH0[(long long)K * ne + E] = ((s & 1) ? 1.0 : -1.0) * (g.vol / g.h[a]) * J;
}

// index of the interior coarse face of axis a whose high-side block is I
__device__ inline int coarse_face_id(const Boxes& B, int a, const int* I) {
    const int R0 = B.N[0] - (a == 0), R1 = B.N[1] - (a == 1);
    const int off1 = (B.N[0] - 1) * B.N[1] * B.N[2], off2 = off1 + B.N[0] * (B.N[1] - 1) * B.N[2];
    const int off = a == 0 ? 0 : a == 1 ? off1 : off2;
    const int i0 = I[0] - (a == 0), i1 = I[1] - (a == 1), i2 = I[2] - (a == 2);
    return off + (i2 * R1 + i1) * R0 + i0;
}

// v_H on the fine faces: the coarse RT0 functions interpolated (each fine face lies between
// two coarse faces of its axis, or on one)
__global__ void k3_rt0_interp(G3 g, Boxes B, const double* __restrict__ vH, double* __restrict__ v) {
    const long long f = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (f >= g.nf) return;
    int q[3];
    const int a = face_pos(g, f, q);
    if (q[a] == 0 || q[a] == g.n[a]) {
        v[f] = 0.0;
        return;
    }
    int I[3];
    for (int d = 0; d < 3; ++d) I[d] = q[d] / B.b[d];
    const int X0 = q[a] / B.b[a], r = q[a] % B.b[a];
    double s = 0.0;
    I[a] = X0;
    if (X0 >= 1 && X0 <= B.N[a] - 1) s += (1.0 - (double)r / B.b[a]) * vH[coarse_face_id(B, a, I)];
    if (r != 0) {
        I[a] = X0 + 1;
        if (X0 + 1 <= B.N[a] - 1) s += ((double)r / B.b[a]) * vH[coarse_face_id(B, a, I)];
    }
    v[f] = s;
}

// gK[K] = sum of F over the block's cells
__global__ void __launch_bounds__(64) k3_block_sums(Boxes B, G3 g, const double* __restrict__ F,
                                                    double* __restrict__ gK) {
    const int K = blockIdx.x;
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    double s = 0.0;
    for (int c = threadIdx.x; c < B.n; c += 64) {
        const int cq[3] = {c % B.E[0], (c / B.E[0]) % B.E[1], c / (B.E[0] * B.E[1])};
        s += F[cell_id(g, lo[0] + cq[0], lo[1] + cq[1], lo[2] + cq[2])];
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) gK[K] = s;
}

// vH[e] = sum_K Q0T[K][e] (gK[K] - mu)
__global__ void k3_vH(const double* __restrict__ Q0T, const double* __restrict__ gK, double mu, int nblk, int ne,
                      double* __restrict__ vH) {
    const int e = blockIdx.x * NT3 + threadIdx.x;
    if (e >= ne) return;
    double s = 0.0;
    for (int K = 0; K < nblk; ++K) s += Q0T[(long long)K * ne + e] * (gK[K] - mu);
    vH[e] = s;
}

// ---------------------------------------------------------------- coarse correction
// bK[K][col] = sum over the block's interior faces of W[K][lf][col] r(f)
__global__ void k3_restrict_blk(Boxes B, G3 g, const double* __restrict__ W, int ncolW, const double* __restrict__ r,
                                double* __restrict__ bK) {
    const int K = blockIdx.x;
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    const double* Wb = W + (long long)K * B.nfc * ncolW;
    for (int col = threadIdx.x; col < ncolW; col += blockDim.x) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            for (int v = 0; v < e[t2]; ++v)
                for (int u = 0; u < e[t1]; ++u)
                    for (int t = 1; t < e[a]; ++t) {
                        int q[3];
                        q[a] = t;
                        q[t1] = u;
                        q[t2] = v;
                        int qg[3] = {lo[0] + q[0], lo[1] + q[1], lo[2] + q[2]};
                        s += Wb[(long long)lface(B.E, a, q) * ncolW + col] * r[face_id(g, a, qg)];
                    }
        }
        bK[(long long)K * ncolW + col] = s;
    }
}

// b[fnoff[E] + k] = bK[K1][high side of E] + bK[K2][low side] + sum_l Y[E][l][k] r(e_l)
__global__ void k3_restrict_face(Boxes B, G3 g, const int* __restrict__ cf, const int* __restrict__ counts,
                                 const int* __restrict__ fnoff, const double* __restrict__ Y, int Jmax, int cmax,
                                 const double* __restrict__ bK, const double* __restrict__ r, int ne,
                                 double* __restrict__ b) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (idx >= (long long)ne * cmax) return;
    const int E = (int)(idx / cmax), k = (int)(idx % cmax);
    if (k >= counts[E]) return;
    const int a = cf[E * 4], I[3] = {cf[E * 4 + 1], cf[E * 4 + 2], cf[E * 4 + 3]};
    const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
    const int J = B.b[t0] * B.b[t1];
    int I1[3] = {I[0], I[1], I[2]};
    I1[a] -= 1;
    const int K1 = (I1[2] * B.N[1] + I1[1]) * B.N[0] + I1[0];
    const int K2 = (I[2] * B.N[1] + I[1]) * B.N[0] + I[0];
    double s = bK[(long long)K1 * 6 * cmax + (2 * a + 1) * cmax + k] + bK[(long long)K2 * 6 * cmax + 2 * a * cmax + k];
    for (int l = 0; l < J; ++l) {
        int q[3];
        q[a] = I[a] * B.b[a];
        q[t0] = I[t0] * B.b[t0] + l % B.b[t0];
        q[t1] = I[t1] * B.b[t1] + l / B.b[t0];
        s += Y[((long long)E * Jmax + l) * Jmax + k] * r[face_id(g, a, q)];
    }
    b[fnoff[E] + k] = s;
}

// y = M x, one wavefront per row (M n x n, row-major)
__global__ void k3_gemv(const double* __restrict__ M, int n, const double* __restrict__ x, double* __restrict__ y) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double* Mr = M + (long long)row * n;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += Mr[j] * x[j];
    s = wave_sum(s);
    if (lane == 0) y[row] = s;
}

// u on the interior faces of each block: sum over its columns of W[K][lf][col] z(col)
__global__ void k3_prolong_blk(Boxes B, G3 g, const double* __restrict__ W, int cmax, const int* __restrict__ slot,
                               const int* __restrict__ counts, const int* __restrict__ fnoff,
                               const double* __restrict__ z, double* __restrict__ u) {
    const int K = blockIdx.y;
    const int lf = blockIdx.x * NT3 + threadIdx.x;
    if (lf >= B.nfc) return;
    int q[3], a;
    const int NX = (B.E[0] + 1) * B.E[1] * B.E[2], NY = B.E[0] * (B.E[1] + 1) * B.E[2];
    if (lf < NX) {
        a = 0;
        q[0] = lf % (B.E[0] + 1);
        q[1] = (lf / (B.E[0] + 1)) % B.E[1];
        q[2] = lf / ((B.E[0] + 1) * B.E[1]);
    } else if (lf < NX + NY) {
        a = 1;
        const int l = lf - NX;
        q[0] = l % B.E[0];
        q[1] = (l / B.E[0]) % (B.E[1] + 1);
        q[2] = l / (B.E[0] * (B.E[1] + 1));
    } else {
        a = 2;
        const int l = lf - NX - NY;
        q[0] = l % B.E[0];
        q[1] = (l / B.E[0]) % B.E[1];
        q[2] = l / (B.E[0] * B.E[1]);
    }
    if (q[a] == 0 || q[a] == B.b[a]) return;
    int lo[3], e[3];
    box_of(B, g, K, lo, e);
    const int m = 6 * cmax;
    const double* Wr = W + ((long long)K * B.nfc + lf) * m;
    double s = 0.0;
    for (int sd = 0; sd < 6; ++sd) {
        const int E = slot[K * 6 + sd];
        if (E < 0) continue;
        for (int k = 0; k < counts[E]; ++k) s += Wr[sd * cmax + k] * z[fnoff[E] + k];
    }
    int qg[3] = {lo[0] + q[0], lo[1] + q[1], lo[2] + q[2]};
    u[face_id(g, a, qg)] = s;
}

// u on the fine faces of each coarse face: sum_k Y[E][l][k] z(fnoff[E] + k)
__global__ void k3_prolong_face(Boxes B, G3 g, const int* __restrict__ cf, const int* __restrict__ counts,
                                const int* __restrict__ fnoff, const double* __restrict__ Y, int Jmax,
                                const double* __restrict__ z, int ne, double* __restrict__ u) {
    const long long idx = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (idx >= (long long)ne * Jmax) return;
    const int E = (int)(idx / Jmax), l = (int)(idx % Jmax);
    const int a = cf[E * 4], I[3] = {cf[E * 4 + 1], cf[E * 4 + 2], cf[E * 4 + 3]};
    const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
    if (l >= B.b[t0] * B.b[t1]) return;
    double s = 0.0;
    for (int k = 0; k < counts[E]; ++k) s += Y[((long long)E * Jmax + l) * Jmax + k] * z[fnoff[E] + k];
    int q[3];
    q[a] = I[a] * B.b[a];
    q[t0] = I[t0] * B.b[t0] + l % B.b[t0];
    q[t1] = I[t1] * B.b[t1] + l / B.b[t0];
    u[face_id(g, a, q)] = s;
}

// ---------------------------------------------------------------- vectors
constexpr int NPART = 256;

__global__ void __launch_bounds__(NT3) k3_dot(const double* __restrict__ x, const double* __restrict__ y, long long n,
                                              double* __restrict__ part) {
    __shared__ double red[NT3 / 64];
    double s = 0.0;
    for (long long i = blockIdx.x * (long long)NT3 + threadIdx.x; i < n; i += (long long)NPART * NT3) s += x[i] * y[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// y = x + b y
__global__ void k3_xpby(const double* __restrict__ x, double b, double* __restrict__ y, long long n) {
    const long long i = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (i < n) y[i] = x[i] + b * y[i];
}

// z = x - y
__global__ void k3_sub(const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ z,
                       long long n) {
    const long long i = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (i < n) z[i] = x[i] - y[i];
}

// the orthonormal DCT-II (or its inverse) along axis a of a cell array
__global__ void k3_dct_axis(G3 g, int a, const double* __restrict__ Q, int inverse, const double* __restrict__ in,
                            double* __restrict__ out) {
    const long long c = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (c >= g.nc) return;
    const int q[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    const int na = g.n[a], kk = q[a];
    const long long st = cell_stride(g, a);
    const long long base = c - kk * st;
    double s = 0.0;
    for (int m = 0; m < na; ++m) s += (inverse ? Q[(long long)m * na + kk] : Q[(long long)kk * na + m]) * in[base + m * st];
    out[c] = s;
}

// divide by the eigenvalues of B B^T (the Neumann cell Laplacian), the constant mode to 0
__global__ void k3_dct_scale(G3 g, double* __restrict__ x) {
    const long long c = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (c >= g.nc) return;
    const int q[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    if (c == 0) {
        x[c] = 0.0;
        return;
    }
    double lam = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double ar = g.vol / g.h[a];
        lam += ar * ar * (2.0 - 2.0 * cos(M_PI * q[a] / g.n[a]));
    }
    x[c] /= lam;
}

__global__ void k3_add_scalar(double* __restrict__ x, long long n, double v) {
    const long long i = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (i < n) x[i] += v;
}

// r += sgn B^T q on the interior faces ((B^T q)_f = |f| (q_L - q_R))
__global__ void k3_add_grad(G3 g, const double* __restrict__ q, double sgn, double* __restrict__ r) {
    const long long f = blockIdx.x * (long long)NT3 + threadIdx.x;
    if (f >= g.nf) return;
    int p[3];
    const int a = face_pos(g, f, p);
    if (p[a] == 0 || p[a] == g.n[a]) return;
    const long long R = cell_id(g, p[0], p[1], p[2]);
    const long long L = R - cell_stride(g, a);
    r[f] += sgn * (g.vol / g.h[a]) * (q[L] - q[R]);
}

}  // namespace

// ---------------------------------------------------------------- host steps
namespace {

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct Tmp {  // device workspace released at scope exit (after the stream drains)
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    Tmp(size_t n, hipStream_t s) : st(s) { p = tgms::dev_alloc(n, &bytes); }
    ~Tmp() {
        if (p) {
            (void)hipStreamSynchronize(st);
            tgms::dev_free(p, bytes);
        }
    }
    template <typename T>
    T* as() {
        return reinterpret_cast<T*>(p);
    }
};

double dot3(tgms_ctx* c, Ctx3* d, const double* x, const double* y, long long n) {
    hipLaunchKernelGGL(k3_dot, dim3(NPART), dim3(NT3), 0, c->stream, x, y, n, d->part);
    LAUNCH_OK();
    double h[NPART];
    HIP_OK(hipMemcpyAsync(h, d->part, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    double s = 0.0;
    for (int k = 0; k < NPART; ++k) s += h[k];
    return s;
}

void applyA(tgms_ctx* c, Ctx3* d, const double* x, double* y) {
    hipLaunchKernelGGL(k3_apply_A, dim3(nblocks(d->g.nf)), dim3(NT3), 0, c->stream, d->g, (const double*)d->w, x, y);
    LAUNCH_OK();
}

// the Schur inverses of a box set for the current weights
void factor_boxes(tgms_ctx* c, Ctx3* d, const Boxes& B, double* S) {
    hipLaunchKernelGGL(k3_schur, dim3(B.count), dim3(NT3), 0, c->stream, B, d->g, (const double*)d->w, S);
    LAUNCH_OK();
    tgms::dense_spd_inverse_batched(c, S, B.n, B.count);
}

size_t box_lds(const Boxes& B) { return sizeof(double) * ((size_t)B.nfc + 2 * (size_t)B.n); }

// S r = eta sum_i ext((L_i^+)^{-1} [r; 0]) (eq. smooth)
void smooth(tgms_ctx* c, Ctx3* d, const double* r, double* z) {
    hipLaunchKernelGGL(k3_box_solve, dim3(d->pat.count), dim3(NT3), box_lds(d->pat), c->stream, d->pat, d->g,
                       (const double*)d->w, (const double*)d->Spat, r, 1.0, (const double*)nullptr, d->patch_out,
                       (double*)nullptr);
    LAUNCH_OK();
    hipLaunchKernelGGL(k3_gather, dim3(nblocks(d->g.nf)), dim3(NT3), 0, c->stream, d->g, d->pat,
                       (const double*)d->patch_out, d->eta, z);
    LAUNCH_OK();
}

// P r = Phi L_H^{-1} Phi^T r (eq. coarsepre); z overwritten
void coarse(tgms_ctx* c, Ctx3* d, const double* r, double* z) {
    const Boxes& B = d->blk;
    const int m = 6 * d->cmax;
    hipLaunchKernelGGL(k3_restrict_blk, dim3(d->nblk), dim3(64), 0, c->stream, B, d->g, (const double*)d->W, m, r,
                       d->cbk);
    LAUNCH_OK();
    hipLaunchKernelGGL(k3_restrict_face, dim3(nblocks((long long)d->ne * d->cmax)), dim3(NT3), 0, c->stream, B, d->g,
                       (const int*)d->cf, (const int*)d->counts, (const int*)d->fnoff, (const double*)d->Y, d->Jmax,
                       d->cmax, (const double*)d->cbk, r, d->ne, d->cb);
    LAUNCH_OK();
    hipLaunchKernelGGL(k3_gemv, dim3((d->nu + 3) / 4), dim3(256), 0, c->stream, (const double*)d->PH, d->nu,
                       (const double*)d->cb, d->cz);
    LAUNCH_OK();
    tgms::zero(c, z, sizeof(double) * d->g.nf);
    hipLaunchKernelGGL(k3_prolong_blk, dim3(nblocks(B.nfc), d->nblk), dim3(NT3), 0, c->stream, B, d->g,
                       (const double*)d->W, d->cmax, (const int*)d->slot, (const int*)d->counts,
                       (const int*)d->fnoff, (const double*)d->cz, z);
    LAUNCH_OK();
    hipLaunchKernelGGL(k3_prolong_face, dim3(nblocks((long long)d->ne * d->Jmax)), dim3(NT3), 0, c->stream, B, d->g,
                       (const int*)d->cf, (const int*)d->counts, (const int*)d->fnoff, (const double*)d->Y, d->Jmax,
                       (const double*)d->cz, d->ne, z);
    LAUNCH_OK();
}

// z = B_TG r: pre-smoothing, coarse correction, post-smoothing, the residual recomputed
// after each (section 5)
void twogrid(tgms_ctx* c, Ctx3* d, const double* r, double* z) {
    const long long nf = d->g.nf;
    smooth(c, d, r, z);
    applyA(c, d, z, d->vt);
    hipLaunchKernelGGL(k3_sub, dim3(nblocks(nf)), dim3(NT3), 0, c->stream, r, (const double*)d->vt, d->vt, nf);
    LAUNCH_OK();
    coarse(c, d, d->vt, d->vt2);
    tgms::axpy(c, nf, 1.0, d->vt2, z);
    applyA(c, d, z, d->vt);
    hipLaunchKernelGGL(k3_sub, dim3(nblocks(nf)), dim3(NT3), 0, c->stream, r, (const double*)d->vt, d->vt, nf);
    LAUNCH_OK();
    smooth(c, d, d->vt, d->vt2);
    tgms::axpy(c, nf, 1.0, d->vt2, z);
}

// S += sigma 1 1^T, sigma the mean diagonal of S (the scale of the constant mode, as in the
// boxes' Schur matrices)
void add_scaled_ones(tgms_ctx* c, Ctx3* d, double* S, int n) {
    hipLaunchKernelGGL(k3_diag_mean, dim3(1), dim3(NT3), 0, c->stream, (const double*)S, n, d->part);
    LAUNCH_OK();
    double sigma = 0.0;
    HIP_OK(hipMemcpyAsync(&sigma, d->part, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (!(sigma > 0.0) || !std::isfinite(sigma)) sigma = 1.0;
    hipLaunchKernelGGL(k3_add_const, dim3(nblocks((long long)n * n)), dim3(NT3), 0, c->stream, S, (long long)n * n,
                       sigma);
    LAUNCH_OK();
}

// the coarse operator over the kept basis: A_H = sum_K W_K^T A^(K) W_K, B_H, and
// P_H = A_H^{-1} - A_H^{-1} B_H^T (B_H A_H^{-1} B_H^T + sigma 1 1^T)^{-1} B_H A_H^{-1}
void build_coarse(tgms_ctx* c, Ctx3* d) {
    const Boxes& B = d->blk;
    const int m = 6 * d->cmax, nu = d->nu, nb = d->nblk;
    const long long wsz = (long long)nb * B.nfc * m;
    Tmp Zw(sizeof(double) * wsz, c->stream), GH(sizeof(double) * (size_t)nb * m * m, c->stream);
    hipLaunchKernelGGL(k3_closure_A, dim3(nblocks((long long)B.nfc * m), nb), dim3(NT3), 0, c->stream, B, d->g,
                       (const double*)d->w, (const double*)d->W, m, Zw.as<double>());
    LAUNCH_OK();
    tgms::gemm_batched(c, 1, 0, m, m, B.nfc, 1.0, d->W, m, tgms::Strided{(long long)B.nfc * m, 0, 1},
                       Zw.as<double>(), m, tgms::Strided{(long long)B.nfc * m, 0, 1}, 0.0, GH.as<double>(), m,
                       tgms::Strided{(long long)m * m, 0, 1}, nb);
    Tmp AH(sizeof(double) * (size_t)nu * nu, c->stream);
    tgms::zero(c, AH.p, sizeof(double) * (size_t)nu * nu);
    for (int color = 0; color < 8; ++color) {
        hipLaunchKernelGGL(k3_assemble_AH, dim3(nblocks((long long)m * m), nb), dim3(NT3), 0, c->stream, B,
                           (const int*)d->slot, (const int*)d->counts, (const int*)d->fnoff, d->cmax,
                           (const double*)GH.as<double>(), nu, color, AH.as<double>());
        LAUNCH_OK();
    }
    if (!d->BH) d->BH = c->alloc<double>((size_t)nb * nu);
    tgms::zero(c, d->BH, sizeof(double) * (size_t)nb * nu);
    hipLaunchKernelGGL(k3_BH, dim3(nblocks((long long)nb * 6 * d->cmax)), dim3(NT3), 0, c->stream, d->g,
                       (const int*)d->slot, (const int*)d->counts, (const int*)d->fnoff, (const double*)d->Y, d->Jmax,
                       d->cmax, nb, nu, d->BH);
    LAUNCH_OK();
    if (!d->PH) d->PH = c->alloc<double>((size_t)nu * nu);
    tgms::dense_spd_inverse(c, AH.as<double>(), nu, d->PH);  // PH = A_H^{-1}
    Tmp T1(sizeof(double) * (size_t)nb * nu, c->stream), SH(sizeof(double) * (size_t)nb * nb, c->stream),
        SHi(sizeof(double) * (size_t)nb * nb, c->stream), T2(sizeof(double) * (size_t)nb * nu, c->stream);
    tgms::gemm(c, 0, 0, nb, nu, nu, 1.0, d->BH, nu, d->PH, nu, 0.0, T1.as<double>(), nu);
    tgms::gemm(c, 0, 1, nb, nb, nu, 1.0, T1.as<double>(), nu, d->BH, nu, 0.0, SH.as<double>(), nb);
    add_scaled_ones(c, d, SH.as<double>(), nb);
    tgms::dense_spd_inverse(c, SH.as<double>(), nb, SHi.as<double>());
    tgms::gemm(c, 0, 0, nb, nu, nb, 1.0, SHi.as<double>(), nb, T1.as<double>(), nu, 0.0, T2.as<double>(), nu);
    tgms::gemm(c, 1, 0, nu, nu, nb, -1.0, T1.as<double>(), nu, T2.as<double>(), nu, 1.0, d->PH, nu);
    HIP_OK(hipStreamSynchronize(c->stream));
}

// the preprocessing's coarse RT0 operator: vH = Q0T^T (gK - mu), Q0T = (S + sigma 1 1^T)^{-1} B_H0 A_H0^{-1}
void build_rt0(tgms_ctx* c, Ctx3* d) {
    const int ne = d->ne, nb = d->nblk;
    Tmp AH0(sizeof(double) * (size_t)ne * ne, c->stream), AH0i(sizeof(double) * (size_t)ne * ne, c->stream),
        BH0(sizeof(double) * (size_t)nb * ne, c->stream), T1(sizeof(double) * (size_t)nb * ne, c->stream),
        SH(sizeof(double) * (size_t)nb * nb, c->stream), SHi(sizeof(double) * (size_t)nb * nb, c->stream);
    tgms::zero(c, AH0.p, sizeof(double) * (size_t)ne * ne);
    tgms::zero(c, BH0.p, sizeof(double) * (size_t)nb * ne);
    for (int color = 0; color < 8; ++color) {
        hipLaunchKernelGGL(k3_rt0_AH0, dim3(nb), dim3(64), 0, c->stream, d->blk, d->g, (const double*)d->w,
                           (const int*)d->slot, ne, color, AH0.as<double>());
        LAUNCH_OK();
    }
    hipLaunchKernelGGL(k3_rt0_BH0, dim3(nblocks((long long)nb * 6)), dim3(NT3), 0, c->stream, d->g, d->blk,
                       (const int*)d->slot, nb, ne, BH0.as<double>());
    LAUNCH_OK();
    tgms::dense_spd_inverse(c, AH0.as<double>(), ne, AH0i.as<double>());
    tgms::gemm(c, 0, 0, nb, ne, ne, 1.0, BH0.as<double>(), ne, AH0i.as<double>(), ne, 0.0, T1.as<double>(), ne);
    tgms::gemm(c, 0, 1, nb, nb, ne, 1.0, T1.as<double>(), ne, BH0.as<double>(), ne, 0.0, SH.as<double>(), nb);
    add_scaled_ones(c, d, SH.as<double>(), nb);
    tgms::dense_spd_inverse(c, SH.as<double>(), nb, SHi.as<double>());
    if (!d->Q0T) d->Q0T = c->alloc<double>((size_t)nb * ne);
    tgms::gemm(c, 0, 0, nb, ne, nb, 1.0, SHi.as<double>(), nb, T1.as<double>(), ne, 0.0, d->Q0T, ne);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void dct_matrices(tgms_ctx* c, Ctx3* d) {
    for (int a = 0; a < 3; ++a) {
        const int n = d->g.n[a];
        std::vector<double> Q((size_t)n * n);
        for (int k = 0; k < n; ++k)
            for (int m = 0; m < n; ++m)
                Q[(size_t)k * n + m] = (k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n)) *
                                       std::cos(M_PI * k * (2.0 * m + 1.0) / (2.0 * n));
        d->dctq[a] = c->alloc<double>((size_t)n * n);
        HIP_OK(hipMemcpyAsync(d->dctq[a], Q.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, c->stream));
    }
    HIP_OK(hipStreamSynchronize(c->stream));
}

// x = (B B^T)^{+} b (the Neumann cell Laplacian, constant mode removed) by the orthonormal
// DCT-II, which diagonalises it on a uniform grid; b in cell1, the result in cell1
void cell_laplace_solve(tgms_ctx* c, Ctx3* d) {
    const G3& g = d->g;
    double* a = d->cell1;
    double* b = d->cell2;
    for (int ax = 0; ax < 3; ++ax) {
        hipLaunchKernelGGL(k3_dct_axis, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, ax, (const double*)d->dctq[ax],
                           0, (const double*)a, b);
        LAUNCH_OK();
        std::swap(a, b);
    }
    hipLaunchKernelGGL(k3_dct_scale, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, a);
    LAUNCH_OK();
    for (int ax = 0; ax < 3; ++ax) {
        hipLaunchKernelGGL(k3_dct_axis, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, ax, (const double*)d->dctq[ax],
                           1, (const double*)a, b);
        LAUNCH_OK();
        std::swap(a, b);
    }
    // three swaps each way: the result is back in cell2 after an odd count; copy if needed
    if (a != d->cell1) tgms::copy(c, g.nc, a, d->cell1);
}

// r <- the Euclidean projection of r onto ker B (r zero on the boundary): r - B^T (B B^T)^+ B r
void project(tgms_ctx* c, Ctx3* d, double* r) {
    const G3& g = d->g;
    hipLaunchKernelGGL(k3_div, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, (const double*)r, d->cell1,
                       (const double*)nullptr);
    LAUNCH_OK();
    cell_laplace_solve(c, d);
    hipLaunchKernelGGL(k3_add_grad, dim3(nblocks(g.nf)), dim3(NT3), 0, c->stream, g, (const double*)d->cell1, -1.0, r);
    LAUNCH_OK();
}

// p = argmin |B_I^T p - (A u)_I| with zero mean: the Neumann cell Laplacian B B^T by the DCT
void pressure(tgms_ctx* c, Ctx3* d, const double* u, double* p) {
    const G3& g = d->g;
    applyA(c, d, u, d->vt);
    hipLaunchKernelGGL(k3_div, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, (const double*)d->vt, d->cell1,
                       (const double*)nullptr);
    LAUNCH_OK();
    cell_laplace_solve(c, d);
    tgms::copy(c, g.nc, d->cell1, p);
    // zero mean
    tgms::zero(c, d->cell1, sizeof(double) * g.nc);
    hipLaunchKernelGGL(k3_add_scalar, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, d->cell1, g.nc, 1.0);
    LAUNCH_OK();
    const double mean = dot3(c, d, p, d->cell1, g.nc) / (double)g.nc;
    hipLaunchKernelGGL(k3_add_scalar, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, p, g.nc, -mean);
    LAUNCH_OK();
}

// w with B w = G (section 3's construction): the coarse RT0 solve for the block sums of G,
// interpolated to the fine faces, then one local saddle solve per block for the rest
// (f = -A w_H, g = G - B w_H); uses vt, cell1, gK, vH
void particular(tgms_ctx* c, Ctx3* d, const double* G, double* w) {
    const G3& g = d->g;
    hipLaunchKernelGGL(k3_block_sums, dim3(d->nblk), dim3(64), 0, c->stream, d->blk, g, G, d->gK);
    LAUNCH_OK();
    std::vector<double> gk(d->nblk);
    HIP_OK(hipMemcpyAsync(gk.data(), d->gK, sizeof(double) * d->nblk, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    double mu = 0.0;
    for (double v : gk) mu += v;
    mu /= d->nblk;
    hipLaunchKernelGGL(k3_vH, dim3(nblocks(d->ne)), dim3(NT3), 0, c->stream, (const double*)d->Q0T,
                       (const double*)d->gK, mu, d->nblk, d->ne, d->vH);
    LAUNCH_OK();
    hipLaunchKernelGGL(k3_rt0_interp, dim3(nblocks(g.nf)), dim3(NT3), 0, c->stream, g, d->blk, (const double*)d->vH,
                       w);
    LAUNCH_OK();
    applyA(c, d, w, d->vt);
    hipLaunchKernelGGL(k3_div, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, (const double*)w, d->cell1, G);
    LAUNCH_OK();
    hipLaunchKernelGGL(k3_box_solve, dim3(d->blk.count), dim3(NT3), box_lds(d->blk), c->stream, d->blk, g,
                       (const double*)d->w, (const double*)d->Sblk, (const double*)d->vt, -1.0,
                       (const double*)d->cell1, (double*)nullptr, w);
    LAUNCH_OK();
}

// vbar with B vbar = F (section 3)
void preprocess(tgms_ctx* c, Ctx3* d, const double* F, double* vbar) {
    const G3& g = d->g;
    particular(c, d, F, vbar);
    // The block solves meet B vbar = F only to about eps cond(S_K) of the right-hand side
    // (explicit Schur inverses), and the PCG, kept in ker B, cannot repair it: the minimal
    // correction vbar += B^T (B B^T)^+ (F - B vbar) restores the constraint to round-off.
    // Any vbar with B vbar = F gives the same solution.
    hipLaunchKernelGGL(k3_div, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, (const double*)vbar, d->cell1, F);
    LAUNCH_OK();
    cell_laplace_solve(c, d);
    hipLaunchKernelGGL(k3_add_grad, dim3(nblocks(g.nf)), dim3(NT3), 0, c->stream, g, (const double*)d->cell1, 1.0,
                       vbar);
    LAUNCH_OK();
}

// z -= w with B w = B z: every part of the two-grid cycle returns a divergence-free field in
// exact arithmetic, but the local solves leave a divergence of about eps cond(S) |z|, and
// the PCG iterate, a sum of such directions, would drift off ker B (an energy error of 1e-6
// at contrasts of 1e8).  The correction is section 3's particular solution of that tiny
// divergence: block-local and energy-weighted, so it does not disturb the low-permeability
// faces the way a Euclidean projection does.  A no-op in exact arithmetic.
void repair_divergence(tgms_ctx* c, Ctx3* d, double* z) {
    const G3& g = d->g;
    hipLaunchKernelGGL(k3_div, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, g, (const double*)z, d->cell2,
                       (const double*)nullptr);
    LAUNCH_OK();
    particular(c, d, d->cell2, d->vt2);
    tgms::axpy(c, g.nf, -1.0, d->vt2, z);
}

}  // namespace

// ---------------------------------------------------------------- entry points
void setup3(tgms_ctx* c, const tgms_grid* grid, const double* kappa, double eig_tol, const tgms_options* o) {
    const int n[3] = {grid->nx, grid->ny, grid->nz}, b[3] = {grid->bx, grid->by, grid->bz};
    for (int a = 0; a < 3; ++a)
        if (n[a] <= 0 || b[a] <= 0 || n[a] % b[a])
            throw TgmsError{TGMS_E_INVAL, "grid sizes must be positive and divisible by the block size"};
    if (!(eig_tol > 0) || !(o->eta > 0)) throw TgmsError{TGMS_E_INVAL, "bad tolerance or eta"};
    if (o->overlap < 1) throw TgmsError{TGMS_E_INVAL, "overlap must be at least 1"};
    if (o->precision != 0 || o->warm_start != 0 || o->smooth_steps != 1 || o->additive != 0)
        throw TgmsError{TGMS_E_UNSUPPORTED,
                        "on the cube: FP64 only, no warm start, one pre- and one post-smoothing, multiplicative cycle"};
    if (o->coarse_space < 0 || o->coarse_space > 2) throw TgmsError{TGMS_E_INVAL, "coarse_space must be 0, 1 or 2"};
    for (int a = 0; a < 3; ++a) {
        if (n[a] / b[a] < 2) throw TgmsError{TGMS_E_UNSUPPORTED, "need at least 2 blocks per axis"};
        if (o->overlap > b[a]) throw TgmsError{TGMS_E_UNSUPPORTED, "overlap larger than a block"};
        if (std::min(b[a] + 2 * o->overlap, n[a]) > MAXE) throw TgmsError{TGMS_E_UNSUPPORTED, "patches wider than 32 cells"};
    }
    const int J[3] = {b[1] * b[2], b[0] * b[2], b[0] * b[1]};
    if (std::max(J[0], std::max(J[1], J[2])) > JM)
        throw TgmsError{TGMS_E_UNSUPPORTED, "a coarse face with more than 64 fine faces"};
    auto t_all = std::chrono::steady_clock::now();
    auto* d = new Ctx3();
    c->d3 = d;
    c->dim = 3;
    G3& g = d->g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.h[a] = 1.0 / n[a];
    }
    g.vol = g.h[0] * g.h[1] * g.h[2];
    g.foff[0] = 0;
    g.foff[1] = (long long)(n[0] + 1) * n[1] * n[2];
    g.foff[2] = g.foff[1] + (long long)n[0] * (n[1] + 1) * n[2];
    g.nf = g.foff[2] + (long long)n[0] * n[1] * (n[2] + 1);
    g.nc = (long long)n[0] * n[1] * n[2];
    auto boxes = [&](int ov) {
        Boxes B;
        for (int a = 0; a < 3; ++a) {
            B.b[a] = b[a];
            B.N[a] = n[a] / b[a];
            B.E[a] = std::min(b[a] + 2 * ov, n[a]);
        }
        B.ov = ov;
        B.n = B.E[0] * B.E[1] * B.E[2];
        B.nfc = closure_faces(B.E);
        B.count = B.N[0] * B.N[1] * B.N[2];
        return B;
    };
    d->blk = boxes(0);
    d->pat = boxes(o->overlap);
    d->nblk = d->blk.count;
    for (int a = 0; a < 3; ++a) d->Jax[a] = J[a];
    d->Jmax = std::max(J[0], std::max(J[1], J[2]));
    d->eta = o->eta;
    d->s_scale = o->s_scale > 0 ? o->s_scale : std::cbrt(b[0] * g.h[0] * b[1] * g.h[1] * b[2] * g.h[2]);
    d->tol = eig_tol;
    d->coarse_space = o->coarse_space;
    c->eta = o->eta;
    c->tol = eig_tol;
    c->overlap = o->overlap;
    c->precision = 0;
    c->coarse_space = o->coarse_space;
    {
        int dev = 0, v = 0;
        HIP_OK(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            c->lds_max = v;
    }
    if (box_lds(d->pat) > (size_t)c->lds_max)
        throw TgmsError{TGMS_E_UNSUPPORTED, "smoother patches too large for the LDS of one workgroup"};
    // coarse faces in the order x, y, z, each by (I2, I1, I0), I the block on the high side
    std::vector<int> cf, slot((size_t)d->nblk * 6, -1);
    const int* N = d->blk.N;
    for (int a = 0; a < 3; ++a)
        for (int i2 = 0; i2 < N[2]; ++i2)
            for (int i1 = 0; i1 < N[1]; ++i1)
                for (int i0 = 0; i0 < N[0]; ++i0) {
                    const int I[3] = {i0, i1, i2};
                    if (I[a] < 1) continue;
                    const int E = (int)(cf.size() / 4);
                    cf.insert(cf.end(), {a, i0, i1, i2});
                    int I1[3] = {i0, i1, i2};
                    I1[a] -= 1;
                    const int K1 = (I1[2] * N[1] + I1[1]) * N[0] + I1[0], K2 = (i2 * N[1] + i1) * N[0] + i0;
                    slot[(size_t)K1 * 6 + 2 * a + 1] = E;
                    slot[(size_t)K2 * 6 + 2 * a] = E;
                }
    d->ne = (int)(cf.size() / 4);
    c->ne = d->ne;
    c->nblk = d->nblk;
    c->nx = n[0];
    c->ny = n[1];
    c->bx = b[0];
    c->by = b[1];
    c->jmax = d->Jmax;
    d->cf = c->alloc<int>(cf.size());
    d->slot = c->alloc<int>(slot.size());
    HIP_OK(hipMemcpyAsync(d->cf, cf.data(), sizeof(int) * cf.size(), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(d->slot, slot.data(), sizeof(int) * slot.size(), hipMemcpyHostToDevice, c->stream));
    d->part = c->alloc<double>(NPART);
    // cell weights
    d->w = c->alloc<double>(g.nc);
    d->kinv = c->alloc<double>(g.nc);
    {
        int* bad = c->alloc<int>(1);
        hipLaunchKernelGGL(k3_weights, dim3(nblocks(g.nc)), dim3(NT3), 0, c->stream, kappa, g.nc, g.vol, d->w, d->kinv,
                           bad);
        LAUNCH_OK();
        int hbad = 0;
        HIP_OK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        if (hbad) throw TgmsError{TGMS_E_INVAL, "permeability must be finite and positive"};
    }
    // local Schur inverses of the blocks and the smoother patches
    auto t0 = std::chrono::steady_clock::now();
    d->Sblk = c->alloc<double>((size_t)d->nblk * d->blk.n * d->blk.n);
    d->Spat = c->alloc<double>((size_t)d->nblk * d->pat.n * d->pat.n);
    factor_boxes(c, d, d->blk, d->Sblk);
    HIP_OK(hipStreamSynchronize(c->stream));
    const double t_blk = ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    factor_boxes(c, d, d->pat, d->Spat);
    HIP_OK(hipStreamSynchronize(c->stream));
    d->t_smoother_ms = ms_since(t0);
    // the coarse space
    const int Jm = d->Jmax, ncol = 6 * Jm;
    const Boxes& B = d->blk;
    d->eigs = c->alloc<double>((size_t)d->ne * Jm);
    d->counts = c->alloc<int>(d->ne);
    d->Y = c->alloc<double>((size_t)d->ne * Jm * Jm);
    int* eig_bad = c->alloc<int>(1);
    t0 = std::chrono::steady_clock::now();
    if (d->coarse_space == 2) {
        hipLaunchKernelGGL(k3_unit_Y, dim3(nblocks((long long)d->ne * Jm)), dim3(NT3), 0, c->stream,
                           (const int*)d->cf, B, Jm, d->ne, d->Y, d->counts);
        LAUNCH_OK();
        d->cmax = 1;
        d->W = c->alloc<double>((size_t)d->nblk * B.nfc * 6);
        hipLaunchKernelGGL(k3_rt0_basis, dim3(nblocks(B.nfc), d->nblk), dim3(NT3), 0, c->stream, B,
                           (const int*)d->slot, d->W);
        LAUNCH_OK();
        HIP_OK(hipStreamSynchronize(c->stream));
        d->counts_h.assign(d->ne, 1);
        d->eigs_h.assign((size_t)d->ne * Jm, 0.0);
    } else {
        // snapshots: H = B A^{-1} f - g + mu, P = S^{-1} H, then v = A^{-1} (f - B^T p)
        const size_t hsz = (size_t)d->nblk * B.n * ncol, csz = (size_t)d->nblk * B.nfc * ncol;
        Tmp C(sizeof(double) * csz, c->stream);
        {
            Tmp H(sizeof(double) * hsz, c->stream), P(sizeof(double) * hsz, c->stream);
            hipLaunchKernelGGL(k3_snap_rhs, dim3(d->nblk, (ncol + 63) / 64), dim3(64), 0, c->stream, B, g,
                               (const double*)d->w, (const int*)d->slot, Jm, H.as<double>());
            LAUNCH_OK();
            tgms::gemm_batched(c, 0, 0, B.n, ncol, B.n, 1.0, d->Sblk, B.n,
                               tgms::Strided{(long long)B.n * B.n, 0, 1}, H.as<double>(), ncol,
                               tgms::Strided{(long long)B.n * ncol, 0, 1}, 0.0, P.as<double>(), ncol,
                               tgms::Strided{(long long)B.n * ncol, 0, 1}, d->nblk);
            hipLaunchKernelGGL(k3_snap_finish, dim3(d->nblk, (ncol + 63) / 64), dim3(64), 0, c->stream, B, g,
                               (const double*)d->w, (const int*)d->slot, Jm, (const double*)P.as<double>(),
                               C.as<double>());
            LAUNCH_OK();
            HIP_OK(hipStreamSynchronize(c->stream));
        }
        d->t_snap_ms = ms_since(t0) + t_blk;
        t0 = std::chrono::steady_clock::now();
        // the Gram matrices of each side's snapshots, then the pencils and their eigenpairs
        Tmp G(sizeof(double) * (size_t)d->nblk * 6 * Jm * Jm, c->stream);
        {
            Tmp Z(sizeof(double) * csz, c->stream);
            hipLaunchKernelGGL(k3_closure_A, dim3(nblocks((long long)B.nfc * ncol), d->nblk), dim3(NT3), 0, c->stream,
                               B, g, (const double*)d->w, (const double*)C.as<double>(), ncol, Z.as<double>());
            LAUNCH_OK();
            tgms::gemm_batched(c, 1, 0, Jm, Jm, B.nfc, 1.0, C.as<double>(), ncol,
                               tgms::Strided{(long long)B.nfc * ncol, Jm, 6}, Z.as<double>(), ncol,
                               tgms::Strided{(long long)B.nfc * ncol, Jm, 6}, 0.0, G.as<double>(), Jm,
                               tgms::Strided{6ll * Jm * Jm, (long long)Jm * Jm, 6}, (long long)d->nblk * 6);
            HIP_OK(hipStreamSynchronize(c->stream));
        }
        int* force = nullptr;
        if (o->force_counts) {
            for (int E = 0; E < d->ne; ++E) {
                const int l = o->force_counts[E];
                if (l < 1 || l > J[cf[E * 4]]) throw TgmsError{TGMS_E_INVAL, "force_counts entries must lie in [1, J_i]"};
            }
            force = c->alloc<int>(d->ne);
            HIP_OK(hipMemcpyAsync(force, o->force_counts, sizeof(int) * d->ne, hipMemcpyHostToDevice, c->stream));
        }
        hipLaunchKernelGGL(k3_pencil_eig, dim3(d->ne), dim3(64), 0, c->stream, B, g, (const int*)d->cf, Jm,
                           (const double*)G.as<double>(), (const double*)d->kinv, eig_tol, 1.0 / d->s_scale,
                           (const int*)force, d->coarse_space == 1 ? 1 : 0, d->eigs, d->counts, d->Y, eig_bad);
        LAUNCH_OK();
        d->counts_h.resize(d->ne);
        d->eigs_h.resize((size_t)d->ne * Jm);
        HIP_OK(hipMemcpyAsync(d->counts_h.data(), d->counts, sizeof(int) * d->ne, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipMemcpyAsync(d->eigs_h.data(), d->eigs, sizeof(double) * d->eigs_h.size(), hipMemcpyDeviceToHost,
                              c->stream));
        int hbad = 0;
        HIP_OK(hipMemcpyAsync(&hbad, eig_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        c->eig_unconverged = hbad;
        d->t_eig_ms = ms_since(t0);
        t0 = std::chrono::steady_clock::now();
        d->cmax = *std::max_element(d->counts_h.begin(), d->counts_h.end());
        // the basis on the block closures: W[K][:, s cmax + k] = C_s Y_{E(K, s)}[:, k]
        Tmp Ys(sizeof(double) * (size_t)d->nblk * 6 * Jm * d->cmax, c->stream);
        hipLaunchKernelGGL(k3_gather_Y, dim3(nblocks((long long)d->nblk * 6 * Jm * d->cmax)), dim3(NT3), 0, c->stream,
                           (const int*)d->slot, (const double*)d->Y, Jm, d->cmax, d->nblk, Ys.as<double>());
        LAUNCH_OK();
        const int m = 6 * d->cmax;
        d->W = c->alloc<double>((size_t)d->nblk * B.nfc * m);
        tgms::gemm_batched(c, 0, 0, B.nfc, d->cmax, Jm, 1.0, C.as<double>(), ncol,
                           tgms::Strided{(long long)B.nfc * ncol, Jm, 6}, Ys.as<double>(), d->cmax,
                           tgms::Strided{6ll * Jm * d->cmax, (long long)Jm * d->cmax, 6}, 0.0, d->W, m,
                           tgms::Strided{(long long)B.nfc * m, d->cmax, 6}, (long long)d->nblk * 6);
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    // coarse unknown numbering
    {
        std::vector<int> off(d->ne + 1, 0);
        for (int E = 0; E < d->ne; ++E) off[E + 1] = off[E] + d->counts_h[E];
        d->nu = off[d->ne];
        d->fnoff = c->alloc<int>(d->ne + 1);
        HIP_OK(hipMemcpyAsync(d->fnoff, off.data(), sizeof(int) * (d->ne + 1), hipMemcpyHostToDevice, c->stream));
        c->counts_h = d->counts_h;
    }
    build_coarse(c, d);
    d->t_coarse_ms = ms_since(t0);
    build_rt0(c, d);
    dct_matrices(c, d);
    // solve workspaces
    const long long nf = g.nf;
    for (double** v : {&d->vbar, &d->vx, &d->vr, &d->vz, &d->vp, &d->vq, &d->vt, &d->vt2, &d->vrold})
        *v = c->alloc<double>(nf);
    d->patch_out = c->alloc<double>((size_t)d->nblk * d->pat.nfc);
    d->cbk = c->alloc<double>((size_t)d->nblk * 6 * d->cmax);
    d->cb = c->alloc<double>(d->nu);
    d->cz = c->alloc<double>(d->nu);
    d->cell1 = c->alloc<double>(g.nc);
    d->cell2 = c->alloc<double>(g.nc);
    d->gK = c->alloc<double>(d->nblk);
    d->vH = c->alloc<double>(d->ne);
    HIP_OK(hipStreamSynchronize(c->stream));
    c->t_snap_ms = d->t_snap_ms;
    c->t_eig_ms = d->t_eig_ms;
    c->t_coarse_ms = d->t_coarse_ms;
    c->t_smoother_ms = d->t_smoother_ms;
    c->t_setup_ms = ms_since(t_all);
}

void update_mobility3(tgms_ctx* c, const double* lambda) {
    Ctx3* d = c->d3;
    int* bad = c->alloc_scratch_int();
    Tmp wn(sizeof(double) * d->g.nc, c->stream);
    hipLaunchKernelGGL(k3_mob_weights, dim3(nblocks(d->g.nc)), dim3(NT3), 0, c->stream, (const double*)d->kinv, lambda,
                       d->g.nc, d->g.vol, wn.as<double>(), bad);
    LAUNCH_OK();
    int hbad = 0;
    HIP_OK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (hbad) throw TgmsError{TGMS_E_INVAL, "mobility must be finite and positive"};
    tgms::copy(c, d->g.nc, wn.as<double>(), d->w);
    factor_boxes(c, d, d->blk, d->Sblk);
    factor_boxes(c, d, d->pat, d->Spat);
    build_coarse(c, d);
    build_rt0(c, d);
    c->mobility_updated = true;
}

void solve3(tgms_ctx* c, const double* F, double rtol, int maxit, double* u, double* p, int* iters, double* relres,
            tgms_status* st) {
    Ctx3* d = c->d3;
    const long long nf = d->g.nf;
    const unsigned gb = nblocks(nf);
    preprocess(c, d, F, d->vbar);
    // b = -A vbar; PCG from x = 0 with the residual projected onto ker B after every
    // update.  The preconditioner only sees the divergence-free part of r in exact
    // arithmetic, but r also carries an O(|r_0|) pressure-gradient part that does not
    // shrink; the local solves through explicit Schur inverses would cancel it only to
    // about eps cond(S) of its size, which swamps the shrinking divergence-free part.
    applyA(c, d, d->vbar, d->vq);
    tgms::zero(c, d->vr, sizeof(double) * nf);
    tgms::axpy(c, nf, -1.0, d->vq, d->vr);
    project(c, d, d->vr);
    tgms::zero(c, d->vx, sizeof(double) * nf);
    twogrid(c, d, d->vr, d->vz);
    repair_divergence(c, d, d->vz);
    const double z0 = std::sqrt(dot3(c, d, d->vz, d->vz, nf));
    c->alphas.clear();
    c->betas.clear();
    int it = 0;
    double rel = 1.0;
    *st = TGMS_OK;
    if (z0 > 0.0) {
        tgms::copy(c, nf, d->vz, d->vp);
        double rho = dot3(c, d, d->vr, d->vz, nf);
        while (it < maxit) {
            applyA(c, d, d->vp, d->vq);
            const double pq = dot3(c, d, d->vp, d->vq, nf);
            if (!(pq > 0.0)) {
                *st = TGMS_E_BREAKDOWN;
                break;
            }
            const double alpha = rho / pq;
            tgms::axpy(c, nf, alpha, d->vp, d->vx);
            tgms::axpy(c, nf, -alpha, d->vq, d->vr);
            project(c, d, d->vr);
            twogrid(c, d, d->vr, d->vz);
            repair_divergence(c, d, d->vz);
            ++it;
            c->alphas.push_back(alpha);
            rel = std::sqrt(dot3(c, d, d->vz, d->vz, nf)) / z0;
            if (rel <= rtol) break;
            const double rho_new = dot3(c, d, d->vr, d->vz, nf);
            const double beta = rho_new / rho;
            c->betas.push_back(beta);
            hipLaunchKernelGGL(k3_xpby, dim3(gb), dim3(NT3), 0, c->stream, (const double*)d->vz, beta, d->vp, nf);
            LAUNCH_OK();
            rho = rho_new;
        }
        if (*st == TGMS_OK && rel > rtol) *st = TGMS_E_NOTCONV;
    } else {
        rel = 0.0;
    }
    tgms::copy(c, nf, d->vbar, u);
    tgms::axpy(c, nf, 1.0, d->vx, u);
    if (p) pressure(c, d, u, p);
    HIP_OK(hipStreamSynchronize(c->stream));
    if (iters) *iters = it;
    if (relres) *relres = rel;
}

void apply_A3(tgms_ctx* c, const double* x, double* y) {
    applyA(c, c->d3, x, y);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void preprocess3(tgms_ctx* c, const double* F, double* vbar) {
    preprocess(c, c->d3, F, vbar);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void apply_precond3(tgms_ctx* c, int which, const double* r, double* z) {
    Ctx3* d = c->d3;
    // every step reads r on the interior faces only
    if (which == 0)
        smooth(c, d, r, z);
    else if (which == 1)
        coarse(c, d, r, z);
    else
        twogrid(c, d, r, z);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void smooth_patches3(tgms_ctx* c) {
    Ctx3* d = c->d3;
    hipLaunchKernelGGL(k3_box_solve, dim3(d->pat.count), dim3(NT3), box_lds(d->pat), c->stream, d->pat, d->g,
                       (const double*)d->w, (const double*)d->Spat, (const double*)d->vr, 1.0, (const double*)nullptr,
                       d->patch_out, (double*)nullptr);
    LAUNCH_OK();
}

void destroy3(tgms_ctx* c) {
    delete c->d3;
    c->d3 = nullptr;
}

}  // namespace tgms3
