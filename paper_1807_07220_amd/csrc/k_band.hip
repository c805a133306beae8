// Local direct solvers on the coarse blocks K_i (preprocessing and snapshots,
// paper sections 3 and 4.1).
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

// One wavefront per rectangle; band matrix in LDS (n * (b+1) doubles, then m * m for the
// diagonal blocks' inverses).  NQ: pairs of the trailing update per lane
// (ceil(b (b+1) / 2 / 64)).
template <bool WRITE32, int NQ>
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
    // right-looking band Cholesky; the pairs (u, t') of a column's trailing update
    // (u = 1..b, t' = 0..b-u, enumerated column by column) this lane handles, decoded once
    const int npair = b * (b + 1) / 2;
    int pu[NQ], pt[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        int u = 1, rem = lane + TGMS_WAVE * q;
        if (rem < npair) {
            while (rem > b - u) {
                rem -= b - u + 1;
                ++u;
            }
        } else {
            u = 0;  // no pair
        }
        pu[q] = u;
        pt[q] = rem;
    }
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
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int u = pu[q], tp = pt[q];
            if (u > 0 && cidx + u + tp < n) M[(long long)(cidx + u) * ld + tp] -= col[u] * col[u + tp];
        }
        __syncthreads();
        if (lane == 0) col[0] = inv;
        __syncthreads();
    }
    // repack by vertex rows: D_j = L_jj^{-1} (lower, by columns), E_j = L_{j+1,j} (Hessenberg, by columns);
    // each column of L_jj^{-1} is formed in LDS (X, m words a lane) and written out as it goes
    const int tri = btri_tri(m), bs = tri + btri_hes(m);
    double* out = Lpool + R.off;
    double* X = M + (long long)n * ld;
    for (int j = 0; j < mh; ++j) {
        double* D = out + (long long)j * bs;
        if (lane < m) {
            const int cc = lane;  // column of L_jj^{-1}: solve L_jj x = e_cc, rows cc..m-1
            double* xc = X + (long long)cc * m;
            for (int r = cc; r < m; ++r) {
                double acc = (r == cc) ? 1.0 : 0.0;
                for (int k = cc; k < r; ++k) acc -= M[(long long)(j * m + k) * ld + (r - k)] * xc[k];
                // diagonal of L stored as its reciprocal
                const double xr = acc * M[(long long)(j * m + r) * ld];
                xc[r] = xr;
                D[btri_offD(cc, m) + (r - cc)] = xr;
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

}  // namespace

namespace tgms {

// fail_out: a zeroed device flag that a failed factorisation sets, checked by the
// caller later (null: checked here, after waiting)
static void factor_rects(tgms_ctx* c, Rect* rects, int count, int max_n, int max_b, double* L, double* S,
                         int* fail_out) {
    // the band and the columns of one diagonal block's inverse
    size_t lds = ((size_t)max_n * (max_b + 1) + (size_t)(max_b - 1) * (max_b - 1)) * sizeof(double);
    if (lds > 65536) throw TgmsError{TGMS_E_UNSUPPORTED, "local band factor exceeds 64 KiB of LDS"};
    int* fail = fail_out ? fail_out : c->alloc_scratch_int();
    if (max_b - 1 > TGMS_MMAX) throw TgmsError{TGMS_E_UNSUPPORTED, "local rectangle wider than 33 cells"};
    const int npair = max_b * (max_b + 1) / 2;
    float* L32 = nullptr;
    if (npair <= 3 * TGMS_WAVE)
        hipLaunchKernelGGL((k_band_factor<false, 3>), dim3(count), dim3(TGMS_WAVE), lds, c->stream, rects, c->a,
                           c->nx, c->sx * c->sx, c->sy * c->sy, L, S, L32, fail);
    else
        hipLaunchKernelGGL((k_band_factor<false, (34 * 35 / 2 + TGMS_WAVE - 1) / TGMS_WAVE>), dim3(count),
                           dim3(TGMS_WAVE), lds, c->stream, rects, c->a, c->nx, c->sx * c->sx, c->sy * c->sy, L, S,
                           L32, fail);
    LAUNCH_OK();
    if (fail_out) return;
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (h) throw TgmsError{TGMS_E_INVAL, "local stream-function matrix is not positive definite"};
}

void factor_blocks(tgms_ctx* c, int* fail) {
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
    if (!c->blk_rects) {
        c->blk_rects = c->alloc<Rect>(c->nblk);
        HIP_OK(hipMemcpyAsync(c->blk_rects, r.data(), sizeof(Rect) * c->nblk, hipMemcpyHostToDevice, c->stream));
    }
    factor_rects(c, c->blk_rects, c->nblk, c->blk_n, c->blk_b, c->blkL, c->blkS, fail);
}


}  // namespace tgms
