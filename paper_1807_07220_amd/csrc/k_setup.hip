// Adaptive spectral coarse space (paper section 4) and the coarse correction
// (eq. coarsepre).
//
// Snapshots (section 4.1, eq. snapshot_eqn) are computed per coarse block K:
// for every interior side E of K and every fine face e_l of E, the local
// mixed problem with v.n = delta_l on E, zero flux on the rest of dK and
// constant divergence (outward flux / |K|) is solved as
//     v = v_p + C_K psi,  (C_K^T A_K C_K) psi = -C_K^T A_K v_p,
// where v_p is an explicit particular flux with the right boundary flux and
// divergence, and psi lives on K's interior vertices (band factor of
// k_band.hip).  The snapshot of face E_i on omega_i is the pair of K1 and K2
// solutions sharing delta_l on E_i.
//
// The spectral pencil (section 4.2, eq. spectral_eqn) of E_i is assembled
// from the block Gram matrices G_K = Psi_K^T A_K Psi_K of its two blocks plus
// the divergence term sum_K |e_l||e_m|/|K|, scaled by 1/H; the a-form is
// diagonal, D_ll = |e_l| (kappa_L^{-1} + kappa_R^{-1})/2.  T = D^{-1/2} S
// D^{-1/2} is diagonalised by cyclic Jacobi; lambda = 1/mu ascending and the
// first max(1, #{lambda < tol}) modes are kept.
//
// The coarse problem is restricted to its divergence-free subspace, spanned
// by (i) the zero-net-flux combinations of each face's modes and (ii) for each
// interior coarse vertex the coarse-curl combination of the unit-flux
// "carriers" of the four faces meeting there.  Its SPD matrix is the
// divergence-free part of L_H; the coarse correction is
// P = W (Z^T A Z)^{-1} W^T in stream-function coordinates, W holding the
// stream functions of those basis fields on each block's vertices.
#include "common.h"
#include "band.h"
#include "block.h"
#include "jacobi.h"

namespace {

struct BlockGeom {
    int nx, ny, bx, by, Nx, Ny, jmax, nfk, ncol;
    double hx, hy, sx, sy;
};

// Snapshots: one wavefront per block, columns (side s, fine face l) in turn.
template <int MW>
__global__ void __launch_bounds__(64) k_snapshots(BlockGeom G, const double* __restrict__ a, const double* __restrict__ blkL,
                            const double* __restrict__ blkS, double* __restrict__ Psi) {
    extern __shared__ double sm[];
    const int bxl = G.bx, byl = G.by;
    const int nfx = byl * (bxl + 1), nfy = (byl + 1) * bxl, nloc = (bxl - 1) * (byl - 1);
    double* Fw = sm;
    double* Fe = Fw + byl;
    double* Fs = Fe + byl;
    double* Fn = Fs + bxl;
    double* q = Fn + bxl;
    double* vx = q + bxl * byl;
    double* vy = vx + nfx;
    double* ox = vy + nfy;
    double* oy = ox + nfx;
    double* g = oy + nfy;
    double* tmp = g + nloc;
    double* tb = tmp + byl + 2;
    double* xb = tb + 64;
    const int blk = blockIdx.x, I = blk % G.Nx, J = blk / G.Nx;
    const int lane = threadIdx.x;
    const double* aK = a + (long long)J * G.by * G.nx + (long long)I * G.bx;
    const double areaK = G.bx * G.hx * G.by * G.hy;
    const double* L = blkL + (long long)blk * btri_size(bxl - 1, byl - 1);
    double* out = Psi + (long long)blk * G.ncol * G.nfk;
    for (int s = 0; s < 4; ++s) {
        const bool interior = (s == 0 && I > 0) || (s == 1 && I < G.Nx - 1) || (s == 2 && J > 0) ||
                              (s == 3 && J < G.Ny - 1);
        const int nl = (s < 2) ? byl : bxl;
        for (int l = 0; l < G.jmax; ++l) {
            double* col = out + (long long)(s * G.jmax + l) * G.nfk;
            if (!interior || l >= nl) {
                for (int e = lane; e < G.nfk; e += 64) col[e] = 0.0;
                continue;
            }
            // boundary flux delta_l on side s (velocity 1 in the +axis direction)
            for (int e = lane; e < 2 * byl + 2 * bxl; e += 64) Fw[e] = 0.0;
            __syncthreads();
            const double elen = (s < 2) ? G.hy : G.hx;
            double outflow;
            if (lane == 0) {
                if (s == 0) Fw[l] = elen;
                if (s == 1) Fe[l] = elen;
                if (s == 2) Fs[l] = elen;
                if (s == 3) Fn[l] = elen;
            }
            outflow = (s == 1 || s == 3) ? elen : -elen;
            const double qc = outflow / (bxl * byl);  // alpha |c| = outward flux / |K| * |c|
            for (int e = lane; e < bxl * byl; e += 64) q[e] = qc;
            __syncthreads();
            particular_flux(bxl, byl, Fw, Fe, Fs, Fn, q, vx, vy, tmp);
            for (int e = lane; e < nfx; e += 64) vx[e] *= 1.0 / G.hy;
            for (int e = lane; e < nfy; e += 64) vy[e] *= 1.0 / G.hx;
            __syncthreads();
            block_mass(bxl, byl, aK, G.nx, vx, vy, ox, oy);
            block_curlT(bxl, byl, ox, oy, G.sx, G.sy, -1.0, g);
            btri_solve_wave<double, MW>(L, bxl - 1, byl - 1, g, tb, xb);
            __syncthreads();
            block_curl_add(bxl, byl, g, G.sx, G.sy, vx, vy);
            for (int e = lane; e < nfx; e += 64) col[e] = vx[e];
            for (int e = lane; e < nfy; e += 64) col[nfx + e] = vy[e];
            __syncthreads();
        }
    }
}

// Snapshots with one lane per snapshot column (4*jmax <= 64 columns, one wavefront
// per block).  The explicit particular flux of column (side s, fine face l) has a
// closed form: the construction of particular_flux with a single unit boundary
// flux f on side s and the uniform source (outward flux)/|K| gives
//   s = 0 (west, row l):  Fx = f (1 - a/bx) on row l,  Fy(b) = (-b f/by + [b > l] f)/bx
//   s = 1 (east, row l):  Fx = f a/bx on row l,        Fy(b) = (b f/by - [b > l] f)/bx
//   s = 2 (south, col l): Fx(0, a) = -a f/bx + [a > l] f, Fy(0, a) = [a == l] f,
//                         Fy(b) = f (1 - b/by)/bx (0 < b < by)
//   s = 3 (north, col l): Fx(by-1, a) = a f/bx - [a > l] f, Fy(by, a) = [a == l] f,
//                         Fy(b) = b f/(by bx) (0 < b < by)
// (fluxes; every other entry zero).  Any particular flux gives the same snapshot.
// The block's band factor, its cell weights and the 64 right-hand sides /
// solutions ([vertex][column]) live in LDS; each lane runs the block-row sweeps
// of band.h on its own column with the factor entries read as broadcasts.
// The closed forms above, branch-free per lane: the x-fluxes are nonzero on one
// row xr only, Fx(xr, a) = c0 + c1 a + [a > l] c2; interior y-fluxes are uniform
// along a row, Fy(b) = d0 + d1 b + [b > l] d2; the boundary rows carry f at a = l
// on the south (s = 2) or north (s = 3) side.
struct SnapCol {
    int l, xr, by;
    double c0, c1, c2, d0, d1, d2, fs, fn;  // fs, fn: flux at a = l on rows 0 and by
    __device__ void init(int s, int ll, int bx, int byy, double f) {
        l = ll;
        by = byy;
        const double fb = f / bx, fbb = f / ((double)bx * byy);
        xr = s == 0 || s == 1 ? ll : (s == 2 ? 0 : byy - 1);
        c0 = s == 0 ? f : 0.0;
        c1 = (s == 0 || s == 2) ? -fb : fb;
        c2 = s == 2 ? f : (s == 3 ? -f : 0.0);
        d0 = s == 2 ? fb : 0.0;
        d1 = (s == 0 || s == 2) ? -fbb : fbb;
        d2 = s == 0 ? fb : (s == 1 ? -fb : 0.0);
        fs = s == 2 ? f : 0.0;
        fn = s == 3 ? f : 0.0;
    }
    __device__ double Fx(int b, int a) const { return b == xr ? c0 + c1 * a + (a > l ? c2 : 0.0) : 0.0; }
    __device__ double Fy(int b, int a) const {
        if (b == 0) return a == l ? fs : 0.0;
        if (b == by) return a == l ? fn : 0.0;
        return d0 + d1 * b + (b > l ? d2 : 0.0);
    }
};

template <int M, bool VGLOBAL>
__global__ void __launch_bounds__(64) k_snapshots_cols(BlockGeom G, const double* __restrict__ a,
                                                       const double* __restrict__ blkL, double* __restrict__ Psi,
                                                       double* __restrict__ Vg, long long vstride) {
    extern __shared__ __align__(16) double sm[];
    constexpr int TILE = 32;  // faces per transposed output chunk
    const int bx = G.bx, by = G.by;
    const int m = M, mh = by - 1, nloc = m * mh;
    const int tri = btri_tri(m), bs = tri + btri_hes(m);
    const long long fsz = btri_size(m, mh);
    // LDS: the output transpose tile [TILE][64] (without VGLOBAL, the band factor first,
    // in the same region) and the cell weights [by][bx].  With VGLOBAL the right-hand
    // sides / solutions [vertex][64] live in a global scratch of vstride doubles per
    // block and the factor is read from global memory (the same entry in every lane:
    // scalar loads), so that a workgroup's LDS is small and several share a CU.
    const int areg = VGLOBAL ? TILE * 64 : (int)((fsz > TILE * 64 ? fsz : TILE * 64) + 1) & ~1;
    double* Tt = sm;
    double* aK = sm + areg;
    double* V = VGLOBAL ? Vg + (long long)blockIdx.x * vstride : aK + bx * by + 1;
    const int blk = blockIdx.x, I = blk % G.Nx, J = blk / G.Nx;
    const int lane = threadIdx.x;
    const double* F = VGLOBAL ? blkL + (long long)blk * fsz : sm;
    {
        if (!VGLOBAL) {
            const double* src = blkL + (long long)blk * fsz;
            for (long long e = lane; e < fsz; e += 64) sm[e] = src[e];
        }
        for (int e = lane; e < bx * by; e += 64)
            aK[e] = a[(long long)(J * by + e / bx) * G.nx + I * bx + e % bx];
    }
    __syncthreads();
    // this lane's column: side s, fine face l (an all-zero column when the side is on dD
    // or the side has fewer than l+1 fine faces)
    const int side = lane / G.jmax, fl = lane % G.jmax;
    const bool valid = lane < G.ncol &&
                       ((side == 0 && I > 0) || (side == 1 && I < G.Nx - 1) || (side == 2 && J > 0) ||
                        (side == 3 && J < G.Ny - 1)) &&
                       fl < (side < 2 ? by : bx);
    SnapCol col;
    col.init(side < 4 ? side : 3, fl, bx, by, valid ? (side < 2 ? G.hy : G.hx) : 0.0);
    const double c3 = 1.0 / 3.0, c6 = 1.0 / 6.0, ihx = 1.0 / G.hx, ihy = 1.0 / G.hy;
    auto vx = [&](int b, int aa) { return col.Fx(b, aa) * ihy; };
    auto vy = [&](int b, int aa) { return col.Fy(b, aa) * ihx; };
    auto AK = [&](int b, int aa) { return aK[b * bx + aa]; };
    auto wy = [&](int b, int aa) {  // (A v_p) on y-face (b, aa), 0 < b < by
        return AK(b - 1, aa) * (vy(b, aa) * c3 + vy(b - 1, aa) * c6) + AK(b, aa) * (vy(b, aa) * c3 + vy(b + 1, aa) * c6);
    };
    auto wxr = [&](int aa) {  // (A v_p) on x-face (xr, aa), 0 < aa < bx (zero on every other row)
        const int b = col.xr;
        return AK(b, aa - 1) * (vx(b, aa) * c3 + vx(b, aa - 1) * c6) + AK(b, aa) * (vx(b, aa) * c3 + vx(b, aa + 1) * c6);
    };
    // g = -C_K^T A_K v_p on the interior vertices (p, q), p = 1..bx-1, q = 1..by-1
    for (int q = 1; q < by; ++q) {
        double wprev = wy(q, 0);
        for (int p = 1; p < bx; ++p) {
            const double wcur = wy(q, p);
            double xpart = 0.0;
            if (q - 1 == col.xr) xpart += wxr(p);
            if (q == col.xr) xpart -= wxr(p);
            V[((q - 1) * m + p - 1) * 64 + lane] = -(G.sx * xpart + G.sy * (wcur - wprev));
            wprev = wcur;
        }
    }
    // psi = (C^T A C)^{-1} g by the block-row sweeps (lane-local; factor entries broadcast)
    const double* S = F + (long long)mh * bs;
    double y[M];
#pragma unroll
    for (int k = 0; k < M; ++k) y[k] = 0.0;
    for (int j = 0; j < mh; ++j) {
        const double* D = F + (long long)j * bs;
        double t[M];
#pragma unroll
        for (int k = 0; k < M; ++k) t[k] = V[(j * m + k) * 64 + lane] * S[j * m + k];
        if (j > 0) {
            const double* E = F + (long long)(j - 1) * bs + tri;
#pragma unroll
            for (int c = 0; c < M; ++c)
#pragma unroll
                for (int k = 0; k <= c + 1 && k < M; ++k) t[k] -= E[btri_offE(c) + k] * y[c];
        }
#pragma unroll
        for (int k = 0; k < M; ++k) y[k] = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int k = c; k < M; ++k) y[k] += D[btri_offD(c, m) + k - c] * t[c];
#pragma unroll
        for (int k = 0; k < M; ++k) V[(j * m + k) * 64 + lane] = y[k];
    }
    double w[M];
#pragma unroll
    for (int k = 0; k < M; ++k) w[k] = 0.0;
    for (int j = mh - 1; j >= 0; --j) {
        const double* D = F + (long long)j * bs;
        double t[M];
#pragma unroll
        for (int k = 0; k < M; ++k) t[k] = V[(j * m + k) * 64 + lane];
        if (j + 1 < mh) {
            const double* E = F + (long long)j * bs + tri;
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int r = 0; r <= k + 1 && r < M; ++r) t[k] -= E[btri_offE(k) + r] * w[r];
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int r = k; r < M; ++r) acc += D[btri_offD(k, m) + r - k] * t[r];
            w[k] = acc;
        }
#pragma unroll
        for (int k = 0; k < M; ++k) V[(j * m + k) * 64 + lane] = w[k] * S[j * m + k];
    }
    __syncthreads();  // the factor region (without VGLOBAL) becomes the output tile
    // v = v_p + C_K psi on all block faces, written column by column in chunks of TILE faces
    auto P = [&](int pp, int qq) -> double {
        return (pp <= 0 || pp >= bx || qq <= 0 || qq >= by) ? 0.0 : V[((qq - 1) * m + pp - 1) * 64 + lane];
    };
    const int nfx = by * (bx + 1), nfk = G.nfk;
    double* out = Psi + (long long)blk * G.ncol * nfk;
    for (int f0 = 0; f0 < nfk; f0 += TILE) {
        for (int k = 0; k < TILE && f0 + k < nfk; ++k) {
            const int e = f0 + k;
            double v;
            if (e < nfx) {
                const int b = e / (bx + 1), aa = e % (bx + 1);
                v = vx(b, aa) + (P(aa, b + 1) - P(aa, b)) * G.sx;
            } else {
                const int e2 = e - nfx, b = e2 / bx, aa = e2 % bx;
                v = vy(b, aa) - (P(aa + 1, b) - P(aa, b)) * G.sy;
            }
            Tt[k * 64 + lane] = v;
        }
        __syncthreads();
        const int nk = (nfk - f0) < TILE ? (nfk - f0) : TILE;
        for (int cidx = 0; cidx < G.ncol; cidx += 2) {
            const int cc = cidx + (lane >> 5), k = lane & 31;
            if (cc < G.ncol && k < nk) out[(long long)cc * nfk + f0 + k] = Tt[k * 64 + cc];
        }
        __syncthreads();
    }
}

// APsi = A_K Psi_K (block-local mass applied to every snapshot column); one wavefront per (block, column).
__global__ void k_apply_AK_cols(BlockGeom G, const double* __restrict__ a, const double* __restrict__ Psi,
                                double* __restrict__ APsi) {
    const int blk = blockIdx.x, colid = blockIdx.y;
    const int I = blk % G.Nx, J = blk / G.Nx;
    const double* aK = a + (long long)J * G.by * G.nx + (long long)I * G.bx;
    const int bxl = G.bx, byl = G.by, nfx = byl * (bxl + 1);
    const double* v = Psi + ((long long)blk * G.ncol + colid) * G.nfk;
    double* o = APsi + ((long long)blk * G.ncol + colid) * G.nfk;
    const double c3 = 1.0 / 3.0, c6 = 1.0 / 6.0;
    for (int e = threadIdx.x; e < G.nfk; e += blockDim.x) {
        double s = 0.0;
        if (e < nfx) {
            const int b = e / (bxl + 1), aa = e % (bxl + 1);
            if (aa > 0) s += aK[(long long)b * G.nx + aa - 1] * (v[e] * c3 + v[e - 1] * c6);
            if (aa < bxl) s += aK[(long long)b * G.nx + aa] * (v[e] * c3 + v[e + 1] * c6);
        } else {
            const int f = e - nfx, b = f / bxl, aa = f % bxl;
            if (b > 0) s += aK[(long long)(b - 1) * G.nx + aa] * (v[e] * c3 + v[e - bxl] * c6);
            if (b < byl) s += aK[(long long)b * G.nx + aa] * (v[e] * c3 + v[e + bxl] * c6);
        }
        o[e] = s;
    }
}

// G_K = Psi_K^T (A_K Psi_K): one workgroup of (ncol/4)^2 threads per block, 4 x 4 outputs per thread.
__global__ void k_gram(BlockGeom G, const double* __restrict__ Psi, const double* __restrict__ APsi,
                       double* __restrict__ Gout) {
    constexpr int FC = 32;
    extern __shared__ double sm[];
    const int ncol = G.ncol, q4 = ncol / 4;
    double* Ps = sm;                // [ncol][FC]
    double* As = sm + ncol * FC;    // [ncol][FC]
    const int blk = blockIdx.x;
    const double* P = Psi + (long long)blk * ncol * G.nfk;
    const double* AP = APsi + (long long)blk * ncol * G.nfk;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int r0 = (tid / q4) * 4, c0 = (tid % q4) * 4;
    double acc[4][4] = {};
    for (int f0 = 0; f0 < G.nfk; f0 += FC) {
        for (int e = tid; e < ncol * FC; e += nth) {
            const int cc = e / FC, ff = e % FC;
            const bool ok = f0 + ff < G.nfk;
            Ps[e] = ok ? P[(long long)cc * G.nfk + f0 + ff] : 0.0;
            As[e] = ok ? AP[(long long)cc * G.nfk + f0 + ff] : 0.0;
        }
        __syncthreads();
        for (int ff = 0; ff < FC; ++ff) {
            double x[4], y[4];
            for (int r = 0; r < 4; ++r) x[r] = Ps[(r0 + r) * FC + ff];
            for (int s = 0; s < 4; ++s) y[s] = As[(c0 + s) * FC + ff];
            for (int r = 0; r < 4; ++r)
                for (int s = 0; s < 4; ++s) acc[r][s] += x[r] * y[s];
        }
        __syncthreads();
    }
    double* Gb = Gout + (long long)blk * ncol * ncol;
    for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s) Gb[(r0 + r) * ncol + c0 + s] = acc[r][s];
}

// G_K = Psi_K^T A_K Psi_K with FP64 matrix cores (v_mfma_f64_16x16x4): one workgroup
// of four wavefronts per block.  Chunks of FC faces of Psi and of A_K Psi (A_K applied
// while staging: the two-point line stencil of the RT0 mass on the block's faces) go
// to LDS; wavefront w owns NTL*NTL/4 of the 16 x 16 output tiles.  Operand layout of
// the 16x16x4 instruction: lane l holds A[l%16][l/16] and B[l/16][l%16], and element r
// of the result is D[4r + l/16][l%16].
typedef double d4g_t __attribute__((ext_vector_type(4)));
template <int NTL>
__global__ void __launch_bounds__(256) k_gram_mfma(BlockGeom G, const double* __restrict__ a,
                                                   const double* __restrict__ Psi, double* __restrict__ Gout) {
    constexpr int NC = 16 * NTL, FC = 32, TPW = NTL * NTL / 4;
    __shared__ double Ps[NC][FC + 1];
    __shared__ double As[NC][FC + 1];
    const int blk = blockIdx.x, I = blk % G.Nx, J = blk / G.Nx;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int bxl = G.bx, byl = G.by, nfx = byl * (bxl + 1), nfk = G.nfk;
    const double* aK = a + (long long)J * byl * G.nx + (long long)I * bxl;
    const double* P = Psi + (long long)blk * NC * nfk;
    const double c3 = 1.0 / 3.0, c6 = 1.0 / 6.0;
    d4g_t acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = d4g_t{0.0, 0.0, 0.0, 0.0};
    for (int f0 = 0; f0 < nfk; f0 += FC) {
        for (int e = tid; e < NC * FC; e += 256) {
            const int cc = e / FC, ff = e % FC, f = f0 + ff;
            double pv = 0.0, av = 0.0;
            if (f < nfk) {
                const double* v = P + (long long)cc * nfk;
                pv = v[f];
                if (f < nfx) {
                    const int b = f / (bxl + 1), aa = f % (bxl + 1);
                    if (aa > 0) av += aK[(long long)b * G.nx + aa - 1] * (pv * c3 + v[f - 1] * c6);
                    if (aa < bxl) av += aK[(long long)b * G.nx + aa] * (pv * c3 + v[f + 1] * c6);
                } else {
                    const int q = f - nfx, b = q / bxl, aa = q % bxl;
                    if (b > 0) av += aK[(long long)(b - 1) * G.nx + aa] * (pv * c3 + v[f - bxl] * c6);
                    if (b < byl) av += aK[(long long)b * G.nx + aa] * (pv * c3 + v[f + bxl] * c6);
                }
            }
            Ps[cc][ff] = pv;
            As[cc][ff] = av;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < FC; k4 += 4) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int id = wave * TPW + t, ti = id / NTL, tj = id % NTL;
                const double x = Ps[16 * ti + li][k4 + lk];
                const double y = As[16 * tj + li][k4 + lk];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double* Gb = Gout + (long long)blk * NC * NC;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int id = wave * TPW + t, ti = id / NTL, tj = id % NTL;
#pragma unroll
        for (int r = 0; r < 4; ++r) Gb[(16 * ti + 4 * r + lk) * NC + 16 * tj + li] = acc[t][r];
    }
}

// ---- local spectral problems: one wavefront per coarse face --------------------


__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, TGMS_WAVE));
    return v;
}

// Number of eigenvalues of the symmetric n x n matrix T above sigma: the negative
// pivots of the LDL^T factorisation of sigma I - T without pivoting (Sylvester's law of
// inertia), computed in the workspace A (row stride LD); -1 when a pivot is zero
// relative to the largest entry of sigma I - T.
template <int LD>
__device__ int inertia_above(const double (*T)[LD], double* A, int n, double sigma) {
    const int lane = threadIdx.x;
    double mx = 0.0;
    if (lane < n)
        for (int m = 0; m < n; ++m) {
            const double v = (lane == m ? sigma : 0.0) - T[lane][m];
            A[lane * LD + m] = v;
            mx = fmax(mx, fabs(v));
        }
    mx = wave_max(mx);
    __syncthreads();
    int neg = 0;
    for (int j = 0; j < n; ++j) {
        const double d = A[j * LD + j];
        if (fabs(d) <= 1e-14 * mx) return -1;  // the same value in every lane
        neg += d < 0.0;
        if (lane > j && lane < n) {
            const double l = A[lane * LD + j] / d;
            for (int m = j + 1; m < n; ++m) A[lane * LD + m] -= l * A[j * LD + m];
        }
        __syncthreads();
    }
    return neg;
}

constexpr int KW = 8;  // largest warm-start block

// Pencil (eq. spectral_eqn) of every interior coarse face, its eigenproblem and the
// adaptive selection (section 4.2), and the recombination of the kept modes.
//
// WARM = 0: dense cyclic Jacobi on T = D^{-1/2} S D^{-1/2}.  Vtop (optional) receives the
// eigenvectors of T of the 8 largest mu as float [ne][8][jmax] (training targets).
// WARM = 1: Rayleigh-Ritz subspace iteration on T from a block of kblk vectors (Y0
// [ne][8][jmax] as float, or the DCT-II basis when Y0 is null).  With cnt = #{mu > 1/tol}
// from the inertia of 1/tol - T and l = max(1, cnt), a face is accepted at the first
// iteration where l < k, exactly cnt Ritz values exceed 1/tol, the first l Ritz pairs have
// |T u - theta u| / theta <= rq_tol, and (cnt = 0) exactly one eigenvalue lies above
// theta_1 (1 - 4 rq_tol); otherwise the face falls back to the Jacobi solve.  wstat[f]:
// the accepting iteration, or -1 (fallback).  For accepted faces only the first k
// eigenvalues are computed (the rest are stored as 0).
// JM >= jmax: the LDS tiles are sized for the widest face of the grid (several
// workgroups share a CU when the faces are short).
// Geometry of coarse face fid (x-faces first, then y-faces): the blocks K1 (low side) and
// K2 (high side), the snapshot sides s1, s2 of E in each block's column numbering, the
// number of fine faces Jn on E, their length, and the first cells on either side of E
// with the stride along it.
struct FaceGeom {
    int K1, K2, s1, s2, Jn;
    double elen;
    long long cellL, cellR, step;
};
__device__ inline FaceGeom face_geom(const BlockGeom& G, int fid) {
    FaceGeom f;
    const int nex = (G.Nx - 1) * G.Ny;
    if (fid < nex) {  // x-face (I, J), I = 1..Nx-1
        const int J = fid / (G.Nx - 1), I = fid % (G.Nx - 1) + 1;
        f.K1 = J * G.Nx + I - 1;
        f.K2 = J * G.Nx + I;
        f.s1 = 1;
        f.s2 = 0;
        f.Jn = G.by;
        f.elen = G.hy;
        f.cellL = (long long)(J * G.by) * G.nx + I * G.bx - 1;
        f.cellR = f.cellL + 1;
        f.step = G.nx;
    } else {  // y-face (I, J), J = 1..Ny-1
        const int e = fid - nex, J = e / G.Nx + 1, I = e % G.Nx;
        f.K1 = (J - 1) * G.Nx + I;
        f.K2 = J * G.Nx + I;
        f.s1 = 3;
        f.s2 = 2;
        f.Jn = G.bx;
        f.elen = G.hx;
        f.cellL = (long long)(J * G.by - 1) * G.nx + I * G.bx;
        f.cellR = f.cellL + G.nx;
        f.step = 1;
    }
    return f;
}

// Entry (l, m) of the s-form on the snapshot pair (l, m) of a face (eq. spectral_eqn):
// the kappa^{-1}-weighted mass Gram of the two block halves plus the divergence term
// sum_K |e_l||e_m| / |K|, times the prefactor invH.
__device__ inline double s_entry(const BlockGeom& G, const FaceGeom& f, const double* G1, const double* G2, int l,
                                 int m, double invH) {
    const double areaK = G.bx * G.hx * G.by * G.hy;
    return (G1[(f.s1 * G.jmax + l) * G.ncol + f.s1 * G.jmax + m] + G2[(f.s2 * G.jmax + l) * G.ncol + f.s2 * G.jmax + m] +
            2.0 * f.elen * f.elen / areaK) *
           invH;
}

// The pencil of every coarse face as the eigensolver sees it: D[fid][l] (the diagonal
// a-form) and S[fid][l][m] (the s-form, symmetrised), rows padded to jmax with zeros.
__global__ void k_pencil_probe(BlockGeom G, const double* __restrict__ kinv, const double* __restrict__ Gm,
                               double invH, double* __restrict__ Dout, double* __restrict__ Sout) {
    const int fid = blockIdx.x;
    const FaceGeom f = face_geom(G, fid);
    const double* G1 = Gm + (long long)f.K1 * G.ncol * G.ncol;
    const double* G2 = Gm + (long long)f.K2 * G.ncol * G.ncol;
    for (int l = threadIdx.x; l < G.jmax; l += blockDim.x)
        Dout[(long long)fid * G.jmax + l] =
            l < f.Jn ? f.elen * 0.5 * (kinv[f.cellL + l * f.step] + kinv[f.cellR + l * f.step]) : 0.0;
    for (int e = threadIdx.x; e < G.jmax * G.jmax; e += blockDim.x) {
        const int l = e / G.jmax, m = e % G.jmax;
        double v = 0.0;
        if (l < f.Jn && m < f.Jn) v = 0.5 * (s_entry(G, f, G1, G2, l, m, invH) + s_entry(G, f, G1, G2, m, l, invH));
        Sout[(long long)fid * G.jmax * G.jmax + e] = v;
    }
}

// force: the basis count of every face imposed (clamped to [1, J_i]) instead of the
// threshold count, or null; msfem: one basis per face, the sum of the face's snapshots
// (section 4.2, eq. msfem); eig_bad: counts the faces whose Jacobi solve was still
// rotating at its sweep limit.
template <int WARM, int JM>
__global__ void __launch_bounds__(64) k_pencil_eig(BlockGeom G, const double* __restrict__ kinv,
                                                   const double* __restrict__ Gm, double tol, double invH,
                                                   double* __restrict__ eigs, int* __restrict__ counts,
                                                   double* __restrict__ Yout, double* __restrict__ Qout,
                                                   const float* __restrict__ Y0, int kblk, double rq_tol, int max_it,
                                                   int* __restrict__ wstat, float* __restrict__ Vtop,
                                                   const int* __restrict__ force, int msfem, int* __restrict__ eig_bad) {
    constexpr int LD = JM + 1;
    __shared__ double T[JM][LD];
    __shared__ double V[JM][LD];
    __shared__ double D[JM];
    __shared__ double cs[JM / 2][2];
    __shared__ int pq[JM / 2][2];
    __shared__ int order[JM];
    __shared__ int rot_flag;
    // the subspace iteration's X, T X (rows < JM) and Rayleigh-Ritz matrices
    __shared__ double Wk[WARM ? 2 * JM * KW + 2 * KW * 9 : 1];
    __shared__ double thS[WARM ? KW : 1];  // the Ritz values by descending theta
    const int fid = blockIdx.x, lane = threadIdx.x;
    const FaceGeom fg = face_geom(G, fid);
    const int Jn = fg.Jn;
    const double elen = fg.elen;
    const double* G1 = Gm + (long long)fg.K1 * G.ncol * G.ncol;
    const double* G2 = Gm + (long long)fg.K2 * G.ncol * G.ncol;
    for (int l = lane; l < Jn; l += 64)
        D[l] = elen * 0.5 * (kinv[fg.cellL + l * fg.step] + kinv[fg.cellR + l * fg.step]);
    __syncthreads();
    for (int e = lane; e < Jn * Jn; e += 64) {
        const int l = e / Jn, mm = e % Jn;
        T[l][mm] = s_entry(G, fg, G1, G2, l, mm, invH) / sqrt(D[l] * D[mm]);
    }
    __syncthreads();
    // symmetrise (the two Gram halves are symmetric up to round-off)
    for (int e = lane; e < Jn * Jn; e += 64) {
        const int l = e / Jn, mm = e % Jn;
        if (l < mm) {
            const double avg = 0.5 * (T[l][mm] + T[mm][l]);
            T[l][mm] = avg;
            T[mm][l] = avg;
        }
    }
    __syncthreads();
    double* ev = eigs + (long long)fid * G.jmax;
    double* Yf = Yout + (long long)fid * G.jmax * G.jmax;
    int cnt = 0;
    bool accepted = false;
    if constexpr (WARM) {
        const double sigma = 1.0 / tol;
        const int kk = min(kblk, Jn);
        double* A = &V[0][0];  // LDS workspace of the inertia count (V is not needed before a fallback)
        const int cnt0 = inertia_above<LD>(T, A, Jn, sigma);
        const int l = max(cnt0, 1);
        if (cnt0 >= 0 && l < kk) {
            double* Xs = Wk;           // [JM][KW] rows of X, then of U
            double* Ws = Wk + JM * KW;  // [JM][KW] rows of T X
            double* Hs = Ws + JM * KW; // [KW][9]  X^T T X, then its diagonal form
            double* Zs = Hs + KW * 9;  // [KW][9]  its eigenvectors
            double x[KW], w[KW];
#pragma unroll
            for (int c = 0; c < KW; ++c) {
                double v = 0.0;
                if (c < kk && lane < Jn)
                    v = Y0 ? (double)Y0[((long long)fid * KW + c) * G.jmax + lane]
                           : cos(M_PI * (lane + 0.5) * c / Jn);
                x[c] = v;
            }
            for (int it = 0; it <= max_it; ++it) {
                // modified Gram-Schmidt on the columns of X (lane = row)
                bool rank_ok = true;
#pragma unroll
                for (int c = 0; c < KW; ++c) {
                    if (c < kk && rank_ok) {
                        const double n0 = sqrt(wave_sum(x[c] * x[c]));
#pragma unroll
                        for (int p = 0; p < KW; ++p)
                            if (p < c) x[c] -= wave_sum(x[p] * x[c]) * x[p];
                        const double nq = sqrt(wave_sum(x[c] * x[c]));
                        if (!(nq > 1e-12 * fmax(n0, 1e-300)))
                            rank_ok = false;
                        else
                            x[c] /= nq;
                    }
                }
                if (!rank_ok) break;
                // W = T X
                if (lane < JM)
#pragma unroll
                    for (int c = 0; c < KW; ++c) Xs[lane * KW + c] = x[c];
                __syncthreads();
#pragma unroll
                for (int c = 0; c < KW; ++c) w[c] = 0.0;
                if (lane < Jn)
                    for (int m = 0; m < Jn; ++m) {
                        const double t = T[lane][m];
#pragma unroll
                        for (int c = 0; c < KW; ++c) w[c] += t * Xs[m * KW + c];
                    }
                if (lane < JM)
#pragma unroll
                    for (int c = 0; c < KW; ++c) Ws[lane * KW + c] = w[c];
                __syncthreads();
                // H = X^T W (kk x kk), symmetrised, and its eigenpairs
                if (lane < kk * kk) {
                    const int a = lane / kk, b = lane % kk;
                    double h = 0.0, hT = 0.0;
                    for (int m = 0; m < Jn; ++m) {
                        h += Xs[m * KW + a] * Ws[m * KW + b];
                        hT += Xs[m * KW + b] * Ws[m * KW + a];
                    }
                    Hs[a * 9 + b] = 0.5 * (h + hT);
                    Zs[a * 9 + b] = (a == b) ? 1.0 : 0.0;
                }
                __syncthreads();
                jacobi_rr<KW>(Hs, Zs, 9, kk, cs, pq, &rot_flag);
                if (lane < kk) {
                    const double th = Hs[lane * 9 + lane];
                    int rank = 0;
                    for (int k = 0; k < kk; ++k) {
                        const double o = Hs[k * 9 + k];
                        rank += (o > th) || (o == th && k < lane);
                    }
                    order[rank] = lane;
                }
                __syncthreads();
                // Ritz vectors U = X Z (to the rows of Xs: X is not read again this
                // iteration) and T U = W Z (the next start), columns by descending theta
                double xn[KW];
                int nabove = 0;
                bool ok = true;
#pragma unroll
                for (int c = 0; c < KW; ++c) {
                    double uc = 0.0, tuc = 0.0, thc = 0.0;
                    if (c < kk) {
                        const int oc = order[c];
                        thc = Hs[oc * 9 + oc];
#pragma unroll
                        for (int a = 0; a < KW; ++a)
                            if (a < kk) {
                                uc += x[a] * Zs[a * 9 + oc];
                                tuc += w[a] * Zs[a * 9 + oc];
                            }
                        nabove += thc > sigma;
                    }
                    if (c < l) {
                        const double r = tuc - thc * uc;
                        ok = ok && sqrt(wave_sum(r * r)) / fabs(thc) <= rq_tol;
                    }
                    if (lane < JM) Xs[lane * KW + c] = uc;
                    if (lane == 0) thS[c] = thc;
                    xn[c] = tuc;
                }
                ok = ok && nabove == cnt0;
                __syncthreads();
                if (ok) {
                    // outputs from the Ritz pairs (U in Xs, row = lane)
                    for (int k = lane; k < G.jmax; k += 64) ev[k] = (k < kk && k < KW) ? 1.0 / thS[k] : 0.0;
                    for (int e = lane; e < G.jmax * G.jmax; e += 64) {
                        const int r = e / G.jmax, k = e % G.jmax;
                        Yf[e] = (r < Jn && k < l) ? Xs[r * KW + k] / sqrt(D[r]) : 0.0;
                    }
                    __syncthreads();
                    accepted = true;
                    if (cnt0 == 0) accepted = inertia_above<LD>(T, A, Jn, thS[0] * (1.0 - 4.0 * rq_tol)) == 1;
                    if (accepted) {
                        cnt = l;
                        if (lane == 0) {
                            counts[fid] = cnt;
                            wstat[fid] = it;
                        }
                    }
                    break;
                }
#pragma unroll
                for (int c = 0; c < KW; ++c) x[c] = xn[c];
                __syncthreads();
            }
        }
        if (!accepted && lane == 0) wstat[fid] = -1;
        __syncthreads();
    }
    if (!accepted) {
        for (int e = lane; e < Jn * Jn; e += 64) {
            const int l = e / Jn, mm = e % Jn;
            V[l][mm] = (l == mm) ? 1.0 : 0.0;
        }
        __syncthreads();
        const bool conv = jacobi_rr<JM>(&T[0][0], &V[0][0], LD, Jn, cs, pq, &rot_flag);
        if (!conv && lane == 0 && eig_bad) atomicAdd(eig_bad, 1);
        // sort mu descending (lambda = 1/mu ascending)
        if (lane < Jn) {
            const double mu = T[lane][lane];
            int rank = 0;
            for (int k = 0; k < Jn; ++k) {
                const double o = T[k][k];
                rank += (o > mu) || (o == mu && k < lane);
            }
            order[rank] = lane;
        }
        __syncthreads();
        for (int k = lane; k < G.jmax; k += 64) ev[k] = (k < Jn) ? 1.0 / T[order[k]][order[k]] : 0.0;
        __syncthreads();
        for (int k = 0; k < Jn; ++k) cnt += (1.0 / T[order[k]][order[k]] < tol);
        cnt = cnt < 1 ? 1 : cnt;
        if (force) cnt = min(max(force[fid], 1), Jn);
        if (msfem) cnt = 1;
        if (lane == 0) counts[fid] = cnt;
        // Y[:, k] = D^{-1/2} v_k for the kept modes (MsFEM: all snapshot coefficients 1);
        // flux f_k = |e| sum_l Y[l][k]
        for (int e = lane; e < G.jmax * G.jmax; e += 64) {
            const int l = e / G.jmax, k = e % G.jmax;
            Yf[e] = (l < Jn && k < cnt) ? (msfem ? 1.0 : V[l][order[k]] / sqrt(D[l])) : 0.0;
        }
        if (Vtop)
            for (int e = lane; e < KW * G.jmax; e += 64) {
                const int c = e / G.jmax, r = e % G.jmax;
                Vtop[(long long)fid * KW * G.jmax + e] = (c < Jn && r < Jn) ? (float)V[r][order[c]] : 0.f;
            }
        __syncthreads();
    }
    // recombination Q (cnt x cnt): column 0 = f/|f|^2 (unit-flux carrier), columns 1.. = an
    // orthonormal basis of f^perp (Householder reflector mapping f/|f| to e_1); stored in LDS
    // (V is free now), then YQ = Y Q (jmax x jmax, rows l < Jn, columns k < cnt) to Qout.
    // (lane k holds f_k and w_k; w is staged in LDS for the rows of the reflector)
    double* Qs = &V[0][0];  // Qs[k2 * LD + k]
    __shared__ double wsh[JM];
    {
        double fk = 0.0;
        if (lane < cnt) {
            for (int l = 0; l < Jn; ++l) fk += Yf[l * G.jmax + lane];
            fk *= elen;
        }
        const double nrm2 = wave_sum(fk * fk);
        if (lane < cnt) Qs[lane * LD] = fk / nrm2;
        if (cnt > 1) {
            const double nr = sqrt(nrm2);
            double wk = lane < cnt ? fk / nr : 0.0;
            if (lane == 0) wk += (wk >= 0 ? 1.0 : -1.0);
            const double ww = wave_sum(wk * wk);
            if (lane < cnt) wsh[lane] = wk;
            __syncthreads();
            if (lane < cnt)
                for (int cc = 1; cc < cnt; ++cc) Qs[lane * LD + cc] = ((lane == cc) ? 1.0 : 0.0) - 2.0 * wk * wsh[cc] / ww;
        }
    }
    __syncthreads();
    double* Qf = Qout + (long long)fid * G.jmax * G.jmax;
    for (int e = lane; e < G.jmax * G.jmax; e += 64) {
        const int l = e / G.jmax, k = e % G.jmax;
        double s = 0.0;
        if (l < Jn && k < cnt)
            for (int k2 = 0; k2 < cnt; ++k2) s += Yf[l * G.jmax + k2] * Qs[k2 * LD + k];
        Qf[e] = s;
    }
}

// Td = the coarse basis combination of each block: column kc = side * jmax + l of slot u
// (a coarse unknown touching the block) is sum over the slot's contributions c of
// sign_c * YQ[face_c][l][mode_c] on the contribution's side (l < that side's face count).
// meta[(b * mu + u) * 11]: id, corner, count, then (face, side, mode, sign) twice.
__global__ void k_fill_td(BlockGeom G, int mu, const int* __restrict__ meta, const double* __restrict__ YQ,
                          double* __restrict__ Td) {
    const int b = blockIdx.x;
    for (int e = threadIdx.x; e < G.ncol * mu; e += blockDim.x) {
        const int kc = e / mu, u = e % mu, side = kc / G.jmax, l = kc % G.jmax;
        const int* m = meta + ((long long)b * mu + u) * 11;
        const int nl = side < 2 ? G.by : G.bx;
        double val = 0.0;
        for (int q = 0; q < m[2]; ++q) {
            const int f = m[3 + 4 * q], sd = m[4 + 4 * q], k = m[5 + 4 * q], sg = m[6 + 4 * q];
            if (sd == side && l < nl) val += sg * YQ[((long long)f * G.jmax + l) * G.jmax + k];
        }
        Td[((long long)b * G.ncol + kc) * mu + u] = val;
    }
}

// Per block: Ak = T_K^T G_K T_K scattered into the dense coarse matrix, and the
// path integral of every snapshot column to vertex values (for the stream functions).
// Launched once per colour (I%2, J%2): blocks of one colour share no coarse unknown, so
// their contributions are added without atomics and the assembly is deterministic.
// A_c[unk(u)][unk(w)] += H_K[u][w] for one colour of blocks (blocks of a colour share no
// unknown, so no atomics): H_K = T_K^T G_K T_K, formed by batched products
__global__ void k_coarse_scatter(int Nx, int Ny, const double* __restrict__ H, int mu, const int* __restrict__ unk,
                                 const int* __restrict__ nunk, double* __restrict__ Ac, int ncs, int colour) {
    const int bxc = (Nx + 1 - (colour & 1)) / 2;
    const int bI = 2 * (blockIdx.x % bxc) + (colour & 1), bJ = 2 * (blockIdx.x / bxc) + (colour >> 1);
    if (bI >= Nx || bJ >= Ny) return;
    const int blk = bJ * Nx + bI, nu = nunk[blk];
    const int* ub = unk + (long long)blk * mu;
    const double* Hb = H + (long long)blk * mu * mu;
    for (int e = threadIdx.x; e < nu * nu; e += blockDim.x) {
        const int u = e / nu, w = e % nu;
        Ac[(long long)ub[u] * ncs + ub[w]] += Hb[u * mu + w];
    }
}

// H_K = T_K^T G_K T_K per block (G_K symmetric: column r of G is read as row r, so
// consecutive threads read consecutive words); T and G T in LDS.
__global__ void __launch_bounds__(256) k_coarse_H(BlockGeom G, const double* __restrict__ Gm,
                                                  const double* __restrict__ Tm, int mu,
                                                  const int* __restrict__ nunk, double* __restrict__ H) {
    extern __shared__ double sm[];
    const int blk = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
    const int ncol = G.ncol, nu = nunk[blk];
    double* Ts = sm;            // ncol x mu
    double* GT = Ts + ncol * mu;  // ncol x mu
    const double* Gb = Gm + (long long)blk * ncol * ncol;
    const double* Tb = Tm + (long long)blk * ncol * mu;
    for (int e = tid; e < ncol * mu; e += nth) Ts[e] = Tb[e];
    __syncthreads();
    for (int e = tid; e < ncol * nu; e += nth) {
        const int r = e % ncol, u = e / ncol;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < ncol; ++k) s += Gb[(long long)k * ncol + r] * Ts[k * mu + u];
        GT[r * mu + u] = s;
    }
    __syncthreads();
    double* Hb = H + (long long)blk * mu * mu;
    for (int e = tid; e < nu * nu; e += nth) {
        const int u = e / nu, w = e % nu;
        double s = 0.0;
        for (int k = 0; k < ncol; ++k) s += Ts[k * mu + u] * GT[k * mu + w];
        Hb[u * mu + w] = s;
    }
}

// The stream functions of a block's coarse unknowns.  By linearity the stream function
// of an unknown is the path integral (psi(0,0) = 0, along the bottom edge by the
// y-fluxes, then up each vertex column by the x-fluxes) of its flux field
// Psi_K T_K[:, u], so the snapshots are combined first and only the unknowns' fields are
// integrated; W_K[v][u] = psi_u(v) - psi_u(zero corner of u) on the owned vertices.
// 512 threads: two per fine face for the flux fields (each half of the snapshot
// columns, eight loads in flight, summed across the lane pair), chunks of CL_UC
// unknowns; LDS: T (padded with zero columns to whole chunks), a chunk of the flux
// fields and of their stream functions.
constexpr int CL_UC = 8;
constexpr int CL_NT = 512;
__global__ void __launch_bounds__(CL_NT) k_coarse_W2(BlockGeom G, const double* __restrict__ Psi,
                                                     const double* __restrict__ Tm, int mu,
                                                     const int* __restrict__ nunk, const int* __restrict__ zc,
                                                     double* __restrict__ W, float* __restrict__ W32) {
    extern __shared__ double sm[];
    const int blk = blockIdx.x, tid = threadIdx.x;
    const int I = blk % G.Nx, J = blk / G.Nx;
    const int ncol = G.ncol, nfk = G.nfk, nu = nunk[blk];
    const int bxl = G.bx, byl = G.by, nfx = byl * (bxl + 1);
    const int nown = bxl * byl;
    const int mup = (mu + CL_UC - 1) / CL_UC * CL_UC;
    double* Ts = sm;                           // ncol x mup
    double* Fs = Ts + ncol * mup;              // nfk x CL_UC
    double* Ps = Fs + (long long)nfk * CL_UC;  // nvtx x CL_UC
    const double* Tb = Tm + (long long)blk * ncol * mu;
    for (int e = tid; e < ncol * mup; e += CL_NT) {
        const int r = e / mup, u = e % mup;
        Ts[e] = u < mu ? Tb[r * mu + u] : 0.0;
    }
    __syncthreads();
    const double* Pb = Psi + (long long)blk * ncol * nfk;
    double* Wb = W + (long long)blk * nown * mu;
    float* Wb32 = W32 ? W32 + (long long)blk * nown * mu : nullptr;
    const int half = tid & 1, hc = ncol / 2, c0 = half * hc;
    for (int u0 = 0; u0 < mu; u0 += CL_UC) {
        const int uc = min(CL_UC, mu - u0);
        // flux fields F[f][j] = sum_col Psi[col][f] T[col][u0 + j]; the whole wave runs
        // every pass (lanes past nfk read face nfk - 1 and discard it), so the pair sum is
        // taken by both lanes
        for (int f0 = tid >> 1; f0 < ((nfk + CL_NT / 2 - 1) / (CL_NT / 2)) * (CL_NT / 2); f0 += CL_NT / 2) {
            const int f = min(f0, nfk - 1);
            double acc[CL_UC];
#pragma unroll
            for (int j = 0; j < CL_UC; ++j) acc[j] = 0.0;
            // eight snapshot columns a step: every load issued (clamped rows past hc)
            // before any product uses one
            for (int q0 = 0; q0 < hc; q0 += 8) {
                double pv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) pv[t] = Pb[(long long)(c0 + min(q0 + t, hc - 1)) * nfk + f];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const double w = q0 + t < hc ? pv[t] : 0.0;
                    const double* tr = Ts + (c0 + min(q0 + t, hc - 1)) * mup + u0;
#pragma unroll
                    for (int j = 0; j < CL_UC; ++j) acc[j] += w * tr[j];
                }
            }
#pragma unroll
            for (int j = 0; j < CL_UC; ++j) acc[j] += __shfl_xor(acc[j], 1, 64);
            if (half == 0 && f0 < nfk)
#pragma unroll
                for (int j = 0; j < CL_UC; ++j) Fs[f * CL_UC + j] = acc[j];
        }
        __syncthreads();
        // path integrals: one task per (unknown of the chunk, vertex column)
        for (int task = tid; task < uc * (bxl + 1); task += CL_NT) {
            const int j = task % uc, a = task / uc;
            double p = 0.0;
            for (int q = 0; q < a; ++q) p -= G.hx * Fs[(nfx + q) * CL_UC + j];
            Ps[a * CL_UC + j] = p;
            for (int b = 0; b < byl; ++b) {
                p += G.hy * Fs[(b * (bxl + 1) + a) * CL_UC + j];
                Ps[((b + 1) * (bxl + 1) + a) * CL_UC + j] = p;
            }
        }
        __syncthreads();
        for (int e = tid; e < nown * uc; e += CL_NT) {
            const int v = e / uc, j = e % uc, u = u0 + j;
            const int a = v % bxl, b = v / bxl;
            double val = 0.0;
            if (u < nu && !((I == 0 && a == 0) || (J == 0 && b == 0))) {
                const int corner = zc[(long long)blk * mu + u];
                val = Ps[(b * (bxl + 1) + a) * CL_UC + j] - Ps[corner * CL_UC + j];
            }
            Wb[(long long)v * mu + u] = val;
            if (Wb32) Wb32[(long long)v * mu + u] = (float)val;
        }
        __syncthreads();
    }
}

// The coarse RT0 space as the coarse space of the two-grid preconditioner (the paper's
// comparator, section 5): its divergence-free part with zero boundary flux is the curl of
// the bilinear stream functions of the interior coarse vertices, so a block's slot u
// (the coarse vertex (I + ci, J + cj), ci, cj in {0, 1}) holds the bilinear hat of that
// vertex on the block's owned fine vertices.
__global__ void k_rt0_W(BlockGeom G, int mu, const int* __restrict__ unk, const int* __restrict__ nunk,
                        double* __restrict__ W, float* __restrict__ W32) {
    const int blk = blockIdx.x, I = blk % G.Nx, J = blk / G.Nx;
    const int nown = G.bx * G.by, nu = nunk[blk];
    for (int e = threadIdx.x; e < nown * mu; e += blockDim.x) {
        const int v = e / mu, u = e % mu;
        const int a = v % G.bx, b = v / G.bx;
        double val = 0.0;
        if (u < nu) {
            const int id = unk[(long long)blk * mu + u];
            const int ci = id % (G.Nx - 1) + 1 - I, cj = id / (G.Nx - 1) + 1 - J;
            const double wx = ci ? (double)a / G.bx : 1.0 - (double)a / G.bx;
            const double wy = cj ? (double)b / G.by : 1.0 - (double)b / G.by;
            val = wx * wy;
        }
        W[(long long)blk * nown * mu + e] = val;
        if (W32) W32[(long long)blk * nown * mu + e] = (float)val;
    }
}

// Coarse RT0 Gram per block: linear coarse basis functions W, E (x) and S, N (y).
__global__ void k_rt0_blocks(BlockGeom G, const double* __restrict__ a, double* __restrict__ AH0) {
    const int blk = blockIdx.x, I = blk % G.Nx, J = blk / G.Nx;
    const int lane = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int e = lane; e < G.bx * G.by; e += 64) {
        const int aa = e % G.bx, bb = e / G.bx;
        const double w = a[(long long)(J * G.by + bb) * G.nx + I * G.bx + aa];
        {  // x: phi_W = 1 - x/H at local faces aa, aa+1; phi_E = x/H
            const double eL = (double)aa / G.bx, eR = (double)(aa + 1) / G.bx;
            const double wL = 1.0 - eL, wR = 1.0 - eR;
            s[0] += w * (wL * wL / 3 + wR * wR / 3 + wL * wR / 3);
            s[1] += w * (wL * eL / 3 + wR * eR / 3 + (wL * eR + wR * eL) / 6);
            s[2] += w * (eL * eL / 3 + eR * eR / 3 + eL * eR / 3);
        }
        {
            const double nB = (double)bb / G.by, nT = (double)(bb + 1) / G.by;
            const double sB = 1.0 - nB, sT = 1.0 - nT;
            s[3] += w * (sB * sB / 3 + sT * sT / 3 + sB * sT / 3);
            s[4] += w * (sB * nB / 3 + sT * nT / 3 + (sB * nT + sT * nB) / 6);
            s[5] += w * (nB * nB / 3 + nT * nT / 3 + nB * nT / 3);
        }
    }
    for (int k = 0; k < 6; ++k) {
        const double t = wave_sum(s[k]);
        if (lane == 0) AH0[(long long)blk * 6 + k] = t;
    }
}

// Coarse RT0 stream-function stiffness K_H = C_H^T A_H C_H on the interior coarse
// vertices (dense, row-major; zero on entry).  Each coarse cell contributes a 4 x 4
// block among its corners through its W/E/S/N face fluxes; one thread per vertex
// sums the contributions to its own row (no atomics, fixed order).
__global__ void k_rt0_stiffness(const double* __restrict__ AH0, int Nx, int Ny, double Hx, double Hy,
                                double* __restrict__ K) {
    const int nvx = Nx - 1, nv = (Nx - 1) * (Ny - 1);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int Iv = v % nvx + 1, Jv = v / nvx + 1;
    auto vid = [&](int I, int J) { return (I <= 0 || I >= Nx || J <= 0 || J >= Ny) ? -1 : (J - 1) * nvx + I - 1; };
    double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // neighbour offsets (dI, dJ) + 1
    for (int Jc = Jv - 1; Jc <= Jv; ++Jc)
        for (int Ic = Iv - 1; Ic <= Iv; ++Ic) {
            const double* m = AH0 + 6 * ((long long)Jc * Nx + Ic);
            // face flux of each basis field as combinations of corner stream-function values
            const int vw[2] = {vid(Ic, Jc + 1), vid(Ic, Jc)};
            const double ww[2] = {1 / Hy, -1 / Hy};
            const int ve[2] = {vid(Ic + 1, Jc + 1), vid(Ic + 1, Jc)};
            const int vs[2] = {vid(Ic + 1, Jc), vid(Ic, Jc)};
            const double ws[2] = {-1 / Hx, 1 / Hx};
            const int vn[2] = {vid(Ic + 1, Jc + 1), vid(Ic, Jc + 1)};
            const int* fv[4] = {vw, ve, vs, vn};
            const double* fw[4] = {ww, ww, ws, ws};
            // (face a, face b, weight): W-W, W-E, E-W, E-E, S-S, S-N, N-S, N-N
            const int pa[8] = {0, 0, 1, 1, 2, 2, 3, 3}, pb[8] = {0, 1, 0, 1, 2, 3, 2, 3};
            const double pw[8] = {m[0], m[1], m[1], m[2], m[3], m[4], m[4], m[5]};
            for (int t = 0; t < 8; ++t)
                for (int p = 0; p < 2; ++p) {
                    if (fv[pa[t]][p] != v) continue;
                    for (int q = 0; q < 2; ++q) {
                        const int wv = fv[pb[t]][q];
                        if (wv < 0) continue;
                        const int dI = wv % nvx + 1 - Iv, dJ = wv / nvx + 1 - Jv;
                        acc[dJ + 1][dI + 1] += pw[t] * fw[pa[t]][p] * fw[pb[t]][q];
                    }
                }
        }
    for (int dJ = -1; dJ <= 1; ++dJ)
        for (int dI = -1; dI <= 1; ++dI) {
            const int wv = vid(Iv + dI, Jv + dJ);
            if (wv >= 0) K[(long long)v * nv + wv] = acc[dJ + 1][dI + 1];
        }
}

// ---- coarse apply in stream-function coordinates ----
// Restriction W^T g per block into cy (one workgroup per block).
template <typename T>
__global__ void k_coarse_restrict(const T* __restrict__ W, int mu, const int* __restrict__ nunk,
                                  const T* __restrict__ g, int nx, int bx, int by, int Nx, T* __restrict__ cy,
                                  const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ T part[4][64];
    const int blk = blockIdx.x, I = blk % Nx, J = blk / Nx;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nown = bx * by, nu = nunk[blk];
    const T* Wb = W + (long long)blk * nown * mu;
    for (int u = 0; u < nu; ++u) {
        T s = T(0);
        for (int v = tid; v < nown; v += 256) {
            const int aa = v % bx, bb = v / bx;
            s += Wb[(long long)v * mu + u] * g[(long long)(J * by + bb) * nx + I * bx + aa];
        }
        s = wave_sum(s);
        if (lane == 0) part[wid][u & 63] = s;
        __syncthreads();
        if (tid == 0) cy[(long long)blk * mu + u] = part[0][u & 63] + part[1][u & 63] + part[2][u & 63] + part[3][u & 63];
        __syncthreads();
    }
}

// each coarse unknown: the sum of its contributions from the blocks (fixed order)
template <typename T>
__global__ void k_coarse_accum(const int* __restrict__ ptr, const int* __restrict__ ent, const T* __restrict__ cy,
                               int ncs, T* __restrict__ c, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ncs) return;
    c[u] = gather_sum<T>(ent, cy, ptr[u], ptr[u + 1]);
}

template <typename T>
__global__ void k_coarse_prolong(const T* __restrict__ W, int mu, const int* __restrict__ unk,
                                 const int* __restrict__ nunk, const T* __restrict__ c, int nx, int bx, int by,
                                 int Nx, T* __restrict__ z, int accumulate, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int blk = blockIdx.x, I = blk % Nx, J = blk / Nx;
    const int nown = bx * by, nu = nunk[blk];
    const T* Wb = W + (long long)blk * nown * mu;
    const int* ub = unk + (long long)blk * mu;
    for (int v = threadIdx.x; v < nown; v += blockDim.x) {
        const int aa = v % bx, bb = v / bx;
        T s = T(0);
        for (int u = 0; u < nu; ++u) s += Wb[(long long)v * mu + u] * c[ub[u]];
        T* zp = z + (long long)(J * by + bb) * nx + I * bx + aa;
        *zp = accumulate ? *zp + s : s;
    }
}

BlockGeom geom(tgms_ctx* c) {
    BlockGeom G;
    G.nx = c->nx;
    G.ny = c->ny;
    G.bx = c->bx;
    G.by = c->by;
    G.Nx = c->Nx;
    G.Ny = c->Ny;
    G.jmax = c->jmax;
    G.nfk = c->nfk;
    G.ncol = c->ncol;
    G.hx = c->hx;
    G.hy = c->hy;
    G.sx = c->sx;
    G.sy = c->sy;
    return G;
}

}  // namespace

namespace tgms {

template <int M>
static void launch_snap_cols(tgms_ctx* c, const BlockGeom& G, size_t lds, double* Vg, long long vstride) {
    if (Vg) {
        (void)hipFuncSetAttribute((const void*)k_snapshots_cols<M, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  c->lds_max);
        hipLaunchKernelGGL((k_snapshots_cols<M, true>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL,
                           c->Psi, Vg, vstride);
    } else {
        (void)hipFuncSetAttribute((const void*)k_snapshots_cols<M, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  c->lds_max);
        hipLaunchKernelGGL((k_snapshots_cols<M, false>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL,
                           c->Psi, Vg, vstride);
    }
}

void snapshots(tgms_ctx* c, double* scratch, long long scratch_per_block) {
    BlockGeom G = geom(c);
    // one lane per snapshot column: needs 4*jmax <= 64 and the block's factor and
    // weights in LDS; the 64 columns of interior-vertex values go to LDS too when the
    // blocks are few (one workgroup per CU at most), else to the scratch (when it holds
    // them), which lets several workgroups share a CU
    const int m = c->bx - 1, mh = c->by - 1;
    const long long fsz = btri_size(m, mh);
    const size_t lds_fac = sizeof(double) * ((((fsz > 32 * 64 ? fsz : 32 * 64) + 1) & ~1LL) + c->bx * c->by + 1);
    const size_t lds_cols = lds_fac + sizeof(double) * (size_t)m * mh * 64;
    const size_t lds_tile = sizeof(double) * ((size_t)32 * 64 + c->bx * c->by + 1);  // factor read from global
    int cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    const bool vglobal = scratch && scratch_per_block >= (long long)m * mh * 64 && c->nblk > 2 * cus;
    const size_t lds_use = vglobal ? lds_tile : lds_cols;
    double* Vg = vglobal ? scratch : nullptr;
    if (c->snap_cols && c->ncol <= 64 && lds_use <= (size_t)c->lds_max) {
        switch (m) {
            case 3: launch_snap_cols<3>(c, G, lds_use, Vg, scratch_per_block); LAUNCH_OK(); return;
            case 5: launch_snap_cols<5>(c, G, lds_use, Vg, scratch_per_block); LAUNCH_OK(); return;
            case 7: launch_snap_cols<7>(c, G, lds_use, Vg, scratch_per_block); LAUNCH_OK(); return;
            case 9: launch_snap_cols<9>(c, G, lds_use, Vg, scratch_per_block); LAUNCH_OK(); return;
            case 11: launch_snap_cols<11>(c, G, lds_use, Vg, scratch_per_block); LAUNCH_OK(); return;
            case 15: launch_snap_cols<15>(c, G, lds_use, Vg, scratch_per_block); LAUNCH_OK(); return;
            default: break;
        }
    }
    const int nfx = c->by * (c->bx + 1), nfy = (c->by + 1) * c->bx, nloc = (c->bx - 1) * (c->by - 1);
    size_t lds = sizeof(double) * (2 * c->by + 2 * c->bx + c->bx * c->by + 2 * (nfx + nfy) + nloc + c->by + 2 + 128);
    if (lds > 65536) throw TgmsError{TGMS_E_UNSUPPORTED, "coarse block too large for the snapshot kernel"};
    const int mw = btri_width(c->bx - 1);
    if (mw == 16)
        hipLaunchKernelGGL((k_snapshots<16>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL, c->blkS, c->Psi);
    else if (mw == 24)
        hipLaunchKernelGGL((k_snapshots<24>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL, c->blkS, c->Psi);
    else
        hipLaunchKernelGGL((k_snapshots<32>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL, c->blkS, c->Psi);
    LAUNCH_OK();
}

void gram(tgms_ctx* c) {
    BlockGeom G = geom(c);
    if (gram_uses_mfma(c)) {
        if (c->ncol == 64)
            hipLaunchKernelGGL(k_gram_mfma<4>, dim3(c->nblk), dim3(256), 0, c->stream, G, c->a, c->Psi, c->G);
        else
            hipLaunchKernelGGL(k_gram_mfma<2>, dim3(c->nblk), dim3(256), 0, c->stream, G, c->a, c->Psi, c->G);
        LAUNCH_OK();
        return;
    }
    hipLaunchKernelGGL(k_apply_AK_cols, dim3(c->nblk, c->ncol), dim3(256), 0, c->stream, G, c->a, c->Psi, c->APsi);
    LAUNCH_OK();
    const int q4 = c->ncol / 4;
    size_t lds = sizeof(double) * 2 * c->ncol * 32;
    hipLaunchKernelGGL(k_gram, dim3(c->nblk), dim3(q4 * q4), lds, c->stream, G, c->Psi, c->APsi, c->G);
    LAUNCH_OK();
}

}  // namespace tgms

// Entry points used by the host orchestrator (api.hip) that need the kernels above.
namespace tgms {

template <int JM>
static void pencil_eig_launch(tgms_ctx* c, const BlockGeom& G, double* Q, const float* Y0, float* Vtop) {
    const int msfem = c->coarse_space == 1 ? 1 : 0;
    if (c->warm)
        hipLaunchKernelGGL((k_pencil_eig<1, JM>), dim3(c->ne), dim3(64), 0, c->stream, G, c->kinv, c->G, c->tol,
                           1.0 / c->H, c->eigs, c->counts, c->Y, Q, Y0, KW, c->rq_tol, c->warm_maxit, c->wstat,
                           (float*)nullptr, (const int*)c->force, msfem, c->eig_bad);
    else
        hipLaunchKernelGGL((k_pencil_eig<0, JM>), dim3(c->ne), dim3(64), 0, c->stream, G, c->kinv, c->G, c->tol,
                           1.0 / c->H, c->eigs, c->counts, c->Y, Q, (const float*)nullptr, 0, 0.0, 0, (int*)nullptr,
                           Vtop, (const int*)c->force, msfem, c->eig_bad);
    LAUNCH_OK();
}

void pencil_probe(tgms_ctx* c, double* D, double* S) {
    hipLaunchKernelGGL(k_pencil_probe, dim3(c->ne), dim3(256), 0, c->stream, geom(c), (const double*)c->kinv,
                       (const double*)c->G, 1.0 / c->H, D, S);
    LAUNCH_OK();
}

void pencil_eig_q(tgms_ctx* c, double* Q, const float* Y0, float* Vtop) {
    BlockGeom G = geom(c);
    // LDS tiles sized for the widest face (jmax = max(bx, by) cells)
    if (G.jmax <= 8)
        pencil_eig_launch<8>(c, G, Q, Y0, Vtop);
    else if (G.jmax <= 16)
        pencil_eig_launch<16>(c, G, Q, Y0, Vtop);
    else if (G.jmax <= 32)
        pencil_eig_launch<32>(c, G, Q, Y0, Vtop);
    else if (G.jmax <= 64)
        pencil_eig_launch<64>(c, G, Q, Y0, Vtop);
    else
        throw TgmsError{TGMS_E_UNSUPPORTED, "coarse face wider than 64 cells"};
}

void fill_td(tgms_ctx* c, const int* meta, const double* YQ, double* Td) {
    hipLaunchKernelGGL(k_fill_td, dim3(c->nblk), dim3(256), 0, c->stream, geom(c), c->mu, meta, YQ, Td);
    LAUNCH_OK();
}

void coarse_local_run(tgms_ctx* c, const double* Tm, const int* zc) {
    BlockGeom G = geom(c);
    const int ncol = c->ncol, mu = c->mu, nblk = c->nblk;
    const int nvtx = (c->bx + 1) * (c->by + 1);
    const size_t lds_h = sizeof(double) * 2 * (size_t)ncol * mu;
    const size_t lds_w = sizeof(double) * ((size_t)ncol * ((mu + CL_UC - 1) / CL_UC * CL_UC) +
                                           (size_t)(c->nfk + nvtx) * CL_UC);
    if (lds_h <= (size_t)c->lds_max && lds_w <= (size_t)c->lds_max && ncol % 2 == 0) {
        if (!c->clH) c->clH = c->alloc<double>((size_t)nblk * mu * mu);
        (void)hipFuncSetAttribute((const void*)k_coarse_H, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_h);
        (void)hipFuncSetAttribute((const void*)k_coarse_W2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_w);
        hipLaunchKernelGGL(k_coarse_H, dim3(nblk), dim3(256), lds_h, c->stream, G, (const double*)c->G, Tm, mu,
                           c->blk_nu, c->clH);
        LAUNCH_OK();
        for (int colour = 0; colour < 4; ++colour) {
            const int bxc = (c->Nx + 1 - (colour & 1)) / 2, byc = (c->Ny + 1 - (colour >> 1)) / 2;
            if (bxc <= 0 || byc <= 0) continue;
            hipLaunchKernelGGL(k_coarse_scatter, dim3(bxc * byc), dim3(64), 0, c->stream, c->Nx, c->Ny,
                               (const double*)c->clH, mu, c->blk_unk, c->blk_nu, c->Ac, c->ncs, colour);
            LAUNCH_OK();
        }
        hipLaunchKernelGGL(k_coarse_W2, dim3(nblk), dim3(CL_NT), lds_w, c->stream, G, (const double*)c->Psi, Tm, mu,
                           c->blk_nu, zc, c->W, c->precision ? c->W32 : nullptr);
        LAUNCH_OK();
        return;
    }
    // (blocks up to the band factor's limit, 20 x 20 cells, need at most about 133 KB)
    throw TgmsError{TGMS_E_UNSUPPORTED, "coarse assembly of a block exceeds the LDS"};
}

void rt0_stiffness(tgms_ctx* c, const double* AH0, double* K) {
    const int nv = (c->Nx - 1) * (c->Ny - 1);
    hipLaunchKernelGGL(k_rt0_stiffness, dim3((nv + 255) / 256), dim3(256), 0, c->stream, AH0, c->Nx, c->Ny,
                       c->bx * c->hx, c->by * c->hy, K);
    LAUNCH_OK();
}

void coarse_rt0_blocks(tgms_ctx* c, double* AH0) {
    BlockGeom G = geom(c);
    hipLaunchKernelGGL(k_rt0_blocks, dim3(c->nblk), dim3(64), 0, c->stream, G, c->a, AH0);
    LAUNCH_OK();
}

void rt0_coarse_W(tgms_ctx* c) {
    hipLaunchKernelGGL(k_rt0_W, dim3(c->nblk), dim3(256), 0, c->stream, geom(c), c->mu, (const int*)c->blk_unk,
                       (const int*)c->blk_nu, c->W, c->precision ? c->W32 : nullptr);
    LAUNCH_OK();
}

template <typename T>
struct CoarseBufs {
    const T* W;
    const T* Ainv;
    T* cy;
    T* c1;
};
template <typename T>
static CoarseBufs<T> coarse_bufs(tgms_ctx* c) {
    if constexpr (sizeof(T) == 8)
        return CoarseBufs<T>{(const T*)c->W, (const T*)c->Ac, (T*)c->cy, (T*)c->cvec};
    else
        return CoarseBufs<T>{(const T*)c->W32, (const T*)c->Ac32, (T*)c->cy32, (T*)c->cvec32};
}

template <typename T>
T* coarse_cy(tgms_ctx* c) {
    return coarse_bufs<T>(c).cy;
}
template double* coarse_cy<double>(tgms_ctx*);
template float* coarse_cy<float>(tgms_ctx*);

// the coarse unknowns from the block restrictions cy, then A^{-1} of them (two
// triangular products, or one product with the explicit inverse); returns the
// result (after c1 in the same buffer)
template <typename T>
const T* coarse_solve(tgms_ctx* c, const double* sc) {
    const CoarseBufs<T> B = coarse_bufs<T>(c);
    if (c->cb.nb > 0) {
        // cyclic-reduction Cholesky: accumulate into its padded vector, solve in place
        T* x = sizeof(T) == 8 ? (T*)c->cb.x : (T*)c->cb.x32;
        hipLaunchKernelGGL((k_coarse_accum<T>), dim3((c->ncs + 255) / 256), dim3(256), 0, c->stream, c->unk_ptr,
                           c->unk_ent, (const T*)B.cy, c->ncs, x, sc);
        LAUNCH_OK();
        bcr_solve<T>(c, c->cb, x, sc);
        return x;
    }
    T* res = B.c1 + c->ncs;
    if constexpr (sizeof(T) == 8)
        if (symv_full_acc(c, c->Acf, c->ncs, c->unk_ptr, c->unk_ent, (const double*)B.cy, (double*)res, sc))
            return res;
    if (symv_acc<T>(c, B.Ainv, c->ncs, c->unk_ptr, c->unk_ent, (const T*)B.cy, res, sc)) return res;
    hipLaunchKernelGGL((k_coarse_accum<T>), dim3((c->ncs + 255) / 256), dim3(256), 0, c->stream, c->unk_ptr, c->unk_ent,
                       (const T*)B.cy, c->ncs, B.c1, sc);
    LAUNCH_OK();
    symv<T>(c, B.Ainv, c->ncs, B.c1, res, sc);
    return res;
}
template const double* coarse_solve<double>(tgms_ctx*, const double*);
template const float* coarse_solve<float>(tgms_ctx*, const double*);

template <typename T>
void coarse_apply(tgms_ctx* c, const T* g, T* z, bool accumulate, const double* sc) {
    const CoarseBufs<T> B = coarse_bufs<T>(c);
    {
        ProfScope ps(c, PK_RESTRICT);
        hipLaunchKernelGGL((k_coarse_restrict<T>), dim3(c->nblk), dim3(256), 0, c->stream, B.W, c->mu, c->blk_nu, g,
                           c->nx, c->bx, c->by, c->Nx, B.cy, sc);
        LAUNCH_OK();
    }
    const T* res = coarse_solve<T>(c, sc);
    ProfScope ps(c, PK_PROLONG);
    hipLaunchKernelGGL((k_coarse_prolong<T>), dim3(c->nblk), dim3(256), 0, c->stream, B.W, c->mu, c->blk_unk,
                       c->blk_nu, res, c->nx, c->bx, c->by, c->Nx, z, accumulate ? 1 : 0, sc);
    LAUNCH_OK();
}
template void coarse_apply<double>(tgms_ctx*, const double*, double*, bool, const double*);
template void coarse_apply<float>(tgms_ctx*, const float*, float*, bool, const double*);

}  // namespace tgms
