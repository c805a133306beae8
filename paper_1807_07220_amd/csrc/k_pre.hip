// Preprocessing (paper section 3) and pressure recovery.
//
// Preprocessing: vbar_H solves the problem on the coarse RT0 space
// (coarse normal velocities c): c = c_p + C_H s, with c_p an explicit coarse
// flux whose block divergences are the block sums of F, and s the coarse
// stream function minimising the energy (the coarse saddle system restricted
// to its divergence-free part).  vbar_H is its fine interpolant.  Then on
// every block K (eq. subproblem) the local problem with right-hand side
// [-A vbar_H; F - B vbar_H] is solved as particular flux + C_K psi, and
// vbar = vbar_H + sum_K vbar_K satisfies B vbar = F.
//
// Pressure: the algorithm returns the velocity only; the pressure is the
// least-squares solution of B^T p = A v with zero mean.  On a uniform grid
// B B^T = hy^2 L_x (x) I + hx^2 I (x) L_y with L the 1D Neumann Laplacian,
// which the orthonormal DCT-II diagonalises, so p = Q (Lambda^+ (Q^T B A v)).
#include "common.h"
#include "band.h"
#include "block.h"

namespace {

// Fp = F - B_bnd g ; gb = g on boundary faces, 0 inside
__global__ void k_fprime(const double* __restrict__ F, const double* __restrict__ g, int nx, int ny, double hx,
                         double hy, double* __restrict__ Fp) {
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= (long long)nx * ny) return;
    const int j = (int)(c / nx), i = (int)(c % nx);
    double v = F[c];
    if (g) {
        const long long nfx = (long long)(nx + 1) * ny;
        if (i == 0) v += g[(long long)j * (nx + 1)] * hy;
        if (i == nx - 1) v -= g[(long long)j * (nx + 1) + nx] * hy;
        if (j == 0) v += g[nfx + i] * hx;
        if (j == ny - 1) v -= g[nfx + (long long)ny * nx + i] * hx;
    }
    Fp[c] = v;
}

__global__ void k_bnd_faces(const double* __restrict__ g, double* __restrict__ gb, int nx, int ny) {
    const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nfx = (long long)(nx + 1) * ny, nf = nfx + (long long)nx * (ny + 1);
    if (f >= nf) return;
    bool bnd;
    if (f < nfx) {
        const int i = (int)(f % (nx + 1));
        bnd = (i == 0 || i == nx);
    } else {
        const int j = (int)((f - nfx) / nx);
        bnd = (j == 0 || j == ny);
    }
    gb[f] = (bnd && g) ? g[f] : 0.0;
}

// block sums of F' and the sum of |F| (for the compatibility test)
__global__ void k_block_sums(const double* __restrict__ Fp, int nx, int bx, int by, int Nx, double* __restrict__ FH,
                             double* __restrict__ FabsH) {
    const int blk = blockIdx.x, I = blk % Nx, J = blk / Nx, lane = threadIdx.x;
    double s = 0.0, sa = 0.0;
    for (int e = lane; e < bx * by; e += 64) {
        const double v = Fp[(long long)(J * by + e / bx) * nx + I * bx + e % bx];
        s += v;
        sa += fabs(v);
    }
    s = wave_sum(s);
    sa = wave_sum(sa);
    if (lane == 0) {
        FH[blk] = s;
        FabsH[blk] = sa;
    }
}

// coarse velocities c = c_p + C_H s (s on interior coarse vertices)
__global__ void k_coarse_vel(const double* __restrict__ cp, const double* __restrict__ s, int Nx, int Ny, double Hx,
                             double Hy, double* __restrict__ cvel) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nxf = Ny * (Nx + 1), nyf = (Ny + 1) * Nx;
    if (e >= nxf + nyf) return;
    auto S = [&](int I, int J) -> double {
        return (I <= 0 || I >= Nx || J <= 0 || J >= Ny) ? 0.0 : s[(J - 1) * (Nx - 1) + I - 1];
    };
    if (e < nxf) {
        const int J = e / (Nx + 1), I = e % (Nx + 1);
        cvel[e] = (I == 0 || I == Nx) ? 0.0 : cp[e] + (S(I, J + 1) - S(I, J)) / Hy;
    } else {
        const int f = e - nxf, J = f / Nx, I = f % Nx;
        cvel[e] = (J == 0 || J == Ny) ? 0.0 : cp[e] - (S(I + 1, J) - S(I, J)) / Hx;
    }
}

// fine RT0 interpolant of the coarse velocities (full face layout)
__global__ void k_interp_rt0(const double* __restrict__ cvel, int nx, int ny, int bx, int by, int Nx, int Ny,
                             double* __restrict__ v) {
    const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nfx = (long long)(nx + 1) * ny, nf = nfx + (long long)nx * (ny + 1);
    if (f >= nf) return;
    const int nxf = Ny * (Nx + 1);
    double val;
    if (f < nfx) {
        const int j = (int)(f / (nx + 1)), i = (int)(f % (nx + 1));
        const int I = i / bx, a = i % bx, J = j / by;
        if (i == nx)
            val = cvel[J * (Nx + 1) + Nx];
        else {
            const double w = (double)a / bx;
            val = (1.0 - w) * cvel[J * (Nx + 1) + I] + w * cvel[J * (Nx + 1) + I + 1];
        }
    } else {
        const long long g = f - nfx;
        const int j = (int)(g / nx), i = (int)(g % nx);
        const int J = j / by, b = j % by, I = i / bx;
        if (j == ny)
            val = cvel[nxf + Ny * Nx + I];
        else {
            const double w = (double)b / by;
            val = (1.0 - w) * cvel[nxf + J * Nx + I] + w * cvel[nxf + (J + 1) * Nx + I];
        }
    }
    v[f] = val;
}

// q = Fp - B v (cell outflow residual)
__global__ void k_cell_res(const double* __restrict__ Fp, const double* __restrict__ v, int nx, int ny, double hx,
                           double hy, double* __restrict__ q) {
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= (long long)nx * ny) return;
    const int j = (int)(c / nx), i = (int)(c % nx);
    const long long nfx = (long long)(nx + 1) * ny;
    const long long xf = (long long)j * (nx + 1) + i, yf = nfx + (long long)j * nx + i;
    const double div = (v[xf + 1] - v[xf]) * hy + (v[yf + nx] - v[yf]) * hx;
    q[c] = Fp[c] - div;
}

struct PreGeom {
    int nx, ny, bx, by, Nx, Ny;
    double hx, hy, sx, sy;
};

// Block corrections (eq. subproblem), one wavefront per block; adds into vbar's block-interior faces.
template <int MW>
__global__ void __launch_bounds__(64) k_block_correct(PreGeom G, const double* __restrict__ a, const double* __restrict__ blkL,
                                const double* __restrict__ blkS, const double* __restrict__ q,
                                const double* __restrict__ Av, double* __restrict__ vbar) {
    extern __shared__ double sm[];
    const int bxl = G.bx, byl = G.by;
    const int nfx = byl * (bxl + 1), nfy = (byl + 1) * bxl, nloc = (bxl - 1) * (byl - 1);
    double* Fw = sm;
    double* Fe = Fw + byl;
    double* Fs = Fe + byl;
    double* Fn = Fs + bxl;
    double* ql = Fn + bxl;
    double* vx = ql + bxl * byl;
    double* vy = vx + nfx;
    double* ox = vy + nfy;
    double* oy = ox + nfx;
    double* g = oy + nfy;
    double* tmp = g + nloc;
    double* tb = tmp + byl + 2;
    double* xb = tb + 64;
    const int blk = blockIdx.x, I = blk % G.Nx, J = blk / G.Nx, lane = threadIdx.x;
    const long long cell0 = (long long)J * G.by * G.nx + (long long)I * G.bx;
    const double* aK = a + cell0;
    const long long nfxg = (long long)(G.nx + 1) * G.ny;
    for (int e = lane; e < 2 * byl + 2 * bxl; e += 64) Fw[e] = 0.0;
    for (int e = lane; e < bxl * byl; e += 64) ql[e] = q[cell0 + (long long)(e / bxl) * G.nx + e % bxl];
    __syncthreads();
    particular_flux(bxl, byl, Fw, Fe, Fs, Fn, ql, vx, vy, tmp);
    for (int e = lane; e < nfx; e += 64) vx[e] *= 1.0 / G.hy;
    for (int e = lane; e < nfy; e += 64) vy[e] *= 1.0 / G.hx;
    __syncthreads();
    block_mass(bxl, byl, aK, G.nx, vx, vy, ox, oy);
    // w = rf - A_K v_p with rf = -(A vbar_H) on the block's interior faces
    for (int e = lane; e < nfx; e += 64) {
        const int b = e / (bxl + 1), aa = e % (bxl + 1);
        const bool inner = aa > 0 && aa < bxl;
        const double rf = inner ? -Av[(long long)(J * byl + b) * (G.nx + 1) + I * bxl + aa] : 0.0;
        ox[e] = rf - ox[e];
    }
    for (int e = lane; e < nfy; e += 64) {
        const int b = e / bxl, aa = e % bxl;
        const bool inner = b > 0 && b < byl;
        const double rf = inner ? -Av[nfxg + (long long)(J * byl + b) * G.nx + I * bxl + aa] : 0.0;
        oy[e] = rf - oy[e];
    }
    __syncthreads();
    block_curlT(bxl, byl, ox, oy, G.sx, G.sy, 1.0, g);
    btri_solve_wave<double, MW>(blkL + (long long)blk * btri_size(bxl - 1, byl - 1), bxl - 1, byl - 1, g, tb, xb);
    __syncthreads();
    block_curl_add(bxl, byl, g, G.sx, G.sy, vx, vy);
    for (int e = lane; e < nfx; e += 64) {
        const int b = e / (bxl + 1), aa = e % (bxl + 1);
        if (aa > 0 && aa < bxl) vbar[(long long)(J * byl + b) * (G.nx + 1) + I * bxl + aa] += vx[e];
    }
    for (int e = lane; e < nfy; e += 64) {
        const int b = e / bxl, aa = e % bxl;
        if (b > 0 && b < byl) vbar[nfxg + (long long)(J * byl + b) * G.nx + I * bxl + aa] += vy[e];
    }
}

// rhs[c] = (B_I (A u)_I)_c  with Au a full face array (boundary entries ignored)
__global__ void k_press_rhs(const double* __restrict__ Au, int nx, int ny, double hx, double hy,
                            double* __restrict__ rhs) {
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= (long long)nx * ny) return;
    const int j = (int)(c / nx), i = (int)(c % nx);
    const long long nfx = (long long)(nx + 1) * ny;
    const long long xf = (long long)j * (nx + 1) + i, yf = nfx + (long long)j * nx + i;
    double s = 0.0;
    if (i + 1 < nx) s += hy * Au[xf + 1];
    if (i > 0) s -= hy * Au[xf];
    if (j + 1 < ny) s += hx * Au[yf + nx];
    if (j > 0) s -= hx * Au[yf];
    rhs[c] = s;
}

__global__ void k_press_scale(double* __restrict__ P, const double* __restrict__ lx, const double* __restrict__ ly,
                              int nx, int ny, double hx2, double hy2) {
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= (long long)nx * ny) return;
    const int j = (int)(c / nx), i = (int)(c % nx);
    const double d = hy2 * lx[i] + hx2 * ly[j];
    P[c] = (i == 0 && j == 0) ? 0.0 : P[c] / d;
}

inline unsigned nb(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Orthonormal DCT-II matrix Q[i][k] = s_k cos(pi k (i + 1/2) / n) (s_0 = sqrt(1/n),
// s_k = sqrt(2/n)) and the eigenvalues 2 - 2 cos(pi k / n) of the 1-D Neumann
// Laplacian it diagonalises.
__global__ void k_dct_matrix(int n, double* __restrict__ Q, double* __restrict__ lam) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    const int i = (int)(e / n), k = (int)(e % n);
    Q[e] = (k == 0 ? sqrt(1.0 / n) : sqrt(2.0 / n)) * cos(M_PI * k * (i + 0.5) / n);
    if (i == 0) lam[k] = 2.0 - 2.0 * cos(M_PI * k / n);
}

}  // namespace

namespace tgms {

// vbar (full face array, boundary entries 0); Fp = F - B_bnd g.  Host-side coarse sweep.
void preprocess(tgms_ctx* c, const double* F, const double* g_bnd, double* vbar, double* Fp) {
    const long long ncell = (long long)c->nx * c->ny;
    hipLaunchKernelGGL(k_fprime, dim3(nb(ncell)), dim3(256), 0, c->stream, F, g_bnd, c->nx, c->ny, c->hx, c->hy, Fp);
    LAUNCH_OK();
    double* FH = c->blkbuf;  // nblk block sums, then nblk sums of |F|
    double* FabsH = c->blkbuf + c->nblk;
    hipLaunchKernelGGL(k_block_sums, dim3(c->nblk), dim3(64), 0, c->stream, (const double*)Fp, c->nx, c->bx, c->by,
                       c->Nx, FH, FabsH);
    LAUNCH_OK();
    // the block sums and the coarse RT0 block masses, read back with one wait
    std::vector<double> fh(2 * c->nblk), ah(6 * c->nblk);
    HIP_OK(hipMemcpyAsync(fh.data(), FH, sizeof(double) * 2 * c->nblk, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipMemcpyAsync(ah.data(), c->AH0, sizeof(double) * 6 * c->nblk, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    const int Nx = c->Nx, Ny = c->Ny;
    double tot = 0.0, tabs = 0.0;
    for (int b = 0; b < c->nblk; ++b) {
        tot += fh[b];
        tabs += fh[c->nblk + b];
    }
    if (std::fabs(tot) > 1e-12 * (tabs > 0 ? tabs : 1.0) + 1e-300)
        throw TgmsError{TGMS_E_INCOMPAT, "sources are incompatible with the boundary flux (sum F - outflow = " +
                                             std::to_string(tot) + ")"};
    // coarse particular flux: interior horizontal coarse lines carry the running row imbalance,
    // spread uniformly; x-fluxes follow from the block balances.
    const double Hx = c->bx * c->hx, Hy = c->by * c->hy;
    const int nxf = Ny * (Nx + 1), nyf = (Ny + 1) * Nx;
    std::vector<double> Fx(nxf, 0.0), Fy(nyf, 0.0), cp(nxf + nyf, 0.0);
    double Y = 0.0;
    for (int J = 0; J < Ny; ++J) {
        double row = 0.0;
        for (int I = 0; I < Nx; ++I) row += fh[J * Nx + I];
        Y += row;
        if (J + 1 < Ny)
            for (int I = 0; I < Nx; ++I) Fy[(J + 1) * Nx + I] = Y / Nx;
    }
    for (int J = 0; J < Ny; ++J)
        for (int I = 0; I + 1 < Nx; ++I)
            Fx[J * (Nx + 1) + I + 1] = Fx[J * (Nx + 1) + I] + fh[J * Nx + I] - Fy[(J + 1) * Nx + I] + Fy[J * Nx + I];
    for (int e = 0; e < nxf; ++e) cp[e] = Fx[e] / Hy;
    for (int e = 0; e < nyf; ++e) cp[nxf + e] = Fy[e] / Hx;
    // rhs_s = -C_H^T A_H0 c_p  (per block: 2x2 mass for the x pair and the y pair)
    std::vector<double> rhs(c->nv > 0 ? c->nv : 1, 0.0);
    auto vid = [&](int I, int J) { return (I <= 0 || I >= Nx || J <= 0 || J >= Ny) ? -1 : (J - 1) * (Nx - 1) + I - 1; };
    for (int J = 0; J < Ny; ++J)
        for (int I = 0; I < Nx; ++I) {
            const double* m = &ah[6 * (J * Nx + I)];
            const double cW = cp[J * (Nx + 1) + I], cE = cp[J * (Nx + 1) + I + 1];
            const double cS = cp[nxf + J * Nx + I], cN = cp[nxf + (J + 1) * Nx + I];
            const double gW = m[0] * cW + m[1] * cE, gE = m[1] * cW + m[2] * cE;
            const double gS = m[3] * cS + m[4] * cN, gN = m[4] * cS + m[5] * cN;
            // c_W = (s(I,J+1)-s(I,J))/Hy, c_E = (s(I+1,J+1)-s(I+1,J))/Hy,
            // c_S = -(s(I+1,J)-s(I,J))/Hx, c_N = -(s(I+1,J+1)-s(I,J+1))/Hx
            auto add = [&](int I2, int J2, double v) {
                const int k = vid(I2, J2);
                if (k >= 0) rhs[k] -= v;
            };
            add(I, J + 1, gW / Hy);
            add(I, J, -gW / Hy);
            add(I + 1, J + 1, gE / Hy);
            add(I + 1, J, -gE / Hy);
            add(I + 1, J, -gS / Hx);
            add(I, J, gS / Hx);
            add(I + 1, J + 1, -gN / Hx);
            add(I, J + 1, gN / Hx);
        }
    double* cpd = c->cflux + (nxf + nyf);
    HIP_OK(hipMemcpyAsync(cpd, cp.data(), sizeof(double) * (nxf + nyf), hipMemcpyHostToDevice, c->stream));
    if (c->nv > 0) {
        HIP_OK(hipMemcpyAsync(c->svec2, rhs.data(), sizeof(double) * c->nv, hipMemcpyHostToDevice, c->stream));
        if (c->kb.nb > 0) {
            copy(c, c->nv, c->svec2, c->kb.x);
            bcr_solve<double>(c, c->kb, c->kb.x, nullptr);
            copy(c, c->nv, c->kb.x, c->svec);
        } else {
            double* save = c->cvec2;
            c->cvec2 = c->svec2 + c->nv;  // temporary of the triangular products
            symv<double>(c, c->KH, c->nv, c->svec2, c->svec, nullptr);
            c->cvec2 = save;
        }
    }
    hipLaunchKernelGGL(k_coarse_vel, dim3(nb(nxf + nyf)), dim3(256), 0, c->stream, (const double*)cpd,
                       (const double*)c->svec, Nx, Ny, Hx, Hy, c->cflux);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_interp_rt0, dim3(nb(c->nf)), dim3(256), 0, c->stream, (const double*)c->cflux, c->nx, c->ny,
                       c->bx, c->by, Nx, Ny, vbar);
    LAUNCH_OK();
    faces_A_probe(c, vbar, c->fu);
    hipLaunchKernelGGL(k_cell_res, dim3(nb(ncell)), dim3(256), 0, c->stream, (const double*)Fp, (const double*)vbar,
                       c->nx, c->ny, c->hx, c->hy, c->cellw);
    LAUNCH_OK();
    PreGeom G{c->nx, c->ny, c->bx, c->by, Nx, Ny, c->hx, c->hy, c->sx, c->sy};
    const int nfxl = c->by * (c->bx + 1), nfyl = (c->by + 1) * c->bx, nloc = (c->bx - 1) * (c->by - 1);
    size_t lds = sizeof(double) * (2 * c->by + 2 * c->bx + c->bx * c->by + 2 * (nfxl + nfyl) + nloc + c->by + 2 + 128);
    const int mw = btri_width(c->bx - 1);
    if (mw == 16)
        hipLaunchKernelGGL((k_block_correct<16>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL, c->blkS,
                           (const double*)c->cellw, (const double*)c->fu, vbar);
    else if (mw == 24)
        hipLaunchKernelGGL((k_block_correct<24>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL, c->blkS,
                           (const double*)c->cellw, (const double*)c->fu, vbar);
    else
        hipLaunchKernelGGL((k_block_correct<32>), dim3(c->nblk), dim3(64), lds, c->stream, G, c->a, c->blkL, c->blkS,
                           (const double*)c->cellw, (const double*)c->fu, vbar);
    LAUNCH_OK();
}

void bnd_faces(tgms_ctx* c, const double* g, double* gb) {
    hipLaunchKernelGGL(k_bnd_faces, dim3(nb(c->nf)), dim3(256), 0, c->stream, g, gb, c->nx, c->ny);
    LAUNCH_OK();
}

// p = argmin |B_I^T p - (A u)_I| with zero mean, via the DCT-II diagonalisation of B B^T.
void dct_matrix(tgms_ctx* c, int n, double* Q, double* lam) {
    const long long tot = (long long)n * n;
    hipLaunchKernelGGL(k_dct_matrix, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, n, Q, lam);
    LAUNCH_OK();
}

void pressure(tgms_ctx* c, const double* u, double* p) {
    const long long ncell = (long long)c->nx * c->ny;
    faces_A(c, u, c->fu);
    hipLaunchKernelGGL(k_press_rhs, dim3(nb(ncell)), dim3(256), 0, c->stream, (const double*)c->fu, c->nx, c->ny,
                       c->hx, c->hy, c->cellw);
    LAUNCH_OK();
    const int nx = c->nx, ny = c->ny;
    double* T1 = c->cellw2;
    // P^ = Qy^T R Qx
    gemm(c, 0, 0, ny, nx, nx, 1.0, c->cellw, nx, c->Qx, nx, 0.0, T1, nx);
    gemm(c, 1, 0, ny, nx, ny, 1.0, c->Qy, ny, T1, nx, 0.0, c->cellw, nx);
    hipLaunchKernelGGL(k_press_scale, dim3(nb(ncell)), dim3(256), 0, c->stream, c->cellw, c->lamx, c->lamy, nx, ny,
                       c->hx * c->hx, c->hy * c->hy);
    LAUNCH_OK();
    // p = Qy P^ Qx^T
    gemm(c, 0, 1, ny, nx, nx, 1.0, c->cellw, nx, c->Qx, nx, 0.0, T1, nx);
    gemm(c, 0, 0, ny, nx, ny, 1.0, c->Qy, ny, T1, nx, 0.0, p, nx);
}

}  // namespace tgms
