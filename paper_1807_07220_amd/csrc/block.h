// Block-local helpers on one coarse block (bxl x byl cells), executed by one
// wavefront: an explicit particular flux, the block-local RT0 mass matrix,
// and the local curl / transposed curl on the block's interior vertices.
#pragma once
#include "common.h"

// ---- explicit particular flux on a bxl x byl block (fluxes = velocity * face length).
// Inputs in LDS: Fw[byl], Fe[byl], Fs[bxl], Fn[bxl], q[byl*bxl] (cell outflow).
// Output in LDS: Fx[byl*(bxl+1)], Fy[(byl+1)*bxl]; tmp needs byl+1 entries.
// Interior horizontal lines carry the running row imbalance spread uniformly;
// x-fluxes then follow from the cell balances row by row.
__device__ inline void particular_flux(int bxl, int byl, const double* Fw, const double* Fe, const double* Fs,
                                const double* Fn, const double* q, double* Fx, double* Fy, double* tmp) {
    const int lane = threadIdx.x & 63;
    for (int b = lane; b < byl; b += 64) {
        double s = 0.0;
        for (int a = 0; a < bxl; ++a) s += q[b * bxl + a];
        tmp[b + 1] = s;
    }
    __syncthreads();
    if (lane == 0) {
        double Y = 0.0;
        for (int a = 0; a < bxl; ++a) Y += Fs[a];
        tmp[0] = Y;
        for (int b = 0; b < byl; ++b) {
            Y = Y + tmp[b + 1] - Fe[b] + Fw[b];
            tmp[b + 1] = Y;
        }
    }
    __syncthreads();
    for (int e = lane; e < (byl + 1) * bxl; e += 64) {
        const int b = e / bxl, a = e % bxl;
        Fy[e] = (b == 0) ? Fs[a] : (b == byl ? Fn[a] : tmp[b] / bxl);
    }
    __syncthreads();
    for (int b = lane; b < byl; b += 64) {
        double* row = Fx + b * (bxl + 1);
        row[0] = Fw[b];
        for (int a = 0; a + 1 < bxl; ++a)
            row[a + 1] = row[a] + q[b * bxl + a] - Fy[(b + 1) * bxl + a] + Fy[b * bxl + a];
        row[bxl] = Fe[b];
    }
    __syncthreads();
}

// Block-local mass matrix applied to a block face field (velocities), all faces of the block.
__device__ inline void block_mass(int bxl, int byl, const double* __restrict__ aK, int nx, const double* vx,
                           const double* vy, double* ox, double* oy) {
    const int lane = threadIdx.x & 63;
    const double c3 = 1.0 / 3.0, c6 = 1.0 / 6.0;
    for (int e = lane; e < byl * (bxl + 1); e += 64) {
        const int b = e / (bxl + 1), a = e % (bxl + 1);
        const double* vr = vx + b * (bxl + 1);
        double s = 0.0;
        if (a > 0) s += aK[(long long)b * nx + a - 1] * (vr[a] * c3 + vr[a - 1] * c6);
        if (a < bxl) s += aK[(long long)b * nx + a] * (vr[a] * c3 + vr[a + 1] * c6);
        ox[e] = s;
    }
    for (int e = lane; e < (byl + 1) * bxl; e += 64) {
        const int b = e / bxl, a = e % bxl;
        double s = 0.0;
        if (b > 0) s += aK[(long long)(b - 1) * nx + a] * (vy[e] * c3 + vy[e - bxl] * c6);
        if (b < byl) s += aK[(long long)b * nx + a] * (vy[e] * c3 + vy[e + bxl] * c6);
        oy[e] = s;
    }
    __syncthreads();
}

// g = scale * C_K^T w on the interior vertices of the block (row-major, width bxl-1).
__device__ inline void block_curlT(int bxl, int byl, const double* wx, const double* wy, double sx, double sy,
                            double scale, double* g) {
    const int lane = threadIdx.x & 63;
    const int m = bxl - 1, n = (bxl - 1) * (byl - 1);
    for (int r = lane; r < n; r += 64) {
        const int p = r % m + 1, q = r / m + 1;  // local vertex (p, q)
        const double xs = wx[(q - 1) * (bxl + 1) + p], xn = wx[q * (bxl + 1) + p];
        const double yw = wy[q * bxl + p - 1], ye = wy[q * bxl + p];
        g[r] = scale * (sx * (xs - xn) + sy * (ye - yw));
    }
    __syncthreads();
}

// v += C_K psi (psi on interior vertices, zero on the block boundary).
__device__ inline void block_curl_add(int bxl, int byl, const double* psi, double sx, double sy, double* vx,
                               double* vy) {
    const int lane = threadIdx.x & 63;
    const int m = bxl - 1;
    auto P = [&](int p, int q) -> double {
        return (p <= 0 || p >= bxl || q <= 0 || q >= byl) ? 0.0 : psi[(q - 1) * m + p - 1];
    };
    for (int e = lane; e < byl * (bxl + 1); e += 64) {
        const int b = e / (bxl + 1), a = e % (bxl + 1);
        vx[e] += (P(a, b + 1) - P(a, b)) * sx;
    }
    for (int e = lane; e < (byl + 1) * bxl; e += 64) {
        const int b = e / bxl, a = e % bxl;
        vy[e] -= (P(a + 1, b) - P(a, b)) * sy;
    }
    __syncthreads();
}

