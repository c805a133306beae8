// Wavefront band solver for an equilibrated band Cholesky factor.
//
// Solves M w = g where S M S = L L^T, L lower triangular with bandwidth b < 64,
// stored column band: L[c*(b+1) + t] = L(c+t, c) for t = 1..b and
// L[c*(b+1)] = 1 / L(c, c).  vec (LDS, n entries) holds g on entry and w on
// exit.  One wavefront executes the call; every lane must enter it.
//
// Forward sweep (L y = S g): lane p keeps the running value of the row r with
// r = p (mod 64); after row r is final its value is broadcast and the b rows
// below it are updated (column-oriented, no reduction); lane r%64 then loads
// row r+64.  Backward sweep (L^T w = y): each row is a dot product of column
// r of L with w_{r+1..r+b}, which the lanes hold in the same rotating layout.
#pragma once
#include "common.h"

template <typename T>
__device__ inline void band_solve_wave(const T* __restrict__ L, const T* __restrict__ S, int n, int b, T* vec) {
    const int lane = threadIdx.x & 63;
    const long long ld = b + 1;
    T acc = (lane < n) ? vec[lane] * S[lane] : T(0);
    for (int r = 0; r < n; ++r) {
        const int lr = r & 63;
        const T y = readlane(acc, lr) * L[(long long)r * ld];
        const int t = (lane - r) & 63;
        if (lane == lr) {
            vec[r] = y;
            if (r + 64 < n) acc = vec[r + 64] * S[r + 64];
        } else if (t <= b && r + t < n) {
            acc -= L[(long long)r * ld + t] * y;
        }
    }
    __syncthreads();
    T wreg = T(0);
    for (int r = n - 1; r >= 0; --r) {
        const int lr = r & 63;
        const int t = (lane - r) & 63;
        T prod = (t >= 1 && t <= b && r + t < n) ? L[(long long)r * ld + t] * wreg : T(0);
        const T s = wave_sum(prod);
        if (lane == lr) {
            const T w = (vec[r] - s) * L[(long long)r * ld];
            wreg = w;
            vec[r] = w * S[r];
        }
    }
}
