// Wavefront solver for the local stream-function systems (block-row form).
//
// A rectangle's interior vertices form mh rows of m vertices; in row-major
// order the equilibrated matrix S M S is block tridiagonal with m x m blocks,
// and its Cholesky factor L is block bidiagonal:
//   L_jj     lower triangular (dense inside the band),
//   L_{j+1,j} upper Hessenberg (row a is nonzero for columns >= a-1).
// The factor is stored per block row j as
//   [ D_j = L_jj^{-1}, lower triangular, packed by columns (column c holds rows c..m-1) ]
//   [ E_j = L_{j+1,j}, packed by columns (column c holds rows 0..min(c+1, m-1)) ]
// followed by the n = m*mh entries of the equilibration scale S.
// Both pieces together hold the same number of words as the band factor.
//
// Forward  L y = S g :  y_j = D_j (S g_j - E_{j-1} y_{j-1})
// Backward L^T w = y :  w_j = D_j^T (y_j - E_j^T w_{j+1}),  result S w.
// Lane a owns entry a of every block vector; the 2*mh block steps are the
// only sequential chain, and every load of a step is issued together.
#pragma once
#include "common.h"

#define TGMS_MMAX 32  // largest supported m (vertices per row of a rectangle)

// smallest register-array width (16, 24 or 32) that holds m
inline int btri_width(int m) { return m <= 16 ? 16 : (m <= 24 ? 24 : 32); }

__host__ __device__ inline int btri_tri(int m) { return m * (m + 1) / 2; }
__host__ __device__ inline int btri_hes(int m) { return (m - 1) * (m + 2) / 2 + m; }
__host__ __device__ inline long long btri_size(int m, int mh) {
    return (long long)mh * (btri_tri(m) + btri_hes(m)) + (long long)m * mh;
}
__host__ __device__ inline int btri_offD(int c, int m) { return c * m - c * (c - 1) / 2; }
__host__ __device__ inline int btri_offE(int c) { return c * (c + 3) / 2; }

// vec (LDS, n = m*mh): g on entry, M^{-1} g on exit.  tb, xb: LDS scratch of m entries each.
template <typename T, int MW = TGMS_MMAX>
__device__ inline void btri_solve_wave(const T* __restrict__ F, int m, int mh, T* vec, T* tb, T* xb) {
    const int lane = threadIdx.x & 63;
    const int tri = btri_tri(m);
    const long long bs = tri + btri_hes(m);
    const T* S = F + (long long)mh * bs;
    const bool act = lane < m;
    // forward sweep
    for (int j = 0; j < mh; ++j) {
        const T* D = F + (long long)j * bs;
        T t = act ? vec[j * m + lane] * S[j * m + lane] : T(0);
        if (j > 0) {
            const T* E = F + (long long)(j - 1) * bs + tri;
            T e[MW];
#pragma unroll
            for (int c = 0; c < MW; ++c)
                e[c] = (c < m && act && c + 1 >= lane) ? E[btri_offE(c) + lane] : T(0);
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < MW; ++c)
                if (c < m) acc += e[c] * xb[c];
            t -= acc;
        }
        T d[MW];
#pragma unroll
        for (int c = 0; c < MW; ++c) d[c] = (c < m && act && c <= lane) ? D[btri_offD(c, m) + lane - c] : T(0);
        if (act) tb[lane] = t;
        __syncthreads();
        T y = T(0);
#pragma unroll
        for (int c = 0; c < MW; ++c)
            if (c < m) y += d[c] * tb[c];
        __syncthreads();
        if (act) {
            xb[lane] = y;
            vec[j * m + lane] = y;
        }
        __syncthreads();
    }
    // backward sweep (xb holds w_{j+1})
    for (int j = mh - 1; j >= 0; --j) {
        const T* D = F + (long long)j * bs;
        T t = act ? vec[j * m + lane] : T(0);
        if (j + 1 < mh) {
            const T* E = F + (long long)j * bs + tri + btri_offE(lane < m ? lane : 0);
            T e[MW];
#pragma unroll
            for (int r = 0; r < MW; ++r) e[r] = (r < m && act && r <= lane + 1) ? E[r] : T(0);
            T acc = T(0);
#pragma unroll
            for (int r = 0; r < MW; ++r)
                if (r < m) acc += e[r] * xb[r];
            t -= acc;
        }
        const T* Dc = D + btri_offD(lane < m ? lane : 0, m) - (lane < m ? lane : 0);  // Dc[r] = D(r, lane)
        T d[MW];
#pragma unroll
        for (int r = 0; r < MW; ++r) d[r] = (r < m && act && r >= lane) ? Dc[r] : T(0);
        if (act) tb[lane] = t;
        __syncthreads();
        T w = T(0);
#pragma unroll
        for (int r = 0; r < MW; ++r)
            if (r < m) w += d[r] * tb[r];
        __syncthreads();
        if (act) {
            xb[lane] = w;
            vec[j * m + lane] = w * S[j * m + lane];
        }
        __syncthreads();
    }
}
