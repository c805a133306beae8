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

// Same solve with the factor F already in LDS: operands are read from LDS inside
// the multiply-add loops (no register staging).
template <typename T>
__device__ inline void btri_solve_lds(const T* F, int m, int mh, T* vec, T* tb, T* xb) {
    const int lane = threadIdx.x;  // every thread of the workgroup passes the barriers; lanes >= m idle
    const int tri = btri_tri(m);
    const int bs = tri + btri_hes(m);
    const T* S = F + mh * bs;
    const bool act = lane < m;
    const int la = act ? lane : 0;
    for (int j = 0; j < mh; ++j) {
        const T* D = F + j * bs;
        T t = act ? vec[j * m + lane] * S[j * m + lane] : T(0);
        if (j > 0) {
            const T* E = F + (j - 1) * bs + tri;
            T a0 = T(0), a1 = T(0);
            const int c0 = la > 0 ? la - 1 : 0;
            int c = c0;
#pragma unroll 4
            for (; c + 1 < m; c += 2) {
                a0 += E[btri_offE(c) + la] * xb[c];
                a1 += E[btri_offE(c + 1) + la] * xb[c + 1];
            }
            if (c < m) a0 += E[btri_offE(c) + la] * xb[c];
            if (act) t -= a0 + a1;
        }
        if (act) tb[lane] = t;
        __syncthreads();
        T y0 = T(0), y1 = T(0);
        int c = 0;
#pragma unroll 4
        for (; c + 1 <= la; c += 2) {
            y0 += D[btri_offD(c, m) + la - c] * tb[c];
            y1 += D[btri_offD(c + 1, m) + la - c - 1] * tb[c + 1];
        }
        if (c <= la) y0 += D[btri_offD(c, m) + la - c] * tb[c];
        __syncthreads();
        if (act) {
            xb[lane] = y0 + y1;
            vec[j * m + lane] = y0 + y1;
        }
        __syncthreads();
    }
    for (int j = mh - 1; j >= 0; --j) {
        const T* D = F + j * bs;
        T t = act ? vec[j * m + lane] : T(0);
        if (j + 1 < mh) {
            const T* E = F + j * bs + tri + btri_offE(la);
            const int rmax = la + 1 < m ? la + 1 : m - 1;
            T a0 = T(0), a1 = T(0);
            int r = 0;
#pragma unroll 4
            for (; r + 1 <= rmax; r += 2) {
                a0 += E[r] * xb[r];
                a1 += E[r + 1] * xb[r + 1];
            }
            if (r <= rmax) a0 += E[r] * xb[r];
            if (act) t -= a0 + a1;
        }
        if (act) tb[lane] = t;
        __syncthreads();
        const T* Dc = D + btri_offD(la, m) - la;
        T w0 = T(0), w1 = T(0);
        int r = la;
#pragma unroll 4
        for (; r + 1 < m; r += 2) {
            w0 += Dc[r] * tb[r];
            w1 += Dc[r + 1] * tb[r + 1];
        }
        if (r < m) w0 += Dc[r] * tb[r];
        __syncthreads();
        if (act) {
            xb[lane] = w0 + w1;
            vec[j * m + lane] = (w0 + w1) * S[j * m + lane];
        }
        __syncthreads();
    }
}

// Solve with the factor in LDS and the row width M fixed at compile time.  The lanes
// form P = 64/M groups of M (lane = p*M + a): group p accumulates the columns
// c = p, p+P, ... of each small matrix-vector product and the P partial sums are
// combined through pbuf (LDS, 64 entries).  vec must hold S*g on entry (pre-scaled).
template <typename T, int M>
__device__ inline void btri_solve_split(const T* F, int mh, T* vec, T* tb, T* xb, T* pbuf) {
    constexpr int P = 64 / M;
    constexpr int K = (M + P - 1) / P;
    constexpr int TRI = M * (M + 1) / 2;
    constexpr int BS = TRI + (M - 1) * (M + 2) / 2 + M;
    const int lane = threadIdx.x;
    const int p = lane / M, a = lane - p * M;
    const bool act = lane < P * M;
    const bool lead = lane < M;
    const T* S = F + mh * BS;
    for (int j = 0; j < mh; ++j) {
        T part = T(0);
        if (j > 0 && act) {
            const T* E = F + (j - 1) * BS + TRI;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int c = p + k * P;
                if (c < M && a <= c + 1) part += E[c * (c + 3) / 2 + a] * xb[c];
            }
        }
        if (act) pbuf[lane] = part;
        __syncthreads();
        if (lead) {
            T s = vec[j * M + a];
#pragma unroll
            for (int q = 0; q < P; ++q) s -= pbuf[q * M + a];
            tb[a] = s;
        }
        __syncthreads();
        part = T(0);
        if (act) {
            const T* D = F + j * BS;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int c = p + k * P;
                if (c < M && c <= a) part += D[c * M - c * (c - 1) / 2 + a - c] * tb[c];
            }
            pbuf[lane] = part;
        }
        __syncthreads();
        if (lead) {
            T y = T(0);
#pragma unroll
            for (int q = 0; q < P; ++q) y += pbuf[q * M + a];
            xb[a] = y;
            vec[j * M + a] = y;
        }
        __syncthreads();
    }
    for (int j = mh - 1; j >= 0; --j) {
        T part = T(0);
        if (j + 1 < mh && act) {
            const T* E = F + j * BS + TRI + a * (a + 3) / 2;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int r = p + k * P;
                if (r < M && r <= a + 1) part += E[r] * xb[r];
            }
        }
        if (act) pbuf[lane] = part;
        __syncthreads();
        if (lead) {
            T s = vec[j * M + a];
#pragma unroll
            for (int q = 0; q < P; ++q) s -= pbuf[q * M + a];
            tb[a] = s;
        }
        __syncthreads();
        part = T(0);
        if (act) {
            const T* Dc = F + j * BS + a * M - a * (a - 1) / 2 - a;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int r = p + k * P;
                if (r < M && r >= a) part += Dc[r] * tb[r];
            }
            pbuf[lane] = part;
        }
        __syncthreads();
        if (lead) {
            T w = T(0);
#pragma unroll
            for (int q = 0; q < P; ++q) w += pbuf[q * M + a];
            xb[a] = w;
            vec[j * M + a] = w * S[j * M + a];
        }
        __syncthreads();
    }
}

// Barrier-free variant: lane a < M owns row a; the entries of the vector a small
// product needs are broadcast from the lanes that own them with readlane, so a block
// step has no LDS round trip for the vectors and no barrier.  Matrix entries are read
// from the LDS-staged factor; the column loops are unrolled at the compile-time M.
// vec must hold S*g on entry (pre-scaled); only the first wavefront may call this.
template <typename T, int M>
__device__ inline void btri_solve_rl(const T* F, int mh, T* vec) {
    constexpr int TRI = M * (M + 1) / 2;
    constexpr int BS = TRI + (M - 1) * (M + 2) / 2 + M;
    const int lane = threadIdx.x & 63;
    const bool act = lane < M;
    const int a = act ? lane : 0;
    const T* S = F + mh * BS;
    T yprev = T(0);
    for (int j = 0; j < mh; ++j) {
        T t = act ? vec[j * M + a] : T(0);
        if (j > 0) {
            const T* E = F + (j - 1) * BS + TRI + a;
            T s0 = T(0), s1 = T(0);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const T e = (a <= c + 1) ? E[c * (c + 3) / 2] : T(0);
                const T yc = readlane(yprev, c);
                if (c & 1)
                    s1 += e * yc;
                else
                    s0 += e * yc;
            }
            t -= s0 + s1;
        }
        const T* D = F + j * BS + a;
        T y0 = T(0), y1 = T(0);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const T d = (c <= a) ? D[c * M - c * (c - 1) / 2 - c] : T(0);
            const T tc = readlane(t, c);
            if (c & 1)
                y1 += d * tc;
            else
                y0 += d * tc;
        }
        yprev = y0 + y1;
        if (act) vec[j * M + a] = yprev;
    }
    T wnext = T(0);
    for (int j = mh - 1; j >= 0; --j) {
        T t = act ? vec[j * M + a] : T(0);
        if (j + 1 < mh) {
            const T* E = F + j * BS + TRI + a * (a + 3) / 2;
            T s0 = T(0), s1 = T(0);
#pragma unroll
            for (int r = 0; r < M; ++r) {
                const T e = (r <= a + 1) ? E[r] : T(0);
                const T wr = readlane(wnext, r);
                if (r & 1)
                    s1 += e * wr;
                else
                    s0 += e * wr;
            }
            t -= s0 + s1;
        }
        const T* Dc = F + j * BS + a * M - a * (a - 1) / 2 - a;
        T w0 = T(0), w1 = T(0);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const T d = (r >= a) ? Dc[r] : T(0);
            const T tr = readlane(t, r);
            if (r & 1)
                w1 += d * tr;
            else
                w0 += d * tr;
        }
        wnext = w0 + w1;
        if (act) vec[j * M + a] = wnext * S[j * M + a];
    }
}
