// Dense FP64 Cholesky of the coarse SPD operator and its application.
//
// The coarse problem (paper eq. coarsepre, L_H = R_H L R_H^T) is solved
// exactly ("direct solver", section 5).  After restriction to its
// divergence-free subspace it is SPD; it is factorised A = L L^T by a blocked
// right-looking Cholesky, then X = L^{-1} is formed by block forward
// substitution.  The factor is kept as one n x n array
//     B = tril(X) + triu(X^T, 1),
// so A^{-1} g = X^T (X g) costs two triangular matrix-vector products that
// each stream one triangle of B row by row.
#include <functional>
#include <vector>

#include "common.h"

namespace {

constexpr int TB = 64;   // output tile
constexpr int NT = 256;  // threads (16 x 16), 4 x 4 outputs each

// C = alpha * op(A) * op(B) + beta * C ; row-major; op(A) is M x K, op(B) is K x N.
// lower_only: skip output tiles strictly above the diagonal (tile row < tile col).
// 64 x 64 output tile per workgroup; each of the 4 wavefronts owns a 32 x 32 quarter made
// of 2 x 2 FP64 MFMA 16x16x4 blocks.  Operand layout of v_mfma_f64_16x16x4f64: lane l
// holds A[l%16][l/16] and B[l/16][l%16]; result element r of lane l is D[4*r + l/16][l%16].
typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int TKG = 32;                  // k step of the GEMM tile
constexpr int GLD = TB * TKG / NT;       // elements of A (and of B) each thread loads per k step

// 64 x 64 output tile of C = alpha op(A) op(B) + beta C.  Software-pipelined: the next
// k step's operands are loaded into registers while the current one is multiplied
// from LDS.
// kbeg (a multiple of TKG): the sum starts there (the terms before it are known zeros).
__device__ inline void gemm_tile(int tm, int tn, int transA, int transB, int M, int N, int K, double alpha,
                                 const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                                 double beta, double* C, int ldc, int kbeg = 0) {
    __shared__ double As[TKG][TB + 1];
    __shared__ double Bs[TKG][TB + 1];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int m0 = tm * TB, n0 = tn * TB;
    d4_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;
    double ra[GLD], rb[GLD];
    // element e of a k step: (row or column of the tile, k) with consecutive threads on
    // consecutive addresses of the operand as stored
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < GLD; ++q) {
            const int e = tid + NT * q;
            const int mm = transA ? e % TB : e / TKG, kk = transA ? e / TB : e % TKG;
            const int gm = m0 + mm, gk = k0 + kk;
            ra[q] = (gm < M && gk < K) ? (transA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk]) : 0.0;
            const int nn = transB ? e / TKG : e % TB, kb = transB ? e % TKG : e / TB;
            const int gn = n0 + nn, gk2 = k0 + kb;
            rb[q] = (gn < N && gk2 < K) ? (transB ? B[(long long)gn * ldb + gk2] : B[(long long)gk2 * ldb + gn]) : 0.0;
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int q = 0; q < GLD; ++q) {
            const int e = tid + NT * q;
            const int mm = transA ? e % TB : e / TKG, kk = transA ? e / TB : e % TKG;
            As[kk][mm] = ra[q];
            const int nn = transB ? e / TKG : e % TB, kb = transB ? e % TKG : e / TB;
            Bs[kb][nn] = rb[q];
        }
    };
    gload(kbeg);
    lstore();
    __syncthreads();
    for (int k0 = kbeg; k0 < K; k0 += TKG) {
        const bool more = k0 + TKG < K;
        if (more) gload(k0 + TKG);  // in flight while this step multiplies
#pragma unroll
        for (int k4 = 0; k4 < TKG; k4 += 4) {
            const double a0 = As[k4 + lk][wm + li], a1 = As[k4 + lk][wm + 16 + li];
            const double b0 = Bs[k4 + lk][wn + li], b1 = Bs[k4 + lk][wn + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            lstore();
            __syncthreads();
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * a + 4 * r + lk, gn = n0 + wn + 16 * b + li;
                if (gm >= M || gn >= N) continue;
                double* cp = C + (long long)gm * ldc + gn;
                *cp = alpha * acc[a][b][r] + (beta == 0.0 ? 0.0 : beta * *cp);
            }
}

__global__ void __launch_bounds__(NT) k_gemm(int transA, int transB, int M, int N, int K, double alpha,
                                             const double* __restrict__ A, int lda, const double* __restrict__ B,
                                             int ldb, double beta, double* C, int ldc, int lower_only) {
    const int tm = blockIdx.y, tn = blockIdx.x;
    if (lower_only && tm < tn) return;
    gemm_tile(tm, tn, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

// The lower tiles (tn <= tm) of an nt x nt tile grid on a 1D grid of nt (nt + 1) / 2
// workgroups.  Workgroups are dealt to the 8 XCDs in turn; tile t of a contiguous,
// equal share of the row-major triangle goes to each XCD, so the tiles of one tile row
// (which read the same rows of op(A)) mostly meet in one L2.
__global__ void __launch_bounds__(NT) k_gemm_lower(int transA, int transB, int M, int N, int K, double alpha,
                                                   const double* __restrict__ A, int lda, const double* __restrict__ B,
                                                   int ldb, double beta, double* C, int ldc) {
    constexpr int NX = 8;
    const int T = gridDim.x, lin = blockIdx.x;
    const int x = lin % NX, l = lin / NX, q = T / NX, r = T % NX;
    const int t = x * q + min(x, r) + l;  // a bijection of [0, T)
    int tm = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    while (tm * (tm + 1) / 2 > t) --tm;
    const int tn = t - tm * (tm + 1) / 2;
    gemm_tile(tm, tn, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

// One level of the recursive inversion X = L^{-1} (n x n, row-major): for every node
// [o, o + n1 + n2) of the level, with X11 and X22 already formed,
//   step 0:  T = L21 X11          (n2 x n1, at Tm + toff, ld n1)
//   step 1:  X21 = -X22 T
// the nodes of a level are disjoint, so one launch covers all of them (blockIdx.z).
constexpr int LEVEL_MAX = 64;
struct InvLevel {
    int count;
    int o[LEVEL_MAX], n1[LEVEL_MAX], n2[LEVEL_MAX];
    long long toff[LEVEL_MAX];
};

__global__ void __launch_bounds__(NT) k_inv_level(InvLevel lv, int step, const double* __restrict__ L,
                                                  double* __restrict__ X, double* __restrict__ Tm, int n) {
    const int z = blockIdx.z;
    const int o = lv.o[z], n1 = lv.n1[z], n2 = lv.n2[z];
    const int tm = blockIdx.y, tn = blockIdx.x;
    if (tm * TB >= n2 || tn * TB >= n1) return;  // tiles beyond this node's output
    double* T = Tm + lv.toff[z];
    // X11 and X22 are lower triangular (zero above the diagonal, written so): the k blocks
    // above tn (step 0) and beyond tm (step 1) contribute nothing and are skipped
    if (step == 0)
        gemm_tile(tm, tn, 0, 0, n2, n1, n1, 1.0, L + (long long)(o + n1) * n + o, n, X + (long long)o * n + o, n, 0.0,
                  T, n1, tn * TB);
    else
        gemm_tile(tm, tn, 0, 0, n2, n1, min(n2, (tm + 1) * TB), -1.0, X + (long long)(o + n1) * n + o + n1, n, T, n1,
                  0.0, X + (long long)(o + n1) * n + o, n);
}

// the inverses of the diagonal blocks (Dinv, [block][64][64]) into the diagonal of X
__global__ void k_copy_diag_blocks(const double* __restrict__ Dinv, double* __restrict__ X, int n) {
    const int b = blockIdx.x, o = b * TB, len = min(TB, n - o);
    for (int e = threadIdx.x; e < len * len; e += blockDim.x) {
        const int i = e / len, j = e % len;
        X[(long long)(o + i) * n + o + j] = Dinv[(long long)b * TB * TB + i * TB + j];
    }
}

// Cholesky of the kb x kb diagonal block at (k0, k0) in place, and its inverse into Dinv (kb x kb, ld 64).
//
// Right-looking LDL^T with both factors formed in one sweep: with d_j the pivots and
// Lu the unit lower factor (A = Lu diag(d) Lu^T), S ends holding Lu[i][j] d_j below the
// diagonal and d_i on it, and U (= I at the start) ends holding Lu^{-1}, by the row
// operations U[i] -= Lu[i][j] U[j].  Then L = Lu diag(d)^{1/2} and
// L^{-1} = diag(d)^{-1/2} U.
//
// Pivots are taken in panels of 4 (one barrier each).  Thread (ty, tx) keeps rows
// 4 ty .. 4 ty + 3 by columns 4 tx .. 4 tx + 3 of S and U in registers.  The owners
// of the panel's columns of S and rows of U publish them to LDS (double-buffered by
// the panel's parity: a buffer is rewritten two panels later, after every thread
// has passed the barrier that follows its last read).  Every thread then factors the
// 4 x 4 pivot block itself, forward-substitutes the panel entries of its own rows
// and columns (w_i[a] = Lu[i][j+a] d_{j+a}), eliminates within the panel rows of U,
// and applies the rank-4 update S[i][k] -= sum_a Lu[i][j+a] w_k[a],
// U[i] -= sum_a Lu[i][j+a] U[j+a] to rows below the panel.  The multipliers of rows
// at or above the panel and the w of columns at or left of it are zero, so those
// entries are unchanged exactly; entries above the diagonal of S are never read.
// Rows and columns past kb are the identity (unit pivots, no coupling).
__device__ inline void potrf_diag(double* __restrict__ A, int lda, int k0, int kb, double* __restrict__ Dinv,
                                  int* __restrict__ fail) {
    __shared__ __align__(16) double colp[2][TB][4];
    __shared__ __align__(16) double rowp[2][4][TB];
    __shared__ __align__(16) double dg[TB];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int i0 = 4 * ty, c0 = 4 * tx;
    double S[4][4], U[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + r, k = c0 + q;
            S[r][q] = (i < kb && k <= i) ? A[(long long)(k0 + i) * lda + k0 + k] : (i == k ? 1.0 : 0.0);
            U[r][q] = i == k ? 1.0 : 0.0;
        }
    const int jtn = (kb + 3) / 4;
    for (int jt = 0; jt < jtn; ++jt) {
        const int j = 4 * jt, pb = jt & 1;
        if (tx == jt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                *reinterpret_cast<double2*>(&colp[pb][i0 + r][0]) = make_double2(S[r][0], S[r][1]);
                *reinterpret_cast<double2*>(&colp[pb][i0 + r][2]) = make_double2(S[r][2], S[r][3]);
            }
        if (ty == jt)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                *reinterpret_cast<double2*>(&rowp[pb][a][c0]) = make_double2(U[a][0], U[a][1]);
                *reinterpret_cast<double2*>(&rowp[pb][a][c0 + 2]) = make_double2(U[a][2], U[a][3]);
            }
        __syncthreads();
        // LDL^T of the pivot block: w[a][b] (b < a) = Lu[j+a][j+b] d_{j+b}, l[a][b] = Lu[j+a][j+b]
        double P[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double2 x = *reinterpret_cast<const double2*>(&colp[pb][j + a][0]);
            const double2 y = *reinterpret_cast<const double2*>(&colp[pb][j + a][2]);
            P[a][0] = x.x;
            P[a][1] = x.y;
            P[a][2] = y.x;
            P[a][3] = y.y;
        }
        double d[4], rd[4], w[4][4], l[4][4];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double da = P[a][a];
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b < a) {
                    double t = P[a][b];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (e < b) t -= l[b][e] * w[a][e];
                    w[a][b] = t;
                    l[a][b] = t * rd[b];
                    da -= l[a][b] * t;
                }
            d[a] = da;
            ok = ok && da > 0.0;
            rd[a] = 1.0 / da;
        }
        if (!ok) {  // every thread computed the same pivots: all leave together
            if (tid == 0) atomicOr(fail, 1);
            return;
        }
        // panel entries of the own rows (w, and the multipliers v of rows below the panel)
        double wr[4][4], vr[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double2 x = *reinterpret_cast<const double2*>(&colp[pb][i0 + r][0]);
            const double2 y = *reinterpret_cast<const double2*>(&colp[pb][i0 + r][2]);
            const double sv[4] = {x.x, x.y, y.x, y.y};
            const bool below = i0 + r >= j + 4;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double t = sv[a];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < a) t -= l[a][e] * wr[r][e];
                wr[r][a] = t;
                vr[r][a] = below ? t * rd[a] : 0.0;
            }
        }
        // panel entries of the own columns (zero for columns at or left of the panel)
        double wc[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 x = *reinterpret_cast<const double2*>(&colp[pb][c0 + q][0]);
            const double2 y = *reinterpret_cast<const double2*>(&colp[pb][c0 + q][2]);
            const double sv[4] = {x.x, x.y, y.x, y.y};
            double t4[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double t = sv[a];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < a) t -= l[a][e] * t4[e];
                t4[a] = t;
            }
            const bool right = c0 + q >= j + 4;
#pragma unroll
            for (int a = 0; a < 4; ++a) wc[q][a] = right ? t4[a] : 0.0;
        }
        // the panel rows of U, eliminated within the panel (own columns)
        double uf[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double2 x = *reinterpret_cast<const double2*>(&rowp[pb][a][c0]);
            const double2 y = *reinterpret_cast<const double2*>(&rowp[pb][a][c0 + 2]);
            const double uv[4] = {x.x, x.y, y.x, y.y};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double t = uv[q];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < a) t -= l[a][e] * uf[e][q];
                uf[a][q] = t;
            }
        }
        // rank-4 update of the rows below the panel
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double sv = S[r][q], uv = U[r][q];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    sv -= vr[r][a] * wc[q][a];
                    uv -= vr[r][a] * uf[a][q];
                }
                S[r][q] = sv;
                U[r][q] = uv;
            }
        // final values of the panel's columns of S and rows of U
        if (tx == jt) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (i0 + r >= j + 4)
#pragma unroll
                    for (int a = 0; a < 4; ++a) S[r][a] = wr[r][a];
            if (ty == jt)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (b < a) S[a][b] = w[a][b];
                    S[a][a] = d[a];
                }
        }
        if (ty == jt)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) U[a][q] = uf[a][q];
    }
    if (tx == ty)
#pragma unroll
        for (int r = 0; r < 4; ++r) dg[i0 + r] = S[r][r];
    __syncthreads();
    double si[4], rsi[4], rsk[4];  // sqrt(d) of the owned rows, reciprocals for rows and columns
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        si[r] = i0 + r < kb ? sqrt(dg[i0 + r]) : 1.0;
        rsi[r] = 1.0 / si[r];
        rsk[r] = 1.0 / (c0 + r < kb ? sqrt(dg[c0 + r]) : 1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + r, k = c0 + q;
            const bool in = i < kb && k < kb && k <= i;
            if (in) A[(long long)(k0 + i) * lda + k0 + k] = (k == i) ? si[r] : S[r][q] * rsk[q];
            Dinv[i * TB + k] = in ? U[r][q] * rsi[r] : 0.0;
        }
}

__global__ void __launch_bounds__(NT) k_potrf_diag(double* __restrict__ A, int lda, int k0, int kb,
                                                   double* __restrict__ Dinv, int* __restrict__ fail) {
    potrf_diag(A, lda, k0, kb, Dinv, fail);
}

// ---- batched forms: matrix z of a batch at base + z * stride (blockIdx.z) -------------
__global__ void __launch_bounds__(NT) k_potrf_diag_b(double* __restrict__ A, long long sA, int lda, int k0, int kb,
                                                     double* __restrict__ Dinv, long long sD, int* __restrict__ fail) {
    const long long z = blockIdx.z;
    potrf_diag(A + z * sA, lda, k0, kb, Dinv + z * sD, fail);
}

// batch index z -> offset (z / nin) * outer + (z % nin) * inner
struct BStride {
    long long outer, inner;
    int nin;
    __device__ long long off(long long z) const { return (z / nin) * outer + (z % nin) * inner; }
};

__global__ void __launch_bounds__(NT) k_gemm_b(int transA, int transB, int M, int N, int K, double alpha,
                                               const double* __restrict__ A, int lda, BStride sa,
                                               const double* __restrict__ B, int ldb, BStride sb, double beta,
                                               double* C, int ldc, BStride sc, int lower_only, long long z0) {
    const int tm = blockIdx.y, tn = blockIdx.x;
    if (lower_only && tm < tn) return;
    const long long z = z0 + blockIdx.z;
    gemm_tile(tm, tn, transA, transB, M, N, K, alpha, A + sa.off(z), lda, B + sb.off(z), ldb, beta, C + sc.off(z),
              ldc);
}

__global__ void k_copy_diag_blocks_b(const double* __restrict__ Dinv, long long sD, double* __restrict__ X,
                                     long long sX, int n) {
    const long long z = blockIdx.z;
    const int b = blockIdx.x, o = b * TB, len = min(TB, n - o);
    for (int e = threadIdx.x; e < len * len; e += blockDim.x) {
        const int i = e / len, j = e % len;
        X[z * sX + (long long)(o + i) * n + o + j] = Dinv[z * sD + (long long)b * TB * TB + i * TB + j];
    }
}

// k_inv_level over a batch: blockIdx.z = node + count * matrix
__global__ void __launch_bounds__(NT) k_inv_level_b(InvLevel lv, int step, const double* __restrict__ L,
                                                    double* __restrict__ X, double* __restrict__ Tm, int n,
                                                    long long sT) {
    const int node = blockIdx.z % lv.count;
    const long long z = blockIdx.z / lv.count;
    const int o = lv.o[node], n1 = lv.n1[node], n2 = lv.n2[node];
    const int tm = blockIdx.y, tn = blockIdx.x;
    if (tm * TB >= n2 || tn * TB >= n1) return;
    const long long sM = (long long)n * n;
    const double* Lz = L + z * sM;
    double* Xz = X + z * sM;
    double* T = Tm + z * sT + lv.toff[node];
    if (step == 0)
        gemm_tile(tm, tn, 0, 0, n2, n1, n1, 1.0, Lz + (long long)(o + n1) * n + o, n, Xz + (long long)o * n + o, n, 0.0,
                  T, n1, tn * TB);
    else
        gemm_tile(tm, tn, 0, 0, n2, n1, min(n2, (tm + 1) * TB), -1.0, Xz + (long long)(o + n1) * n + o + n1, n, T, n1,
                  0.0, Xz + (long long)(o + n1) * n + o, n);
}

__global__ void k_mirror_lower_b(double* __restrict__ F, int n, long long count) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long sM = (long long)n * n;
    if (e >= sM * count) return;
    const long long z = e / sM, r = e % sM;
    const int i = (int)(r / n), j = (int)(r % n);
    if (j > i) F[e] = F[z * sM + (long long)j * n + i];
}

// B[i][j] = X[i][j] (j <= i), B[i][j] = X[j][i] (j > i)
__global__ void k_pack_inverse(const double* __restrict__ X, double* __restrict__ B, int n) {
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    B[e] = (j <= i) ? X[e] : X[(long long)j * n + i];
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
    __device__ static double dot(const double2& b, const double* x) { return b.x * x[0] + b.y * x[1]; }
};
template <>
struct Vec16<float> {
    using type = float4;
    __device__ static float dot(const float4& b, const float* x) { return b.x * x[0] + b.y * x[1] + b.z * x[2] + b.w * x[3]; }
};

// sum over j in [j0, j1) of row[j] x[j] by one wavefront (row = B + base): the
// 16-byte-aligned body with vector loads, four in flight per lane, the unaligned
// head and tail one element per lane; the total in every lane.
template <typename T>
__device__ inline T row_dot(const T* __restrict__ B, long long base, int j0, int j1, const T* __restrict__ x, int lane) {
    constexpr int PER = 16 / sizeof(T);
    using V = typename Vec16<T>::type;
    int ja = j0 + (int)((PER - (base + j0) % PER) % PER);
    if (ja > j1) ja = j1;
    const int jb = ja + ((j1 - ja) / PER) * PER;
    T s = T(0);
    for (int j = j0 + lane; j < ja; j += 64) s += B[base + j] * x[j];
    for (int j = jb + lane; j < j1; j += 64) s += B[base + j] * x[j];
    const V* bv = reinterpret_cast<const V*>(B + base + ja);
    const int nv = (jb - ja) / PER;
    for (int q = lane; q < nv; q += 256) {
        V b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q + 64 * u < nv) b[u] = bv[q + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q + 64 * u < nv) s += Vec16<T>::dot(b[u], x + ja + (q + 64 * u) * PER);
    }
    return wave_sum(s);
}

// y = tril(B) x (part 0) or y = triu(B) x (part 1): one wavefront per row.
template <typename T>
__global__ void k_trimv(const T* __restrict__ B, int n, const T* __restrict__ x, T* __restrict__ y, int part,
                        const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const T s = row_dot<T>(B, (long long)row * n, part ? row : 0, part ? n : row + 1, x, lane);
    if (lane == 0) y[row] = s;
}

// Small coarse systems: y = tril(B) c with c accumulated from the block restrictions
// first (every workgroup forms all of c in LDS, in the fixed order of the
// accumulation kernel): one launch instead of two.
constexpr int ACC_MAX = 1024;
template <typename T>
__global__ void k_trimv_acc(const T* __restrict__ B, int n, const int* __restrict__ ptr, const int* __restrict__ ent,
                            const T* __restrict__ cy, T* __restrict__ y, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ T cs[ACC_MAX];
    for (int u = threadIdx.x; u < n; u += blockDim.x) {
        cs[u] = gather_sum<T>(ent, cy, ptr[u], ptr[u + 1]);
    }
    __syncthreads();
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const T s = row_dot<T>(B, (long long)row * n, 0, row + 1, cs, lane);
    if (lane == 0) y[row] = s;
}

// The same with the explicit inverse F = A^{-1} (symmetric, full rows): y = F c in
// one launch, c accumulated as above.
template <typename T>
__global__ void k_symv_acc(const T* __restrict__ F, int n, const int* __restrict__ ptr, const int* __restrict__ ent,
                           const T* __restrict__ cy, T* __restrict__ y, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ T cs[ACC_MAX];
    for (int u = threadIdx.x; u < n; u += blockDim.x) {
        cs[u] = gather_sum<T>(ent, cy, ptr[u], ptr[u + 1]);
    }
    __syncthreads();
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const T s = row_dot<T>(F, (long long)row * n, 0, n, cs, lane);
    if (lane == 0) y[row] = s;
}

// F[i][j] = F[j][i] for j > i (the upper triangle from the lower one)
__global__ void k_mirror_lower(double* __restrict__ F, int n) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    if (j > i) F[e] = F[(long long)j * n + i];
}

inline unsigned nb(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---- block cyclic reduction: Cholesky of a banded SPD matrix -------------------------
// With its unknowns numbered so that the half-bandwidth is at most bs, the coarse matrix
// is block tridiagonal in blocks of bs rows: diagonal blocks D_i, couplings Lc_i =
// A_{i, i-1}.  Cyclic reduction eliminates the blocks i = s, 3s, 5s, ... (s = 1, 2, 4,
// ...) level by level: C_i = chol(D_i), Gm_i = C_i^{-1} A_{i, i-s}, Gp_i = C_i^{-1}
// A_{i, i+s}; the surviving blocks e (multiples of 2s) take the Schur complements
// D_e -= Gp_{e-s}^T Gp_{e-s} + Gm_{e+s}^T Gm_{e+s} and the new coupling
// A_{e, e-2s} = -Gp_{e-s}^T Gm_{e-s}; block 0 is left last.  This is the Cholesky
// factorisation of the matrix in the odd-even order of its blocks (block factor
// diagonal C_i, off-diagonal Gm_i^T, Gp_i^T); it is stored as C_i^{-1} (lower), Gm_i,
// Gp_i.  A solve is one forward and one backward pass over the levels.  Truncated
// (bcr_factor's truncate): the levels stop at the first step whose surviving blocks
// 0, step, 2 step, ... hold at most symv_acc_max() unknowns; their block tridiagonal
// system (the Schur complements and couplings of that level) is inverted explicitly in
// FP64, and the solve applies that inverse in place of the remaining levels and block 0.
constexpr int BCR_MAX = 256;  // largest block (LDS vectors of the solve kernels)

// D_i and Lc_i from the dense matrix A (n x n, row-major); rows beyond n: identity.
__global__ void k_bcr_extract(const double* __restrict__ A, int n, int bs, int nblk, double* __restrict__ D,
                              double* __restrict__ Lc) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long bb = (long long)bs * bs;
    if (e >= nblk * bb) return;
    const int i = (int)(e / bb), r = (int)((e % bb) / bs), c = (int)(e % bs);
    const long long row = (long long)i * bs + r, col = (long long)i * bs + c;
    D[e] = (row < n && col < n) ? A[row * n + col] : (r == c ? 1.0 : 0.0);
    Lc[e] = (i > 0 && row < n) ? A[row * n + col - bs] : 0.0;
}

// The diagonal blocks eliminated at level s (i = s + 2 s q, one workgroup each; top: block
// 0): Cholesky in LDS, then the inverse of the factor in place; C_i^{-1} (zero above the
// diagonal) to Ci.  A non-positive pivot sets *fail.  1024 threads: the rank-1 updates
// on a 32 x 32 thread grid, each row of the inversion's sums split over 8 lanes.
constexpr int FNT = 1024;
__global__ void __launch_bounds__(FNT) k_bcr_factor(const double* __restrict__ D, double* __restrict__ Ci, int bs,
                                                   int nblk, int s, int top, int* __restrict__ fail) {
    extern __shared__ double A[];
    __shared__ double tmp[BCR_MAX];
    const int i = top ? 0 : s + 2 * s * blockIdx.x;
    if (i >= nblk) return;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const long long bb = (long long)bs * bs;
    const double* Dg = D + i * bb;
    for (int e = tid; e < bs * bs; e += FNT) A[e] = Dg[e];
    __syncthreads();
    bool bad = false;
    for (int k = 0; k < bs; ++k) {
        const double akk = A[k * bs + k];
        bad = bad || !(akk > 0.0);
        const double d = sqrt(akk > 0.0 ? akk : 1.0);
        __syncthreads();  // every thread has read A[k][k]
        if (tid == 0) A[k * bs + k] = d;
        const double rd = 1.0 / d;
        for (int r = k + 1 + tid; r < bs; r += FNT) A[r * bs + k] *= rd;
        __syncthreads();
        for (int r = k + 1 + ty; r < bs; r += 32) {
            const double ark = A[r * bs + k];
            for (int c = k + 1 + tx; c <= r; c += 32) A[r * bs + c] -= ark * A[c * bs + k];
        }
        __syncthreads();
    }
    if (bad && tid == 0) atomicOr(fail, 1);
    // X = L^{-1} in place, column by column from the last: X[r][j] = -(sum_{k=j+1}^{r}
    // X[r][k] L[k][j]) / L[j][j], with the columns right of j already inverted
    const int g = tid >> 3, sub = tid & 7;
    for (int j = bs - 1; j >= 0; --j) {
        const double ljj = A[j * bs + j];
        for (int r0 = j + 1; r0 < bs; r0 += FNT / 8) {
            const int r = r0 + g;
            double acc = 0.0;
            if (r < bs)
                for (int k = j + 1 + sub; k <= r; k += 8) acc += A[r * bs + k] * A[k * bs + j];
#pragma unroll
            for (int o = 4; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (r < bs && sub == 0) tmp[r] = -acc / ljj;
        }
        __syncthreads();
        for (int r = j + 1 + tid; r < bs; r += FNT) A[r * bs + j] = tmp[r];
        if (tid == 0) A[j * bs + j] = 1.0 / ljj;
        __syncthreads();
    }
    double* Cg = Ci + i * bb;
    for (int e = tid; e < bs * bs; e += FNT) Cg[e] = (e % bs <= e / bs) ? A[e] : 0.0;
}

// Gm_i = C_i^{-1} Lc_i and Gp_i = C_i^{-1} Lc_{i+s}^T for the blocks eliminated at level s
// (64 x 64 output tiles on the FP64 matrix cores; blockIdx: tile, product, block).
__global__ void __launch_bounds__(NT) k_bcr_offdiag(const double* __restrict__ Ci, const double* __restrict__ Lc,
                                                   double* __restrict__ Gm, double* __restrict__ Gp, int bs, int nblk,
                                                   int s) {
    const int T = (bs + TB - 1) / TB;
    int b = blockIdx.x;
    const int tile = b % (T * T);
    b /= T * T;
    const int job = b % 2, i = s + 2 * s * (b / 2);
    if (i >= nblk) return;
    const long long bb = (long long)bs * bs;
    const int tm = tile / T, tn = tile % T;
    if (job == 0) {
        gemm_tile(tm, tn, 0, 0, bs, bs, bs, 1.0, Ci + i * bb, bs, Lc + i * bb, bs, 0.0, Gm + i * bb, bs);
    } else {
        if (i + s >= nblk) return;
        gemm_tile(tm, tn, 0, 1, bs, bs, bs, 1.0, Ci + i * bb, bs, Lc + (i + s) * bb, bs, 0.0, Gp + i * bb, bs);
    }
}

// Schur complements of level s on the surviving blocks e = 2 s q: job 0 updates D_e, job 1
// forms the coupling of e with e - 2s (the next level's Lc_e).
__global__ void __launch_bounds__(NT) k_bcr_schur(const double* __restrict__ Gm, const double* __restrict__ Gp,
                                                 double* __restrict__ D, double* __restrict__ Lc, int bs, int nblk,
                                                 int s) {
    const int T = (bs + TB - 1) / TB;
    int b = blockIdx.x;
    const int tile = b % (T * T);
    b /= T * T;
    const int job = b % 2, e = 2 * s * (b / 2);
    if (e >= nblk) return;
    const long long bb = (long long)bs * bs;
    const int tm = tile / T, tn = tile % T;
    if (job == 0) {
        if (e >= s)
            gemm_tile(tm, tn, 1, 0, bs, bs, bs, -1.0, Gp + (e - s) * bb, bs, Gp + (e - s) * bb, bs, 1.0, D + e * bb,
                      bs);
        __syncthreads();
        if (e + s < nblk)
            gemm_tile(tm, tn, 1, 0, bs, bs, bs, -1.0, Gm + (e + s) * bb, bs, Gm + (e + s) * bb, bs, 1.0, D + e * bb,
                      bs);
    } else if (e >= s) {
        gemm_tile(tm, tn, 1, 0, bs, bs, bs, -1.0, Gp + (e - s) * bb, bs, Gm + (e - s) * bb, bs, 0.0, Lc + e * bb, bs);
    }
}

// The system left after the levels s < step: blocks p = 0 .. nr-1 standing for e = p step,
// diagonal D_e, couplings A_{e, e-step} = Lc_e (and their transposes above the
// diagonal); M is (nr bs) x (nr bs), row-major.
__global__ void k_bcr_reduced(const double* __restrict__ D, const double* __restrict__ Lc, int bs, int step, int nr,
                              double* __restrict__ M) {
    const long long nn = (long long)nr * bs, e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= nn * nn) return;
    const int R = (int)(e / nn), Cc = (int)(e % nn);
    const int p = R / bs, r = R % bs, q = Cc / bs, cc = Cc % bs;
    const long long bb = (long long)bs * bs;
    double v = 0.0;
    if (p == q)
        v = D[(long long)p * step * bb + (long long)r * bs + cc];
    else if (q == p - 1)
        v = Lc[(long long)p * step * bb + (long long)r * bs + cc];
    else if (q == p + 1)
        v = Lc[(long long)q * step * bb + (long long)cc * bs + r];
    M[e] = v;
}

__global__ void k_d2f(const double* __restrict__ x, float* __restrict__ y, long long n) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e < n) y[e] = (float)x[e];
}

// The solve.  With R_i = C_i^T C_i = D_i^{-1} and the products Gp_i^T C_i, Gm_i^T C_i,
// C_i^T Gm_i, C_i^T Gp_i formed once per factorisation, every level is one set of
// independent block products:
//   forward, e = 0, 2s, 4s, ...:  x_e -= (Gp^T C)_{e-s} x_{e-s} + (Gm^T C)_{e+s} x_{e+s},
//                                 Y_{e+s} = R_{e+s} x_{e+s};
//   block 0:                      x_0 = R_0 x_0;
//   backward, i = s, 3s, ...:     x_i = Y_i - (C^T Gm)_i x_{i-s} - (C^T Gp)_i x_{i+s},
// where each level reads only blocks it does not write.  The rows of every level are
// split over workgroups of 256 threads (16 rows, 16 lanes a row): a launch is one
// memory latency with every product's loads in flight, spread over many CUs.  Loads
// read clamped addresses unconditionally (an entry beyond bs, or a missing neighbour
// block, re-reads a valid one) and the sums mask what is not needed.
constexpr int SNT = 256;
constexpr int SG = 16;
constexpr int SROWS = SNT / SG;
constexpr int BCR_SOLVE_MAX = 144;

template <typename T>
struct BcrView {
    const T *PGP, *PGM, *QGM, *QGP, *R;
};

template <typename T, int KM>
__global__ void __launch_bounds__(SNT) k_bcr_fwd(BcrView<T> F, T* __restrict__ x, T* __restrict__ Y, int bs,
                                                int nblk, int s, int chunks, int stage,
                                                const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int pos = blockIdx.x / chunks, ch = blockIdx.x - pos * chunks;
    const int e = 2 * s * pos;
    const int r = ch * SROWS + (int)threadIdx.x / SG, l = threadIdx.x % SG, rc = min(r, bs - 1);
    const bool h1 = e >= s, h2 = e + s < nblk;
    const int i1 = h1 ? e - s : e, i2 = h2 ? e + s : e;
    const long long bb = (long long)bs * bs;
    const T* a1 = F.PGP + i1 * bb + (long long)rc * bs;
    const T* a2 = F.PGM + i2 * bb + (long long)rc * bs;
    const T* a3 = F.R + i2 * bb + (long long)rc * bs;
    const T* v1 = x + (long long)i1 * bs;
    const T* v2 = x + (long long)i2 * bs;
    T p1[KM], p2[KM], p3[KM], w1[KM], w2[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const int k = min(l + SG * j, bs - 1);
        p1[j] = a1[k];
        p2[j] = a2[k];
        p3[j] = a3[k];
        w1[j] = v1[k];
        w2[j] = v2[k];
    }
    T t = T(0), y = T(0);
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (l + SG * j < bs) {
            t += (h1 ? p1[j] * w1[j] : T(0)) + (h2 ? p2[j] * w2[j] : T(0));
            y += p3[j] * w2[j];
        }
#pragma unroll
    for (int o = SG / 2; o > 0; o >>= 1) {
        t += __shfl_xor(t, o, 64);
        y += __shfl_xor(y, o, 64);
    }
    if (r < bs && l == 0) {
        const T xe = x[(long long)e * bs + r] - t;
        x[(long long)e * bs + r] = xe;
        if (h2) Y[(long long)i2 * bs + r] = y;
        if (stage) Y[(long long)e * bs + r] = xe;  // the reduced system's right-hand side
    }
}

// The truncated reduction's top: x_e = (Minv b)_e on the remaining blocks e = p step,
// b read from Y there (staged by the last forward level, so that no workgroup reads
// what another writes).  Four rows a workgroup, one wavefront a row, each lane KD
// columns with their loads in flight together; b staged in LDS.  The product is FP64
// (Minv is), also for an FP32 solve (T float: b widened, the result rounded once).
constexpr int DNT = 256;
template <typename T, int KD>
__global__ void __launch_bounds__(DNT) k_bcr_dense(const double* __restrict__ Minv, T* __restrict__ x,
                                                  const T* __restrict__ Y, int bs, int step, int nr,
                                                  const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ double b[64 * KD];
    const int nn = nr * bs, tid = threadIdx.x, lane = tid & 63;
    const int row = blockIdx.x * (DNT / 64) + (tid >> 6), rc = min(row, nn - 1);
    const double* a = Minv + (long long)rc * nn;
    double m[KD];
#pragma unroll
    for (int j = 0; j < KD; ++j) m[j] = a[min(lane + 64 * j, nn - 1)];
    for (int k = tid; k < nn; k += DNT) b[k] = double(Y[((long long)(k / bs) * step) * bs + k % bs]);
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < KD; ++j)
        if (lane + 64 * j < nn) acc += m[j] * b[lane + 64 * j];
    acc = wave_sum(acc);
    if (row < nn && lane == 0) x[((long long)(row / bs) * step) * bs + row % bs] = T(acc);
}

// x_0 = R_0 x_0: one workgroup of 1024 threads (64 rows a pass), x_0 staged in LDS
// first (the rows overwrite it)
constexpr int TNT = 1024;
template <typename T, int KM>
__global__ void __launch_bounds__(TNT) k_bcr_top(BcrView<T> F, T* __restrict__ x, int bs,
                                                const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ T b[BCR_SOLVE_MAX];
    for (int r = threadIdx.x; r < bs; r += TNT) b[r] = x[r];
    __syncthreads();
    const int l = threadIdx.x % SG;
    for (int r0 = 0; r0 < bs; r0 += TNT / SG) {
        const int r = r0 + (int)threadIdx.x / SG, rc = min(r, bs - 1);
        const T* a = F.R + (long long)rc * bs;
        T p[KM];
#pragma unroll
        for (int j = 0; j < KM; ++j) p[j] = a[min(l + SG * j, bs - 1)];
        T y = T(0);
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (l + SG * j < bs) y += p[j] * b[l + SG * j];
#pragma unroll
        for (int o = SG / 2; o > 0; o >>= 1) y += __shfl_xor(y, o, 64);
        if (r < bs && l == 0) x[r] = y;
    }
}

template <typename T, int KM>
__global__ void __launch_bounds__(SNT) k_bcr_bwd(BcrView<T> F, T* __restrict__ x, const T* __restrict__ Y, int bs,
                                                int nblk, int s, int chunks, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int pos = blockIdx.x / chunks, ch = blockIdx.x - pos * chunks;
    const int i = s + 2 * s * pos;
    const int r = ch * SROWS + (int)threadIdx.x / SG, l = threadIdx.x % SG, rc = min(r, bs - 1);
    const bool hb = i + s < nblk;
    const int ib = hb ? i + s : i;
    const long long bb = (long long)bs * bs;
    const T* a1 = F.QGM + i * bb + (long long)rc * bs;
    const T* a2 = F.QGP + i * bb + (long long)rc * bs;
    const T* v1 = x + (long long)(i - s) * bs;
    const T* v2 = x + (long long)ib * bs;
    T p1[KM], p2[KM], w1[KM], w2[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const int k = min(l + SG * j, bs - 1);
        p1[j] = a1[k];
        p2[j] = a2[k];
        w1[j] = v1[k];
        w2[j] = v2[k];
    }
    const T yi = Y[(long long)i * bs + rc];
    T t = T(0);
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (l + SG * j < bs) t += p1[j] * w1[j] + (hb ? p2[j] * w2[j] : T(0));
#pragma unroll
    for (int o = SG / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (r < bs && l == 0) x[(long long)i * bs + r] = yi - t;
}

// The FP32 solve: the two-step form (C_i b, then the couplings), each level one
// workgroup of 1024 threads per block; each row of a product handled by 16 lanes, every
// load of a row slot issued before its sums (the level kernels are latency-bound).  The
// product form of the FP64 solve would apply D_i^{-1} as one rounded product and lose
// eps * kappa instead of eps * sqrt(kappa) per block in FP32.
constexpr int SNT2 = 1024;
constexpr int SG2 = 16;
constexpr int SKM = (BCR_SOLVE_MAX + SG2 - 1) / SG2;

// out[r] = sum_k M1[r][k] v1[k] + sum_k M2[r][k] v2[k] (r < bs; M2 may be null), M row-major
// bs x bs, v in LDS; out to LDS or global
template <typename T>
__device__ inline void bcr_gemv(const T* __restrict__ M1, const T* v1, const T* __restrict__ M2, const T* v2, int bs,
                                T* out) {
    constexpr int NG = SNT2 / SG2;
    const int tid = threadIdx.x, g = tid / SG2, l = tid % SG2;
    for (int r0 = 0; r0 < bs; r0 += NG) {
        const int r = r0 + g;
        T acc = T(0);
        if (r < bs) {
            T a[SKM], b[SKM];
#pragma unroll
            for (int j = 0; j < SKM; ++j) {
                const int k = l + SG2 * j;
                a[j] = k < bs ? M1[(long long)r * bs + k] : T(0);
                b[j] = (M2 != nullptr && k < bs) ? M2[(long long)r * bs + k] : T(0);
            }
#pragma unroll
            for (int j = 0; j < SKM; ++j) {
                const int k = l + SG2 * j;
                if (k < bs) acc += a[j] * v1[k] + (M2 != nullptr ? b[j] * v2[k] : T(0));
            }
        }
#pragma unroll
        for (int o = SG2 / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (r < bs && l == 0) out[r] = acc;
    }
}

// Factors the solve reads: C_i^{-1} (C), its transpose (CT), Gm, Gp and their transposes.
template <typename T>
struct BcrView2 {
    const T *C, *CT, *Gm, *Gp, *GmT, *GpT;
};

// Forward pass of level s: every surviving block e = 2 s q forms y of its eliminated
// neighbours (y_k = C_k^{-1} b_k), keeps y_{e+s} in Y, and takes
// b_e -= Gp_{e-s}^T y_{e-s} + Gm_{e+s}^T y_{e+s}.
template <typename T>
__global__ void __launch_bounds__(SNT2) k_bcr2_fwd(BcrView2<T> F, T* __restrict__ x, T* __restrict__ Y, int bs, int nblk,
                                                int s, int stage, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int e = 2 * s * blockIdx.x;
    if (e >= nblk) return;
    __shared__ T bl[BCR_SOLVE_MAX], br[BCR_SOLVE_MAX], yl[BCR_SOLVE_MAX], yr[BCR_SOLVE_MAX], t[BCR_SOLVE_MAX];
    const int tid = threadIdx.x;
    const long long bb = (long long)bs * bs;
    const bool h1 = e >= s, h2 = e + s < nblk;
    const int i1 = e - s, i2 = e + s;
    for (int r = tid; r < bs; r += SNT2) {
        bl[r] = h1 ? x[(long long)i1 * bs + r] : T(0);
        br[r] = h2 ? x[(long long)i2 * bs + r] : T(0);
        yl[r] = T(0);
        yr[r] = T(0);
    }
    __syncthreads();
    if (h1) bcr_gemv<T>(F.C + i1 * bb, bl, nullptr, nullptr, bs, yl);
    if (h2) bcr_gemv<T>(F.C + i2 * bb, br, nullptr, nullptr, bs, yr);
    __syncthreads();
    if (h2)
        for (int r = tid; r < bs; r += SNT2) Y[(long long)i2 * bs + r] = yr[r];
    bcr_gemv<T>(h1 ? F.GpT + i1 * bb : F.GmT + i2 * bb, h1 ? yl : yr, (h1 && h2) ? F.GmT + i2 * bb : nullptr, yr, bs,
                t);
    __syncthreads();
    for (int r = tid; r < bs; r += SNT2) {
        const T xe = x[(long long)e * bs + r] - t[r];
        x[(long long)e * bs + r] = xe;
        if (stage) Y[(long long)e * bs + r] = xe;  // the truncated top's right-hand side
    }
}

// Block 0 after the last level: x_0 = C_0^{-T} C_0^{-1} b_0.
template <typename T>
__global__ void __launch_bounds__(SNT2) k_bcr2_top(BcrView2<T> F, T* __restrict__ x, int bs,
                                                const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ T b[BCR_SOLVE_MAX], y[BCR_SOLVE_MAX];
    for (int r = threadIdx.x; r < bs; r += SNT2) b[r] = x[r];
    __syncthreads();
    bcr_gemv<T>(F.C, b, nullptr, nullptr, bs, y);
    __syncthreads();
    bcr_gemv<T>(F.CT, y, nullptr, nullptr, bs, x);
}

// Backward pass of level s: x_i = C_i^{-T} (y_i - Gm_i x_{i-s} - Gp_i x_{i+s}) for the
// blocks eliminated at this level (their neighbours are solved at higher levels).
template <typename T>
__global__ void __launch_bounds__(SNT2) k_bcr2_bwd(BcrView2<T> F, T* __restrict__ x, const T* __restrict__ Y, int bs,
                                                int nblk, int s, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int i = s + 2 * s * blockIdx.x;
    if (i >= nblk) return;
    __shared__ T xa[BCR_SOLVE_MAX], xb[BCR_SOLVE_MAX], t[BCR_SOLVE_MAX];
    const int tid = threadIdx.x;
    const long long bb = (long long)bs * bs;
    const bool hb = i + s < nblk;
    for (int r = tid; r < bs; r += SNT2) {
        xa[r] = x[(long long)(i - s) * bs + r];
        xb[r] = hb ? x[(long long)(i + s) * bs + r] : T(0);
    }
    __syncthreads();
    bcr_gemv<T>(F.Gm + i * bb, xa, hb ? F.Gp + i * bb : nullptr, xb, bs, t);
    __syncthreads();
    for (int r = tid; r < bs; r += SNT2) t[r] = Y[(long long)i * bs + r] - t[r];
    __syncthreads();
    bcr_gemv<T>(F.CT + i * bb, t, nullptr, nullptr, bs, x + (long long)i * bs);
}

// The same three kernels with every matrix entry a thread uses loaded into registers
// at entry: row r = tid / SGX of each bs x bs block, columns l + SGX j (l = tid % SGX,
// j < KM; bs <= SNT2 / SGX and bs <= SGX KM), so one memory latency per launch instead
// of one per product.  Waves whose rows all lie beyond bs skip the loads and sums
// (a wave-uniform test); the others read clamped addresses unconditionally (an entry
// beyond bs, or a missing neighbour block, re-reads a valid one) and the sums mask
// what is not needed, so nothing waits on a load before all are in flight.
template <typename T, int SGX, int KM>
struct BcrRows {
    T a[KM];
    __device__ __attribute__((always_inline)) void load(const T* __restrict__ M, int bs) {
        const int r = min((int)threadIdx.x / SGX, bs - 1), l = threadIdx.x % SGX;
#pragma unroll
        for (int j = 0; j < KM; ++j) a[j] = M[(long long)r * bs + min(l + SGX * j, bs - 1)];
    }
};

// this wave holds at least one row of a bs x bs block
template <int SGX>
__device__ inline bool bcr_wave_live(int bs) {
    return (int)(threadIdx.x & ~63u) / SGX < bs;
}

// out[r] = sum_k A[r][k] v1[k] (+ B[r][k] v2[k] when `two`), from the preloaded rows
template <typename T, int SGX, int KM>
__device__ __attribute__((always_inline)) inline void bcr_gemv_rows(const BcrRows<T, SGX, KM>& A, const T* v1,
                                                                    const BcrRows<T, SGX, KM>& B, bool two,
                                                                    const T* v2, int bs, T* out) {
    const int r = threadIdx.x / SGX, l = threadIdx.x % SGX;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const int k = l + SGX * j;
        if (r < bs && k < bs) acc += A.a[j] * v1[k] + (two ? B.a[j] * v2[k] : T(0));
    }
#pragma unroll
    for (int o = SGX / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (r < bs && l == 0) out[r] = acc;
}

template <typename T, int SGX, int KM>
__global__ void __launch_bounds__(SNT2) k_bcr2_fwd_r(BcrView2<T> F, T* __restrict__ x, T* __restrict__ Y, int bs,
                                                  int nblk, int s, int stage, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int e = 2 * s * blockIdx.x;
    if (e >= nblk) return;
    __shared__ T bl[BCR_SOLVE_MAX], br[BCR_SOLVE_MAX], yl[BCR_SOLVE_MAX], yr[BCR_SOLVE_MAX], t[BCR_SOLVE_MAX];
    const int tid = threadIdx.x;
    const long long bb = (long long)bs * bs;
    const bool h1 = e >= s, h2 = e + s < nblk;
    const int i1 = h1 ? e - s : e, i2 = h2 ? e + s : e;  // clamped: a missing neighbour reads block e
    const bool live = bcr_wave_live<SGX>(bs);
    BcrRows<T, SGX, KM> c1, c2, g1, g2;
    if (live) {
        c1.load(F.C + i1 * bb, bs);
        c2.load(F.C + i2 * bb, bs);
        g1.load(h1 ? F.GpT + i1 * bb : F.GmT + i2 * bb, bs);
        g2.load(F.GmT + i2 * bb, bs);
    }
    for (int r = tid; r < bs; r += SNT2) {
        bl[r] = h1 ? x[(long long)i1 * bs + r] : T(0);
        br[r] = h2 ? x[(long long)i2 * bs + r] : T(0);
    }
    __syncthreads();
    if (live) {
        bcr_gemv_rows<T, SGX, KM>(c1, bl, c1, false, bl, bs, yl);
        bcr_gemv_rows<T, SGX, KM>(c2, br, c2, false, br, bs, yr);
    }
    __syncthreads();
    if (h2)
        for (int r = tid; r < bs; r += SNT2) Y[(long long)i2 * bs + r] = yr[r];
    if (live) bcr_gemv_rows<T, SGX, KM>(g1, h1 ? yl : yr, g2, h1 && h2, yr, bs, t);
    __syncthreads();
    for (int r = tid; r < bs; r += SNT2) {
        const T xe = x[(long long)e * bs + r] - t[r];
        x[(long long)e * bs + r] = xe;
        if (stage) Y[(long long)e * bs + r] = xe;  // the truncated top's right-hand side
    }
}

template <typename T, int SGX, int KM>
__global__ void __launch_bounds__(SNT2) k_bcr2_top_r(BcrView2<T> F, T* __restrict__ x, int bs,
                                                  const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    __shared__ T b[BCR_SOLVE_MAX], y[BCR_SOLVE_MAX];
    const bool live = bcr_wave_live<SGX>(bs);
    BcrRows<T, SGX, KM> c, ct;
    if (live) {
        c.load(F.C, bs);
        ct.load(F.CT, bs);
    }
    for (int r = threadIdx.x; r < bs; r += SNT2) b[r] = x[r];
    __syncthreads();
    if (live) bcr_gemv_rows<T, SGX, KM>(c, b, c, false, b, bs, y);
    __syncthreads();
    if (live) bcr_gemv_rows<T, SGX, KM>(ct, y, ct, false, y, bs, x);
}

template <typename T, int SGX, int KM>
__global__ void __launch_bounds__(SNT2) k_bcr2_bwd_r(BcrView2<T> F, T* __restrict__ x, const T* __restrict__ Y,
                                                  int bs, int nblk, int s, const double* __restrict__ sc) {
    if (sc != nullptr && sc[SC_DONE] != 0.0) return;
    const int i = s + 2 * s * blockIdx.x;
    if (i >= nblk) return;
    __shared__ T xa[BCR_SOLVE_MAX], xb[BCR_SOLVE_MAX], t[BCR_SOLVE_MAX];
    const int tid = threadIdx.x;
    const long long bb = (long long)bs * bs;
    const bool hb = i + s < nblk;
    const bool live = bcr_wave_live<SGX>(bs);
    BcrRows<T, SGX, KM> gm, gp, ct;
    if (live) {
        gm.load(F.Gm + i * bb, bs);
        gp.load(F.Gp + i * bb, bs);  // unused without the upper neighbour
        ct.load(F.CT + i * bb, bs);
    }
    for (int r = tid; r < bs; r += SNT2) {
        xa[r] = x[(long long)(i - s) * bs + r];
        xb[r] = hb ? x[(long long)(i + s) * bs + r] : T(0);
    }
    __syncthreads();
    if (live) bcr_gemv_rows<T, SGX, KM>(gm, xa, gp, hb, xb, bs, t);
    __syncthreads();
    for (int r = tid; r < bs; r += SNT2) t[r] = Y[(long long)i * bs + r] - t[r];
    __syncthreads();
    if (live) bcr_gemv_rows<T, SGX, KM>(ct, t, ct, false, t, bs, x + (long long)i * bs);
}

// B_i = A_i^T for every block
__global__ void k_bcr_transpose(const double* __restrict__ A, double* __restrict__ B, int bs, long long tot) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const long long bb = (long long)bs * bs, base = e / bb * bb;
    const int r = (int)((e % bb) / bs), c = (int)(e % bs);
    B[base + (long long)c * bs + r] = A[e];
}

}  // namespace

namespace tgms {

void gemm(tgms_ctx* c, int transA, int transB, int M, int N, int K, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB);
    hipLaunchKernelGGL(k_gemm, grid, dim3(NT), 0, c->stream, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C,
                       ldc, 0);
    LAUNCH_OK();
}

// The launches of the inverse on c->stream, with no host synchronisation:
//   1. blocked Cholesky (lower), failures flagged in w.fail;
//   2. X = L^{-1} by recursive halving: [L11 0; L21 L22]^{-1} = [X11 0; -X22 L21 X11, X22],
//      whose products are large square GEMMs; the 64 x 64 leaves are the inverses from 1;
//   3. A = tril(X) + triu(X^T, 1).
static void dense_inverse_enqueue(tgms_ctx* c, double* A, int n, const DenseInvWork& w) {
    const int nblk = (n + TB - 1) / TB;
    double* Dinv = w.Dinv;
    // the recursion multiplies whole square blocks of X, whose parts above the
    // diagonal it never writes: they must be zero
    zero(c, w.X, sizeof(double) * (size_t)n * n);
    // Two-level right-looking blocking: outer panels of OB (512) columns are factorised by
    // inner steps of 64 (diagonal block, panel below it, update of the rest of the outer
    // panel only); the trailing matrix is then updated once per outer panel, with
    // k = OB (OB / 64 times fewer passes over it than 64-wide updates).
    constexpr int OB = 8 * TB;
    for (int c0 = 0; c0 < n; c0 += OB) {
        const int c1 = std::min(n, c0 + OB);
        for (int k0 = c0; k0 < c1; k0 += TB) {
            const int kb0 = k0 / TB, kb = std::min(TB, n - k0), k1 = k0 + kb;
            hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(NT), 0, c->stream, A, n, k0, kb,
                               Dinv + (size_t)kb0 * TB * TB, w.fail);
            LAUNCH_OK();
            const int m = n - k1;
            if (m <= 0) break;
            // panel: A[k1:, k0:k1] = A[k1:, k0:k1] * Dinv^T (each output row tile reads only its own row tile)
            {
                dim3 grid(1, (m + TB - 1) / TB);
                hipLaunchKernelGGL(k_gemm, grid, dim3(NT), 0, c->stream, 0, 1, m, kb, kb, 1.0,
                                   (const double*)(A + (size_t)k1 * n + k0), n,
                                   (const double*)(Dinv + (size_t)kb0 * TB * TB), TB, 0.0, A + (size_t)k1 * n + k0,
                                   n, 0);
                LAUNCH_OK();
            }
            // the rest of the outer panel: A[k1:, k1:c1] -= P P[k1:c1]^T (above the diagonal
            // of the panel's square part the result is never read)
            if (c1 > k1) {
                dim3 grid((c1 - k1 + TB - 1) / TB, (m + TB - 1) / TB);
                hipLaunchKernelGGL(k_gemm, grid, dim3(NT), 0, c->stream, 0, 1, m, c1 - k1, kb, -1.0,
                                   (const double*)(A + (size_t)k1 * n + k0), n,
                                   (const double*)(A + (size_t)k1 * n + k0), n, 1.0, A + (size_t)k1 * n + k1, n, 0);
                LAUNCH_OK();
            }
        }
        // trailing: A[c1:, c1:] -= Q Q^T with Q = A[c1:, c0:c1] (lower tiles only)
        const int mt = n - c1;
        if (mt > 0) {
            const int nt = (mt + TB - 1) / TB;
            hipLaunchKernelGGL(k_gemm_lower, dim3(nt * (nt + 1) / 2), dim3(NT), 0, c->stream, 0, 1, mt, mt, c1 - c0,
                               -1.0, (const double*)(A + (size_t)c1 * n + c0), n,
                               (const double*)(A + (size_t)c1 * n + c0), n, 1.0, A + (size_t)c1 * n + c1, n);
            LAUNCH_OK();
        }
    }
    // X = L^{-1} by recursive halving, [L11 0; L21 L22]^{-1} = [X11 0; -X22 L21 X11, X22]:
    // the 64 x 64 leaves are the diagonal-block inverses of the factorisation; the
    // internal nodes are grouped by height (children first) and each group is two
    // batched launches of square MFMA GEMMs
    hipLaunchKernelGGL(k_copy_diag_blocks, dim3(nblk), dim3(256), 0, c->stream, (const double*)Dinv, w.X, n);
    LAUNCH_OK();
    struct Node {
        int o, n1, n2, height;
    };
    std::vector<Node> nodes;
    std::function<int(int, int)> build = [&](int o, int len) -> int {
        if (len <= TB) return 0;
        const int n1 = ((len / TB + 1) / 2) * TB, n2 = len - n1;
        const int h = 1 + std::max(build(o, n1), build(o + n1, n2));
        nodes.push_back(Node{o, n1, n2, h});
        return h;
    };
    const int hmax = build(0, n);
    for (int h = 1; h <= hmax; ++h) {
        InvLevel lv{};
        long long toff = 0;
        int mx1 = 0, mx2 = 0;
        auto flush = [&]() {
            if (lv.count == 0) return;
            const dim3 grid((mx1 + TB - 1) / TB, (mx2 + TB - 1) / TB, lv.count);
            for (int step = 0; step < 2; ++step) {
                hipLaunchKernelGGL(k_inv_level, grid, dim3(NT), 0, c->stream, lv, step, (const double*)A, w.X, w.Tm,
                                   n);
                LAUNCH_OK();
            }
            lv.count = 0;
            toff = 0;
            mx1 = mx2 = 0;
        };
        for (const Node& nd : nodes) {
            if (nd.height != h) continue;
            if (lv.count == LEVEL_MAX) flush();
            lv.o[lv.count] = nd.o;
            lv.n1[lv.count] = nd.n1;
            lv.n2[lv.count] = nd.n2;
            lv.toff[lv.count] = toff;
            toff += (long long)nd.n1 * nd.n2;
            mx1 = std::max(mx1, nd.n1);
            mx2 = std::max(mx2, nd.n2);
            ++lv.count;
        }
        flush();
    }
    hipLaunchKernelGGL(k_pack_inverse, dim3(nb((long long)n * n)), dim3(256), 0, c->stream, (const double*)w.X, A, n);
    LAUNCH_OK();
}

static void dense_inverse_sizes(int n, size_t& dinv, size_t& x, size_t& tm) {
    const int nblk = (n + TB - 1) / TB;
    dinv = (size_t)nblk * TB * TB;
    x = (size_t)n * n;
    tm = (size_t)n * (n / 2 + TB);
}

void gemm_batched(tgms_ctx* c, int transA, int transB, int M, int N, int K, double alpha, const double* A, int lda,
                  Strided sa, const double* B, int ldb, Strided sb, double beta, double* C, int ldc, Strided sc,
                  long long batch, bool lower_only) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    const BStride a{sa.outer, sa.inner, sa.nin}, b{sb.outer, sb.inner, sb.nin}, cc{sc.outer, sc.inner, sc.nin};
    for (long long z0 = 0; z0 < batch; z0 += 65535) {
        const unsigned nz = (unsigned)std::min<long long>(65535, batch - z0);
        dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB, nz);
        hipLaunchKernelGGL(k_gemm_b, grid, dim3(NT), 0, c->stream, transA, transB, M, N, K, alpha, A, lda, a, B, ldb,
                           b, beta, C, ldc, cc, lower_only ? 1 : 0, z0);
        LAUNCH_OK();
    }
}

// In place: each of the batch matrices A_z (n x n, row-major, consecutive, symmetric
// positive definite) -> its explicit inverse.  Per chunk of matrices: blocked Cholesky
// (64-wide panels, the diagonal blocks and their inverses by potrf_diag), X = L^{-1} by
// the recursive halving of the single-matrix inverse, then A = X^T X (lower tiles,
// mirrored).  The workspace of a chunk comes from the device cache.
void dense_spd_inverse_batched(tgms_ctx* c, double* A, int n, long long batch) {
    if (n <= 0 || batch <= 0) return;
    size_t nd, nx, nt;
    dense_inverse_sizes(n, nd, nx, nt);
    const size_t per = sizeof(double) * (nd + nx + nt);
    const long long chunk =
        std::max<long long>(1, std::min<long long>(std::min<long long>(batch, 65535), (4ll << 30) / (long long)per));
    size_t got[3] = {0, 0, 0}, gotf = 0;
    double* Dinv = (double*)dev_alloc(sizeof(double) * nd * chunk, &got[0]);
    double* X = (double*)dev_alloc(sizeof(double) * nx * chunk, &got[1]);
    double* Tm = (double*)dev_alloc(sizeof(double) * nt * chunk, &got[2]);
    int* fail = (int*)dev_alloc(sizeof(int) * 64, &gotf);
    struct Free {
        void* p[4];
        size_t b[4];
        hipStream_t st;
        ~Free() {
            (void)hipStreamSynchronize(st);
            for (int k = 0; k < 4; ++k) dev_free(p[k], b[k]);
        }
    } fr{{Dinv, X, Tm, fail}, {got[0], got[1], got[2], gotf}, c->stream};
    zero(c, fail, sizeof(int) * 64);
    const long long sM = (long long)n * n;
    const int nblk = (n + TB - 1) / TB;
    // the halving tree of the inverse (the same for every matrix)
    struct Node {
        int o, n1, n2, height;
    };
    std::vector<Node> nodes;
    std::function<int(int, int)> build = [&](int o, int len) -> int {
        if (len <= TB) return 0;
        const int n1 = ((len / TB + 1) / 2) * TB, n2 = len - n1;
        const int h = 1 + std::max(build(o, n1), build(o + n1, n2));
        nodes.push_back(Node{o, n1, n2, h});
        return h;
    };
    const int hmax = build(0, n);
    for (long long b0 = 0; b0 < batch; b0 += chunk) {
        const long long nbch = std::min(chunk, batch - b0);
        double* Ab = A + b0 * sM;
        const Strided one{sM, 0, 1};
        zero(c, X, sizeof(double) * nx * nbch);
        // Cholesky, 64 columns at a time
        for (int k0 = 0; k0 < n; k0 += TB) {
            const int kb0 = k0 / TB, kb = std::min(TB, n - k0), k1 = k0 + kb;
            hipLaunchKernelGGL(k_potrf_diag_b, dim3(1, 1, (unsigned)nbch), dim3(NT), 0, c->stream, Ab, sM, n, k0, kb,
                               Dinv + (size_t)kb0 * TB * TB, (long long)nd, fail);
            LAUNCH_OK();
            const int m = n - k1;
            if (m <= 0) break;
            // panel A[k1:, k0:k1] *= Dinv^T, then the trailing lower part -= P P^T
            gemm_batched(c, 0, 1, m, kb, kb, 1.0, Ab + (size_t)k1 * n + k0, n, one,
                         Dinv + (size_t)kb0 * TB * TB, TB, Strided{(long long)nd, 0, 1}, 0.0,
                         Ab + (size_t)k1 * n + k0, n, one, nbch);
            gemm_batched(c, 0, 1, m, m, kb, -1.0, Ab + (size_t)k1 * n + k0, n, one, Ab + (size_t)k1 * n + k0, n, one,
                         1.0, Ab + (size_t)k1 * n + k1, n, one, nbch, true);
        }
        hipLaunchKernelGGL(k_copy_diag_blocks_b, dim3(nblk, 1, (unsigned)nbch), dim3(256), 0, c->stream,
                           (const double*)Dinv, (long long)nd, X, sM, n);
        LAUNCH_OK();
        for (int h = 1; h <= hmax; ++h) {
            InvLevel lv{};
            long long toff = 0;
            int mx1 = 0, mx2 = 0;
            for (const Node& nd_ : nodes) {
                if (nd_.height != h) continue;
                if (lv.count == LEVEL_MAX) throw TgmsError{TGMS_E_UNSUPPORTED, "batched inverse: matrix too large"};
                lv.o[lv.count] = nd_.o;
                lv.n1[lv.count] = nd_.n1;
                lv.n2[lv.count] = nd_.n2;
                lv.toff[lv.count] = toff;
                toff += (long long)nd_.n1 * nd_.n2;
                mx1 = std::max(mx1, nd_.n1);
                mx2 = std::max(mx2, nd_.n2);
                ++lv.count;
            }
            if (lv.count == 0) continue;
            // matrices per launch so that count * matrices fits the grid's z range
            const long long per_launch = std::max<long long>(1, 65535 / lv.count);
            for (long long z0 = 0; z0 < nbch; z0 += per_launch) {
                const long long nz = std::min(per_launch, nbch - z0);
                const dim3 grid((mx1 + TB - 1) / TB, (mx2 + TB - 1) / TB, (unsigned)(nz * lv.count));
                for (int step = 0; step < 2; ++step) {
                    hipLaunchKernelGGL(k_inv_level_b, grid, dim3(NT), 0, c->stream, lv, step,
                                       (const double*)(Ab + z0 * sM), X + z0 * sM, Tm + z0 * (long long)nt, n,
                                       (long long)nt);
                    LAUNCH_OK();
                }
            }
        }
        // A = X^T X (lower tiles), mirrored
        gemm_batched(c, 1, 0, n, n, n, 1.0, X, n, one, X, n, one, 0.0, Ab, n, one, nbch, true);
        hipLaunchKernelGGL(k_mirror_lower_b, dim3(nb(sM * nbch)), dim3(256), 0, c->stream, Ab, n, nbch);
        LAUNCH_OK();
    }
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (h) throw TgmsError{TGMS_E_INVAL, "a local Schur complement is not positive definite"};
}


// In place: A (n x n, row-major, symmetric positive definite) -> B = tril(L^{-1}) + triu(L^{-T}, 1);
// full (optional, n x n): the explicit inverse L^{-T} L^{-1}, exactly symmetric.
void dense_spd_inverse(tgms_ctx* c, double* A, int n, double* full) {
    if (n <= 0) return;
    size_t nd, nx, nt;
    dense_inverse_sizes(n, nd, nx, nt);
    DenseInvWork w;
    w.Dinv = c->alloc<double>(nd);
    w.fail = c->alloc<int>(1);
    w.X = c->alloc<double>(nx);
    w.Tm = c->alloc<double>(nt);
    dense_inverse_enqueue(c, A, n, w);
    if (full) {
        // X = L^{-1} (zero above the diagonal): full = X^T X, its lower triangle mirrored
        gemm(c, 1, 0, n, n, n, 1.0, w.X, n, w.X, n, 0.0, full, n);
        hipLaunchKernelGGL(k_mirror_lower, dim3(nb((long long)n * n)), dim3(256), 0, c->stream, full, n);
        LAUNCH_OK();
    }
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, w.fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    // release the temporaries (they are the last allocations)
    for (int k = 0; k < 4; ++k) {
        dev_free(c->owned.back().p, c->owned.back().bytes);
        c->owned.pop_back();
    }
    if (h) throw TgmsError{TGMS_E_INVAL, "coarse operator is not positive definite"};
}

// The same, queued on c->stream without waiting: the workspace is allocated here
// (released by dense_spd_inverse_end, or by the destructor if that is not reached).
void dense_spd_inverse_begin(tgms_ctx* c, double* A, int n, DenseInvAsync& h) {
    if (n <= 0) return;
    size_t nd, nx, nt;
    dense_inverse_sizes(n, nd, nx, nt);
    h.w.Dinv = (double*)dev_alloc(sizeof(double) * nd, &h.w.bytes[0]);
    h.w.fail = (int*)dev_alloc(sizeof(int) * 64, &h.w.bytes[1]);
    h.w.X = (double*)dev_alloc(sizeof(double) * nx, &h.w.bytes[2]);
    h.w.Tm = (double*)dev_alloc(sizeof(double) * nt, &h.w.bytes[3]);
    h.stream = c->stream;
    zero(c, h.w.fail, sizeof(int) * 64);
    dense_inverse_enqueue(c, A, n, h.w);
}

// Waits for the queued inverse, releases its workspace and reports a failed factorisation.
void dense_spd_inverse_end(DenseInvAsync& h) {
    if (!h.w.fail) return;
    int f = 0;
    HIP_OK(hipStreamSynchronize(h.stream));
    HIP_OK(hipMemcpy(&f, h.w.fail, sizeof(int), hipMemcpyDeviceToHost));
    h.release();
    if (f) throw TgmsError{TGMS_E_INVAL, "coarse operator is not positive definite"};
}

DenseInvAsync::~DenseInvAsync() {
    if (w.fail && stream) (void)hipStreamSynchronize(stream);
    release();
}

void DenseInvAsync::release() {
    void* ps[4] = {(void*)w.Dinv, (void*)w.fail, (void*)w.X, (void*)w.Tm};
    for (int k = 0; k < 4; ++k)
        if (ps[k]) dev_free(ps[k], w.bytes[k]);
    w = DenseInvWork{};
}

// y = A^{-1} x with A^{-1} held as B = tril(X) + triu(X^T, 1); tmp has n entries.
template <typename T>
void symv(tgms_ctx* c, const T* B, int n, const T* x, T* y, const double* sc) {
    if (n <= 0) return;
    T* tmp;
    if constexpr (sizeof(T) == 8)
        tmp = (T*)c->cvec2;
    else
        tmp = (T*)c->cvec2_32;
    hipLaunchKernelGGL((k_trimv<T>), dim3((n + 3) / 4), dim3(256), 0, c->stream, B, n, x, tmp, 0, sc);
    LAUNCH_OK();
    hipLaunchKernelGGL((k_trimv<T>), dim3((n + 3) / 4), dim3(256), 0, c->stream, B, n, (const T*)tmp, y, 1, sc);
    LAUNCH_OK();
}
template void symv<double>(tgms_ctx*, const double*, int, const double*, double*, const double*);
template void symv<float>(tgms_ctx*, const float*, int, const float*, float*, const double*);

// y = A^{-1} c with c the accumulation (CSR ptr/ent) of the block restrictions cy;
// false when n is too large for the fused first product (then nothing is launched)
template <typename T>
bool symv_acc(tgms_ctx* c, const T* B, int n, const int* ptr, const int* ent, const T* cy, T* y, const double* sc) {
    if (n <= 0 || n > ACC_MAX) return false;
    T* tmp;
    if constexpr (sizeof(T) == 8)
        tmp = (T*)c->cvec2;
    else
        tmp = (T*)c->cvec2_32;
    hipLaunchKernelGGL((k_trimv_acc<T>), dim3((n + 3) / 4), dim3(256), 0, c->stream, B, n, ptr, ent, cy, tmp, sc);
    LAUNCH_OK();
    hipLaunchKernelGGL((k_trimv<T>), dim3((n + 3) / 4), dim3(256), 0, c->stream, B, n, (const T*)tmp, y, 1, sc);
    LAUNCH_OK();
    return true;
}
template bool symv_acc<double>(tgms_ctx*, const double*, int, const int*, const int*, const double*, double*,
                               const double*);

// y = F c with F the explicit inverse and c accumulated from cy (one launch)
bool symv_full_acc(tgms_ctx* c, const double* F, int n, const int* ptr, const int* ent, const double* cy, double* y,
                   const double* sc) {
    if (n <= 0 || n > ACC_MAX || F == nullptr) return false;
    hipLaunchKernelGGL((k_symv_acc<double>), dim3((n + 3) / 4), dim3(256), 0, c->stream, F, n, ptr, ent, cy, y, sc);
    LAUNCH_OK();
    return true;
}
int symv_acc_max() { return ACC_MAX; }
template bool symv_acc<float>(tgms_ctx*, const float*, int, const int*, const int*, const float*, float*,
                              const double*);

// ---- block cyclic reduction (see the kernels above) ----
int bcr_max_block(const tgms_ctx* c) {
    // the factor kernel keeps a block in LDS; the solve kernels hold rows in registers
    int bs = BCR_SOLVE_MAX;
    while (bs > 0 && (long long)bs * bs * 8 + 8 * BCR_MAX > c->lds_max) --bs;
    return bs;
}

void bcr_factor(tgms_ctx* c, const double* A, int n, int bs, Bcr& F, bool fp32, bool truncate) {
    if (bs < 1 || bs > bcr_max_block(c)) throw TgmsError{TGMS_E_UNSUPPORTED, "coarse bandwidth too large"};
    const int nblk = (n + bs - 1) / bs;
    const long long bb = (long long)bs * bs, tot = nblk * bb;
    if (!F.D || F.n != n || F.bs != bs) {
        F.D = c->alloc<double>(tot);
        F.Lc = c->alloc<double>(tot);
        F.C = c->alloc<double>(tot);
        F.Gm = c->alloc<double>(tot);
        F.Gp = c->alloc<double>(tot);
        F.PGP = c->alloc<double>(tot);
        F.PGM = c->alloc<double>(tot);
        F.QGM = c->alloc<double>(tot);
        F.QGP = c->alloc<double>(tot);
        F.R = c->alloc<double>(tot);
        F.Y = c->alloc<double>((size_t)nblk * bs);
        F.x = c->alloc<double>((size_t)nblk * bs);
        F.fail = c->alloc<int>(1);
        F.Minv = nullptr;
        if (fp32) {
            F.CT = c->alloc<double>(tot);
            F.GmT = c->alloc<double>(tot);
            F.GpT = c->alloc<double>(tot);
            F.C32 = c->alloc<float>(tot);
            F.Gm32 = c->alloc<float>(tot);
            F.Gp32 = c->alloc<float>(tot);
            F.CT32 = c->alloc<float>(tot);
            F.GmT32 = c->alloc<float>(tot);
            F.GpT32 = c->alloc<float>(tot);
            F.Y32 = c->alloc<float>((size_t)nblk * bs);
            F.x32 = c->alloc<float>((size_t)nblk * bs);
        }
    }
    F.n = n;
    F.bs = bs;
    F.nb = nblk;
    zero(c, F.fail, sizeof(int) * 2);
    zero(c, F.Gp, sizeof(double) * tot);  // blocks without a right neighbour keep zeros
    hipLaunchKernelGGL(k_bcr_extract, dim3(nb(tot)), dim3(256), 0, c->stream, A, n, bs, nblk, F.D, F.Lc);
    LAUNCH_OK();
    const size_t lds = sizeof(double) * (size_t)bb;
    HIP_OK(hipFuncSetAttribute((const void*)k_bcr_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int T = (bs + TB - 1) / TB;
    // truncation: the smallest step (a power of two, at least 2) whose remaining system
    // fits the explicit-inverse apply, if that skips at least one level
    int step = 0;
    if (truncate) {
        int full = 1;
        while (full < nblk) full *= 2;
        for (int st = 2; st < full; st *= 2)
            if ((long long)((nblk + st - 1) / st) * bs <= symv_acc_max()) {
                step = st;
                break;
            }
    }
    F.step = step;
    F.nr = step ? (nblk + step - 1) / step : 0;
    for (int s = 1; s < nblk && (step == 0 || s < step); s *= 2) {
        const int ne = (nblk - s - 1) / (2 * s) + 1, na = (nblk - 1) / (2 * s) + 1;
        hipLaunchKernelGGL(k_bcr_factor, dim3(ne), dim3(FNT), lds, c->stream, (const double*)F.D, F.C, bs, nblk, s, 0,
                           F.fail);
        LAUNCH_OK();
        hipLaunchKernelGGL(k_bcr_offdiag, dim3(ne * 2 * T * T), dim3(NT), 0, c->stream, (const double*)F.C,
                           (const double*)F.Lc, F.Gm, F.Gp, bs, nblk, s);
        LAUNCH_OK();
        hipLaunchKernelGGL(k_bcr_schur, dim3(na * 2 * T * T), dim3(NT), 0, c->stream, (const double*)F.Gm,
                           (const double*)F.Gp, F.D, F.Lc, bs, nblk, s);
        LAUNCH_OK();
    }
    if (step) {
        // the remaining blocks 0, step, 2 step, ...: their system, inverted explicitly
        const long long nn = (long long)F.nr * bs;
        if (!F.Minv) F.Minv = c->alloc<double>(nn * nn);
        double* M = c->alloc<double>(nn * nn);
        hipLaunchKernelGGL(k_bcr_reduced, dim3(nb(nn * nn)), dim3(256), 0, c->stream, (const double*)F.D,
                           (const double*)F.Lc, bs, step, F.nr, M);
        LAUNCH_OK();
        dense_spd_inverse(c, M, (int)nn, F.Minv);  // synchronises: M is free again
        dev_free(c->owned.back().p, c->owned.back().bytes);
        c->owned.pop_back();
    } else {
        hipLaunchKernelGGL(k_bcr_factor, dim3(1), dim3(FNT), lds, c->stream, (const double*)F.D, F.C, bs, nblk, 1, 1,
                           F.fail);
        LAUNCH_OK();
    }
    // the products the solve applies (MFMA, batched over the blocks; rows of Gp and
    // columns of Gm without a neighbour are zero)
    const Strided one{bb, 0, 1};
    gemm_batched(c, 1, 0, bs, bs, bs, 1.0, F.Gp, bs, one, F.C, bs, one, 0.0, F.PGP, bs, one, nblk);
    gemm_batched(c, 1, 0, bs, bs, bs, 1.0, F.Gm, bs, one, F.C, bs, one, 0.0, F.PGM, bs, one, nblk);
    gemm_batched(c, 1, 0, bs, bs, bs, 1.0, F.C, bs, one, F.Gm, bs, one, 0.0, F.QGM, bs, one, nblk);
    gemm_batched(c, 1, 0, bs, bs, bs, 1.0, F.C, bs, one, F.Gp, bs, one, 0.0, F.QGP, bs, one, nblk);
    gemm_batched(c, 1, 0, bs, bs, bs, 1.0, F.C, bs, one, F.C, bs, one, 0.0, F.R, bs, one, nblk);
    if (fp32) {
        hipLaunchKernelGGL(k_bcr_transpose, dim3(nb(tot)), dim3(256), 0, c->stream, (const double*)F.C, F.CT, bs, tot);
        hipLaunchKernelGGL(k_bcr_transpose, dim3(nb(tot)), dim3(256), 0, c->stream, (const double*)F.Gm, F.GmT, bs,
                           tot);
        hipLaunchKernelGGL(k_bcr_transpose, dim3(nb(tot)), dim3(256), 0, c->stream, (const double*)F.Gp, F.GpT, bs,
                           tot);
        LAUNCH_OK();
        const double* src[6] = {F.C, F.Gm, F.Gp, F.CT, F.GmT, F.GpT};
        float* dst[6] = {F.C32, F.Gm32, F.Gp32, F.CT32, F.GmT32, F.GpT32};
        for (int k = 0; k < 6; ++k)
            hipLaunchKernelGGL(k_d2f, dim3(nb(tot)), dim3(256), 0, c->stream, src[k], dst[k], tot);
        LAUNCH_OK();
    }
}

bool bcr_failed(tgms_ctx* c, const Bcr& F) {
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, F.fail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return h != 0;
}

// the truncated top: x on the remaining blocks = Minv (their staged right-hand side)
template <typename T>
void bcr_dense_top(tgms_ctx* c, const Bcr& F, T* x, const T* Y, const double* sc) {
    const int nn = F.nr * F.bs;
    const dim3 grid((unsigned)((nn + DNT / 64 - 1) / (DNT / 64)));
    if (nn <= 64 * 4)
        hipLaunchKernelGGL((k_bcr_dense<T, 4>), grid, dim3(DNT), 0, c->stream, F.Minv, x, Y, F.bs, F.step, F.nr, sc);
    else if (nn <= 64 * 8)
        hipLaunchKernelGGL((k_bcr_dense<T, 8>), grid, dim3(DNT), 0, c->stream, F.Minv, x, Y, F.bs, F.step, F.nr, sc);
    else if (nn <= 64 * 16)
        hipLaunchKernelGGL((k_bcr_dense<T, 16>), grid, dim3(DNT), 0, c->stream, F.Minv, x, Y, F.bs, F.step, F.nr, sc);
    else
        throw TgmsError{TGMS_E_UNSUPPORTED, "reduced coarse system too large"};
    LAUNCH_OK();
}

template <typename T, int KM>
void bcr_solve_k(tgms_ctx* c, const Bcr& F, const BcrView<T>& V, T* x, T* Y, int bs, int nblk, const double* sc) {
    const int chunks = (bs + SROWS - 1) / SROWS;
    int top = 1;
    while (top < nblk) top *= 2;
    const int step = F.step;
    for (int s = 1; s < nblk && (step == 0 || s < step); s *= 2) {
        const int na = (nblk - 1) / (2 * s) + 1;
        hipLaunchKernelGGL((k_bcr_fwd<T, KM>), dim3(na * chunks), dim3(SNT), 0, c->stream, V, x, Y, bs, nblk, s,
                           chunks, step != 0 && 2 * s == step ? 1 : 0, sc);
        LAUNCH_OK();
    }
    if (step) {
        bcr_dense_top<T>(c, F, x, Y, sc);
        top = step;
    } else {
        hipLaunchKernelGGL((k_bcr_top<T, KM>), dim3(1), dim3(TNT), 0, c->stream, V, x, bs, sc);
        LAUNCH_OK();
    }
    for (int s = top / 2; s >= 1; s /= 2) {
        if (s >= nblk) continue;
        const int ne = (nblk - s - 1) / (2 * s) + 1;
        hipLaunchKernelGGL((k_bcr_bwd<T, KM>), dim3(ne * chunks), dim3(SNT), 0, c->stream, V, x, (const T*)Y, bs,
                           nblk, s, chunks, sc);
        LAUNCH_OK();
    }
}

template <int SGX, int KM>
void bcr_solve2_r(tgms_ctx* c, const Bcr& F, const BcrView2<float>& V, float* x, float* Y, int bs, int nblk, int top,
                  const double* sc) {
    const int step = F.step;
    for (int s = 1; s < nblk && (step == 0 || s < step); s *= 2) {
        hipLaunchKernelGGL((k_bcr2_fwd_r<float, SGX, KM>), dim3((nblk - 1) / (2 * s) + 1), dim3(SNT2), 0, c->stream,
                           V, x, Y, bs, nblk, s, step != 0 && 2 * s == step ? 1 : 0, sc);
        LAUNCH_OK();
    }
    if (step) {
        bcr_dense_top<float>(c, F, x, Y, sc);
        top = step;
    } else {
        hipLaunchKernelGGL((k_bcr2_top_r<float, SGX, KM>), dim3(1), dim3(SNT2), 0, c->stream, V, x, bs, sc);
        LAUNCH_OK();
    }
    for (int s = top / 2; s >= 1; s /= 2) {
        if (s >= nblk) continue;
        hipLaunchKernelGGL((k_bcr2_bwd_r<float, SGX, KM>), dim3((nblk - s - 1) / (2 * s) + 1), dim3(SNT2), 0,
                           c->stream, V, x, (const float*)Y, bs, nblk, s, sc);
        LAUNCH_OK();
    }
}

// FP32: the two-step form (see k_bcr2_fwd)
void bcr_solve2(tgms_ctx* c, const Bcr& F, float* x, const double* sc) {
    const BcrView2<float> V{F.C32, F.CT32, F.Gm32, F.Gp32, F.GmT32, F.GpT32};
    float* Y = F.Y32;
    const int nblk = F.nb, bs = F.bs;
    int top = 1;
    while (top < nblk) top *= 2;
    // blocks of up to 64 rows (16 lanes a row) or 72 and 128 rows (8 lanes a row): the
    // register-prefetched kernels
    if (bs <= 64) {
        bcr_solve2_r<16, 4>(c, F, V, x, Y, bs, nblk, top, sc);
        return;
    }
    if (bs <= 72) {
        bcr_solve2_r<8, 9>(c, F, V, x, Y, bs, nblk, top, sc);
        return;
    }
    if (bs <= 128) {
        bcr_solve2_r<8, 16>(c, F, V, x, Y, bs, nblk, top, sc);
        return;
    }
    const int step = F.step;
    for (int s = 1; s < nblk && (step == 0 || s < step); s *= 2) {
        hipLaunchKernelGGL((k_bcr2_fwd<float>), dim3((nblk - 1) / (2 * s) + 1), dim3(SNT2), 0, c->stream, V, x, Y, bs,
                           nblk, s, step != 0 && 2 * s == step ? 1 : 0, sc);
        LAUNCH_OK();
    }
    if (step) {
        bcr_dense_top<float>(c, F, x, Y, sc);
        top = step;
    } else {
        hipLaunchKernelGGL((k_bcr2_top<float>), dim3(1), dim3(SNT2), 0, c->stream, V, x, bs, sc);
        LAUNCH_OK();
    }
    for (int s = top / 2; s >= 1; s /= 2) {
        if (s >= nblk) continue;
        hipLaunchKernelGGL((k_bcr2_bwd<float>), dim3((nblk - s - 1) / (2 * s) + 1), dim3(SNT2), 0, c->stream, V, x,
                           (const float*)Y, bs, nblk, s, sc);
        LAUNCH_OK();
    }
}

template <typename T>
void bcr_solve(tgms_ctx* c, const Bcr& F, T* x, const double* sc) {
    const int nblk = F.nb, bs = F.bs;
    if (bs > BCR_SOLVE_MAX) throw TgmsError{TGMS_E_UNSUPPORTED, "coarse block too wide for the solve"};
    if constexpr (sizeof(T) == 4) {
        bcr_solve2(c, F, x, sc);
    } else {
        const BcrView<T> V{F.PGP, F.PGM, F.QGM, F.QGP, F.R};
        T* Y = F.Y;
        // column slots per lane: 16 lanes a row
        if (bs <= 4 * SG)
            bcr_solve_k<T, 4>(c, F, V, x, Y, bs, nblk, sc);
        else if (bs <= 5 * SG)
            bcr_solve_k<T, 5>(c, F, V, x, Y, bs, nblk, sc);
        else if (bs <= 8 * SG)
            bcr_solve_k<T, 8>(c, F, V, x, Y, bs, nblk, sc);
        else
            bcr_solve_k<T, 9>(c, F, V, x, Y, bs, nblk, sc);
    }
}
template void bcr_solve<double>(tgms_ctx*, const Bcr&, double*, const double*);
template void bcr_solve<float>(tgms_ctx*, const Bcr&, float*, const double*);

}  // namespace tgms
