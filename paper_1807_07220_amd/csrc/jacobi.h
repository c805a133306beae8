// Batched dense symmetric eigensolver for the local spectral problems (section 4.2): one
// workgroup of one wavefront per matrix held in LDS.
#pragma once
#include <hip/hip_runtime.h>

// Cyclic Jacobi on the symmetric n x n matrix A (row stride ld, LDS), round-robin
// ordering over the pairs, one wavefront: A becomes diagonal (the eigenvalues), and
// V (the identity on entry) accumulates the rotations (eigenvectors in its columns).
// NM: a power of two >= n (the element loops' stride); pq: LDS room for the pairs of
// one round ([NM / 2][2]), published with their rotations so that the update loops
// do no index arithmetic beyond shifts and masks.
template <int NM>
__device__ bool jacobi_rr(double* A, double* V, int ld, int n, double (*cs)[2], int (*pq)[2], int* rot_flag) {
    static_assert((NM & (NM - 1)) == 0, "NM must be a power of two");
    constexpr int SH = NM == 1 ? 0 : NM == 2 ? 1 : NM == 4 ? 2 : NM == 8 ? 3 : NM == 16 ? 4 : NM == 32 ? 5 : 6;
    const int lane = threadIdx.x;
    const int N = (n + 1) & ~1, half = N / 2;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (lane == 0) *rot_flag = 0;
        __syncthreads();
        for (int rnd = 0; rnd < N - 1; ++rnd) {
            if (lane < half) {
                auto pos = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + rnd) % (N - 1); };
                const int p = pos(lane), qq = pos(N - 1 - lane);
                double c = 1.0, s = 0.0;
                if (p < n && qq < n) {
                    const double apq = A[p * ld + qq], app = A[p * ld + p], aqq = A[qq * ld + qq];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        *rot_flag = 1;
                    }
                }
                cs[lane][0] = c;
                cs[lane][1] = s;
                pq[lane][0] = (p < n && qq < n) ? p : -1;  // -1: no rotation on this pair
                pq[lane][1] = qq;
            }
            __syncthreads();
            for (int e = lane; e < (half << SH); e += 64) {  // rows: A <- P^T A
                const int k = e >> SH, x = e & (NM - 1);
                const int p = pq[k][0], qq = pq[k][1];
                if (x < n && p >= 0) {
                    const double c = cs[k][0], s = cs[k][1];
                    const double tp = A[p * ld + x], tq = A[qq * ld + x];
                    A[p * ld + x] = c * tp - s * tq;
                    A[qq * ld + x] = s * tp + c * tq;
                }
            }
            __syncthreads();
            for (int e = lane; e < (half << SH); e += 64) {  // columns: A <- A P, V <- V P
                const int k = e >> SH, x = e & (NM - 1);
                const int p = pq[k][0], qq = pq[k][1];
                if (x < n && p >= 0) {
                    const double c = cs[k][0], s = cs[k][1];
                    const double tp = A[x * ld + p], tq = A[x * ld + qq];
                    A[x * ld + p] = c * tp - s * tq;
                    A[x * ld + qq] = s * tp + c * tq;
                    const double vp = V[x * ld + p], vq = V[x * ld + qq];
                    V[x * ld + p] = c * vp - s * vq;
                    V[x * ld + qq] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
        if (!*rot_flag) return true;
        __syncthreads();
    }
    return false;  // still rotating after the sweep limit
}
