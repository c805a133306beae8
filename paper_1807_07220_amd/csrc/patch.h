// Storage of the smoother's local solvers on the oversampled blocks K_i^+.
//
// The local matrix K = C^T A C on an m x mh rectangle of interior vertices is
// block tridiagonal by vertex rows (row j couples only to rows j-1 and j+1).
// It is diagonally equilibrated (K~ = S K S, S = diag(K)^{-1/2}) and factorised
// by a two-sided ("twisted") block elimination: rows 0..k-1 are eliminated
// downwards, rows mh-1..k+1 upwards, and the two sweeps meet at the middle row
// k = mh/2.  With A_j the diagonal blocks and B_j = K~_{j+1,j}:
//
//   top:    T_0 = A_0,      G_j = B_j T_j^{-1},          T_{j+1} = A_{j+1} - G_j B_j^T
//   bottom: U_{mh-1} = A_{mh-1}, H_j = B_j^T U_{j+1}^{-1}, U_j = A_j - H_j B_j
//   middle: M_k = A_k - G_{k-1} B_{k-1}^T - H_k B_k
//
// Stored, per patch, in this order:
//   P_j  (j = 0..mh-1): the inverse pivot block (T_j^{-1}, M_k^{-1} or U_j^{-1}),
//                       symmetric, lower triangle packed by columns;
//   link l (l = 0..mh-2): G_l for l < k, H_l for l >= k, dense m x m row-major;
//   S    (m*mh entries): the equilibration scale.
// A solve is then two chains of matrix-vector products that run concurrently
// (w_{l+1} = b_{l+1} - G_l w_l from the top, w_l = b_l - H_l w_{l+1} from the
// bottom), one batch of independent products u_j = P_j w_j, and two backward
// chains (x_l = u_l - G_l^T x_{l+1}, x_{l+1} = u_{l+1} - H_l^T x_l): about mh
// dependent steps instead of 2 mh for a one-sided block factorisation.
#pragma once

__host__ __device__ inline int tw_tri(int m) { return m * (m + 1) / 2; }
__host__ __device__ inline int tw_offP(int c, int m) { return c * m - c * (c - 1) / 2; }
__host__ __device__ inline long long tw_links(int m, int mh) { return (long long)mh * tw_tri(m); }
__host__ __device__ inline long long tw_scale(int m, int mh) {
    return tw_links(m, mh) + (long long)(mh - 1) * m * m;
}
__host__ __device__ inline long long tw_size(int m, int mh) { return tw_scale(m, mh) + (long long)m * mh; }
