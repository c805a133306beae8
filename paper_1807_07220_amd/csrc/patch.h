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
// Stored, per patch, in this order (each block padded to a multiple of four words,
// so that every block starts on a 16-byte boundary):
//   P_j  (j = 0..mh-1): the inverse pivot block (T_j^{-1}, M_k^{-1} or U_j^{-1}),
//                       symmetric, lower triangle packed by columns;
//   B_l  (l = 0..mh-2): the coupling block, tridiagonal, as three rows of m words:
//                       n_l[s] = K~(v, v + north), e_l[s] = K~(v, v + north-east),
//                       w_l[s] = K~(v, v + north-west) for the vertex v = (s, l)
//                       (zero where the neighbour is not a patch vertex);
//   S    (m*mh entries): the equilibration scale.
// With u_j = P_j w_j a solve is two forward chains that run concurrently,
//   w_{t+1} = b_{t+1} - B_t u_t from the top, w_{r-1} = b_{r-1} - B_{r-1}^T u_r from
//   the bottom, meeting at w_k = b_k - B_{k-1} u_{k-1} - B_k^T u_{k+1}, x_k = P_k w_k,
// and two backward chains, x_l = u_l - P_l B_l^T x_{l+1} (l < k) and
// x_{l+1} = u_{l+1} - P_{l+1} B_l x_l (l >= k): about mh dependent steps of one
// dense symmetric product and one tridiagonal product each, instead of 2 mh for a
// one-sided block factorisation; the dense links G_j, H_j of the elimination are
// never stored (they are B_j P_j and B_j^T P_{j+1}).
#pragma once

__host__ __device__ inline int tw_tri(int m) { return m * (m + 1) / 2; }
__host__ __device__ inline int tw_trip(int m) { return (tw_tri(m) + 3) & ~3; }  // padded pivot block
__host__ __device__ inline int tw_b3(int m) { return (3 * m + 3) & ~3; }        // padded coupling block
__host__ __device__ inline int tw_offP(int c, int m) { return c * m - c * (c - 1) / 2; }
__host__ __device__ inline long long tw_links(int m, int mh) { return (long long)mh * tw_trip(m); }
__host__ __device__ inline long long tw_scale(int m, int mh) {
    return tw_links(m, mh) + (long long)(mh - 1) * tw_b3(m);
}
__host__ __device__ inline long long tw_size(int m, int mh) { return tw_scale(m, mh) + (long long)m * mh; }
