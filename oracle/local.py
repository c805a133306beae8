"""Direct solution of restricted saddle-point systems R L R^T.

Section 2 defines the local matrices L_i = R_i L R_i^T (coarse block K_i) and
L_i^+ = R_i^+ L R_i^{+T} (oversampled block K_i^+) as restrictions of the
global saddle matrix [A B^T; B 0] to the faces strictly inside the subdomain
and to its cells.  With zero flux on the subdomain boundary the pressure is
determined up to a constant; one Lagrange multiplier enforcing a zero cell
sum removes that null space (the '+1' in the paper's DOF counts of section 6
is this multiplier).  The bordered system is factorised once by SuperLU.

The paper solves every subproblem with a direct solver.  SuperLU's pivoting on
these saddle matrices (mass entries spanning the permeability contrast, zero
pressure block) leaves relative errors up to ~1e-9 at contrast 1e6, so every
solve here takes one step of iterative refinement with the same factors
(x <- x + K^{-1}(b - K x)), which brings it to FP64 round-off.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class RefinedLU:
    """SuperLU factorisation of a sparse matrix K with one refinement step per solve."""

    def __init__(self, K: sp.spmatrix):
        self.K = sp.csr_matrix(K)
        self.lu = spla.splu(sp.csc_matrix(K))
        self.shape = K.shape

    def solve(self, b: np.ndarray) -> np.ndarray:
        b = np.asarray(b, dtype=np.float64)
        x = self.lu.solve(b)
        return x + self.lu.solve(b - self.K @ x)


class BorderedSaddle:
    """Factorised [[A_ff, B_cf^T, 0], [B_cf, 0, 1], [0, 1^T, 0]]."""

    def __init__(self, A: sp.spmatrix, B: sp.spmatrix, faces: np.ndarray, cells: np.ndarray):
        self.faces = np.asarray(faces)
        self.cells = np.asarray(cells)
        Aff = A[self.faces][:, self.faces]
        Bcf = B[self.cells][:, self.faces]
        nfl, ncl = self.faces.size, self.cells.size
        one = sp.csr_matrix(np.ones((ncl, 1)))
        K = sp.bmat([[Aff, Bcf.T, None], [Bcf, None, one], [None, one.T, None]], format="csc")
        self.nfl, self.ncl = nfl, ncl
        self.lu = RefinedLU(K)

    def solve(self, rhs_f: np.ndarray, rhs_c: np.ndarray):
        """Return (velocity on self.faces, pressure multiplier p' on self.cells)."""
        rhs_f = np.asarray(rhs_f, dtype=np.float64)
        rhs_c = np.asarray(rhs_c, dtype=np.float64)
        squeeze = rhs_f.ndim == 1
        if squeeze:
            rhs_f, rhs_c = rhs_f[:, None], rhs_c[:, None]
        m = rhs_f.shape[1]
        rhs = np.vstack([rhs_f, rhs_c, np.zeros((1, m))])
        sol = self.lu.solve(rhs)
        v, p = sol[: self.nfl], sol[self.nfl: self.nfl + self.ncl]
        if squeeze:
            return v[:, 0], p[:, 0]
        return v, p
