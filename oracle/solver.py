"""The paper's algorithm, step by step, in plain FP64 (section 5, "the precise algorithm").

Step 1  preprocessing (section 3): coarse RT0 solve, then block corrections,
        giving vbar with B vbar = F.
Step 2  adaptive coarse space (section 4) and the coarse operator
        L_H = R_H L R_H^T on V_ms x Q_H (Q_H = piecewise constants on blocks).
Step 3  PCG on the reduced system (eq. reduced_fine_system) with the two-grid
        preconditioner: pre-smoothing S (eq. smooth), coarse correction P
        (eq. coarsepre), post-smoothing S, the residual recomputed after
        every step.
Step 4  v = vbar + vtilde.

Readings where the paper is silent (each also listed in the design notes):
  * the stopping test compares the l2 norm of the preconditioned residual
    z_k with that of z_0 (the velocity residual itself tends to B^T p, not 0);
  * the smoother solves on the oversampled blocks K_i^+ (L_i^+, not L_i);
  * K_i^+ is K_i enlarged by ``overlap`` fine cells on every side, clipped to D;
  * the pressure is recovered by least squares from A v = B^T p with zero
    mean (the algorithm only returns the velocity);
  * nonzero boundary data g (normal velocity on boundary faces) moves to the
    right-hand side: F' = F - B_bnd g and the reduced right-hand side gains
    -A_{I,bnd} g; the paper itself uses g = 0;
  * the PCG residual is kept in ker B by the Euclidean projection
    r <- r - B^T (B B^T)^+ B r after every update.  The preconditioner
    annihilates range(B^T) and z lies in ker B, so this changes nothing in
    exact arithmetic; without it the residual converges to B^T p (large
    where kappa is small) and the local saddle solves amplify that part
    until r^T z loses all accuracy (PCG stalls at contrast 1e-6).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import Grid2D, div_matrix, mass_matrix
from .local import BorderedSaddle, RefinedLU
from .spectral import block_rect, face_geometry, pencil, select, snapshots


def coarse_rt0_interpolation(g: Grid2D) -> sp.csr_matrix:
    """R_H^T: coarse RT0 face unknowns -> fine face values (full numbering).

    The coarse basis of a coarse face at X is linear in the normal coordinate,
    1 - |x - X|/H on the two adjacent blocks, so its fine RT0 interpolant is
    that value at every fine face position (section 2, V_H subset V_h).
    """
    rows, cols, vals = [], [], []
    for col, (kind, I, J) in enumerate(g.coarse_faces()):
        if kind == "x":
            i = np.arange((I - 1) * g.bx, (I + 1) * g.bx + 1)
            w = 1.0 - np.abs(i - I * g.bx) / g.bx
            for j in range(J * g.by, (J + 1) * g.by):
                rows.append(g.xf(i, j)); vals.append(w); cols.append(np.full(i.size, col))
        else:
            j = np.arange((J - 1) * g.by, (J + 1) * g.by + 1)
            w = 1.0 - np.abs(j - J * g.by) / g.by
            for i in range(I * g.bx, (I + 1) * g.bx):
                rows.append(g.yf(i, j)); vals.append(w); cols.append(np.full(j.size, col))
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.nf, len(g.coarse_faces())))
    R.eliminate_zeros()
    return R


def block_aggregation(g: Grid2D) -> sp.csr_matrix:
    """R_Q: sums fine cells into coarse blocks (Q_H subset Q_h)."""
    blk = g.block_of_cells()
    return sp.csr_matrix((np.ones(g.nc), (blk, np.arange(g.nc))), shape=(g.Nx * g.Ny, g.nc))


def pinned_cell_laplacian(BI):
    """Solver of the singular, consistent system (B_I B_I^T) q = b.

    The null space is the constants; the last cell's value is pinned to zero
    (its equation is implied by the others for a consistent right-hand side),
    which keeps the factorisation sparse.
    """
    L = (BI @ BI.T).tocsc()
    lu = RefinedLU(L[:-1, :-1])

    def solve(b):
        q = np.zeros(L.shape[0])
        q[:-1] = lu.solve(np.asarray(b, dtype=np.float64)[:-1])
        return q
    return solve


def bordered_dense_or_sparse(Ah, Bh):
    """Factorise [[Ah, Bh^T, 0], [Bh, 0, 1], [0, 1^T, 0]] (one mean-zero multiplier)."""
    n, m = Ah.shape[0], Bh.shape[0]
    one = sp.csr_matrix(np.ones((m, 1)))
    K = sp.bmat([[sp.csr_matrix(Ah), sp.csr_matrix(Bh).T, None],
                 [sp.csr_matrix(Bh), None, one], [None, one.T, None]], format="csc")
    return RefinedLU(K), n, m


class OracleSolver:
    """Setup (Steps 1-2 pieces that do not depend on the source) and solve."""

    def __init__(self, g: Grid2D, kappa: np.ndarray, eig_tol: float, eta: float = 0.2,
                 overlap: int = 2, s_scale: float | None = 1.0, basis: str = "gmsfem", force_counts=None,
                 m_pre: int = 1, m_post: int = 1, additive: bool = False):
        """basis: "gmsfem" (section 4, the adaptive space), "msfem" (one function per
        coarse face, the sum of its snapshots, eq. msfem) or "rt0" (the coarse RT0
        space); the last two are the comparators of section 6.  force_counts: the
        number of eigenfunctions kept per coarse face (in the order of
        ``g.coarse_faces()``) instead of #{lambda < tol}, for comparisons where an
        eigenvalue lies at the tolerance.  m_pre, m_post: smoothing steps before and
        after the coarse correction (section 5; 1 and 1 in the paper); additive: the
        two-level additive Schwarz form S r + P r instead of the cycle (section 5 sets the
        two apart by whether the residual is recomputed)."""
        self.m_pre, self.m_post, self.additive = int(m_pre), int(m_post), bool(additive)
        self.g = g
        self.kappa = np.asarray(kappa, dtype=np.float64).reshape(g.ny, g.nx)
        if not np.all(np.isfinite(self.kappa)) or np.any(self.kappa <= 0):
            raise ValueError("permeability must be finite and positive")
        self.kinv = (1.0 / self.kappa).ravel()
        self.eig_tol, self.eta, self.overlap = float(eig_tol), float(eta), int(overlap)
        if self.overlap < 1:
            # without oversampling (K_i^+ = K_i) the smoother misses the fine fluxes
            # across block edges and the two-grid preconditioner is singular on ker B
            raise ValueError("overlap must be at least 1 (oversampled smoother domains)")
        self.A = mass_matrix(g, self.kinv).tocsr()
        self.B = div_matrix(g).tocsr()
        self.mask = g.interior.astype(np.float64)
        self._blocks = {}
        BI = self.B[:, g.interior_idx]
        self._cell_lap = pinned_cell_laplacian(BI)
        self.faces = g.coarse_faces()
        # Step 2: adaptive coarse space (section 4)
        self.omega_faces, self.Psi, self.eigs, self.counts, self.Phi_local = [], [], [], [], []
        if basis not in ("gmsfem", "msfem", "rt0"):
            raise ValueError(basis)
        if basis == "rt0":
            # the coarse RT0 functions themselves (section 2: V_H subset V_h), one per face
            self.Phi = coarse_rt0_interpolation(g)
            self.counts = np.ones(len(self.faces), dtype=np.int64)
        else:
            for k, face in enumerate(self.faces):
                fa, Psi = snapshots(g, self.A, self.B, self.block, face)
                Dg, S = pencil(g, self.A, self.B, self.kinv, face, fa, Psi, s_scale)
                lam, V, cnt = select(Dg, S, self.eig_tol)
                if force_counts is not None:
                    cnt = int(force_counts[k])
                if basis == "msfem":       # sum of all snapshots: unit flux on E (section 4.2, eq. msfem)
                    cnt, Vk = 1, np.ones((Psi.shape[1], 1))
                else:
                    Vk = V[:, :cnt]
                self.omega_faces.append(fa)
                self.Psi.append(Psi)
                self.eigs.append(lam)
                self.counts.append(cnt)
                self.Phi_local.append(Psi @ Vk)
            self.counts = np.asarray(self.counts, dtype=np.int64)
            rows, cols, vals, off = [], [], [], 0
            for fa, Ph in zip(self.omega_faces, self.Phi_local):
                for k in range(Ph.shape[1]):
                    rows.append(fa); cols.append(np.full(fa.size, off + k)); vals.append(Ph[:, k])
                off += Ph.shape[1]
            self.Phi = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                     shape=(g.nf, off))
        self.RQ = block_aggregation(g)
        AH = (self.Phi.T @ self.A @ self.Phi).toarray()
        BH = (self.RQ @ self.B @ self.Phi).toarray()
        self.coarse_lu, self.nH, self.mH = bordered_dense_or_sparse(AH, BH)
        self.dim = int(self.counts.sum()) + g.Nx * g.Ny + 1
        # smoother patches K_i^+
        self.patches = []
        for J in range(g.Ny):
            for I in range(g.Nx):
                r = block_rect(g, I, J, self.overlap)
                self.patches.append(BorderedSaddle(self.A, self.B, g.faces_in(*r), g.cells_in(*r)))

    # ---- mobility update with the coarse space kept (section 6.2) -------------
    def update_mobility(self, lam):
        """Rebuild the operator for total mobility lam (per cell) with the basis kept.

        Section 6.2 keeps the multiscale basis built for the initial permeability
        while the mobility changes between pressure solves.  The flux law becomes
        (lam kappa)^{-1} v = -grad p, so the mass matrix A is rebuilt with
        kappa^{-1}/lam; the coarse operator R_H L R_H^T is formed again over the
        same basis Phi (A_H = Phi^T A Phi, B_H unchanged), the smoother patches and
        the preprocessing blocks are refactorised.  Snapshots, eigenpairs and the
        basis counts stay as they are.
        """
        g = self.g
        lam = np.asarray(lam, dtype=np.float64).ravel()
        if lam.size != g.nc or not np.all(np.isfinite(lam)) or np.any(lam <= 0):
            raise ValueError("mobility must be finite and positive on every cell")
        self.A = mass_matrix(g, self.kinv / lam).tocsr()
        AH = (self.Phi.T @ self.A @ self.Phi).toarray()
        BH = (self.RQ @ self.B @ self.Phi).toarray()
        self.coarse_lu, self.nH, self.mH = bordered_dense_or_sparse(AH, BH)
        self._blocks = {}
        self.patches = []
        for J in range(g.Ny):
            for I in range(g.Nx):
                r = block_rect(g, I, J, self.overlap)
                self.patches.append(BorderedSaddle(self.A, self.B, g.faces_in(*r), g.cells_in(*r)))

    # ---- building blocks ----------------------------------------------
    def block(self, I, J) -> BorderedSaddle:
        """L_K = R_K L R_K^T on coarse block K (faces strictly inside K, cells of K)."""
        key = (I, J)
        if key not in self._blocks:
            r = block_rect(self.g, I, J)
            self._blocks[key] = BorderedSaddle(self.A, self.B, self.g.faces_in(*r), self.g.cells_in(*r))
        return self._blocks[key]

    def apply_A(self, x):
        """A_h x on the faces interior to D (boundary entries stay zero)."""
        return self.mask * (self.A @ x)

    def project(self, r):
        """Euclidean projection of a face vector onto ker B (interior faces)."""
        q = self._cell_lap(self.B @ (self.mask * r))
        return self.mask * (r - self.B.T @ q)

    def smooth(self, r):
        """S r = sum_i eta R_i^{+T} (L_i^+)^{-1} R_i^+ [r; 0] (eq. smooth)."""
        z = np.zeros_like(r)
        for P in self.patches:
            v, _ = P.solve(r[P.faces], np.zeros(P.ncl))
            z[P.faces] += self.eta * v
        return z

    def coarse(self, r):
        """P r = R_H^T L_H^{-1} R_H [r; 0] with V_H = V_ms (eq. coarsepre)."""
        rhs = np.concatenate([self.Phi.T @ r, np.zeros(self.mH + 1)])
        sol = self.coarse_lu.solve(rhs)
        return self.Phi @ sol[: self.nH]

    def twogrid(self, r):
        """Pre-smoothing, coarse correction, post-smoothing, the residual recomputed after
        each step (section 5; one step each in the paper), or the additive form."""
        if self.additive:
            return self.smooth(r) + self.coarse(r)
        z = self.smooth(r)
        for _ in range(self.m_pre - 1):
            z = z + self.smooth(r - self.apply_A(z))
        z = z + self.coarse(r - self.apply_A(z))
        for _ in range(self.m_post):
            z = z + self.smooth(r - self.apply_A(z))
        return z

    # ---- Step 1: preprocessing (section 3) -----------------------------
    def preprocess(self, F, g_full=None):
        g = self.g
        F = np.asarray(F, dtype=np.float64).ravel()
        gb = np.zeros(g.nf) if g_full is None else (1.0 - self.mask) * np.asarray(g_full, dtype=np.float64)
        Fp = F - self.B @ gb
        R = coarse_rt0_interpolation(g)
        AH0 = (R.T @ self.A @ R).toarray()
        BH0 = (self.RQ @ self.B @ R).toarray()
        lu, n, m = bordered_dense_or_sparse(AH0, BH0)
        sol = lu.solve(np.concatenate([np.zeros(n), self.RQ @ Fp, [0.0]]))
        vH = R @ sol[:n]
        vbar = vH.copy()
        AvH = self.A @ vH
        res = Fp - self.B @ vH
        for J in range(g.Ny):
            for I in range(g.Nx):
                bs = self.block(I, J)
                v, _ = bs.solve(-AvH[bs.faces], res[bs.cells])    # eq. subproblem
                vbar[bs.faces] += v
        return vbar, gb, Fp

    # ---- Step 3: PCG ----------------------------------------------------
    def pcg(self, b, rtol, maxit, flexible=False, precond=None, project=True):
        M = self.twogrid if precond is None else precond
        P = self.project if project else (lambda v: v)
        x = np.zeros_like(b)
        r = P(b)
        z = M(r)
        z0 = np.linalg.norm(z)
        hist = [1.0]
        alphas, betas = [], []
        if z0 == 0.0:
            return x, 0, hist, alphas, betas
        p = z.copy()
        rho = r @ z
        it = 0
        while it < maxit:
            q = self.apply_A(p)
            pq = p @ q
            if not pq > 0:
                raise FloatingPointError("PCG breakdown: p^T A p <= 0")
            alpha = rho / pq
            x += alpha * p
            r_old = r.copy() if flexible else None
            r = P(r - alpha * q)
            z = M(r)
            it += 1
            alphas.append(alpha)
            rel = np.linalg.norm(z) / z0
            hist.append(rel)
            if rel <= rtol:
                break
            rho_new = r @ z
            beta = (rho_new - z @ r_old) / rho if flexible else rho_new / rho
            betas.append(beta)
            p = z + beta * p
            rho = rho_new
        return x, it, hist, alphas, betas

    @staticmethod
    def lanczos_cond(alphas, betas):
        """Condition number of the preconditioned operator from the PCG scalars."""
        k = len(alphas)
        if k == 0:
            return 1.0
        T = np.zeros((k, k))
        for i in range(k):
            T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
            if i + 1 < k and i < len(betas):
                T[i, i + 1] = T[i + 1, i] = np.sqrt(abs(betas[i])) / alphas[i]
        ev = np.linalg.eigvalsh(T)
        return float(ev[-1] / ev[0])

    # ---- pressure recovery ----------------------------------------------
    def pressure(self, u_full):
        """p = argmin ||B_I^T p - (A u)_I||_2 with zero mean (physical sign: A v = B^T p)."""
        g = self.g
        BI = self.B[:, g.interior_idx]
        a = (self.A @ u_full)[g.interior_idx]
        p = self._cell_lap(BI @ a)
        return p - p.mean()

    # ---- Steps 1-4 --------------------------------------------------------
    def solve(self, F, g_full=None, rtol=1e-8, maxit=500, flexible=False):
        vbar, gb, _ = self.preprocess(F, g_full)
        b = -self.apply_A(vbar + gb)
        x, it, hist, al, be = self.pcg(b, rtol, maxit, flexible)
        u = vbar + x + gb
        p = self.pressure(u)
        return {"u": u, "p": p, "iters": it, "relres": hist[-1], "hist": hist,
                "cond": self.lanczos_cond(al, be), "vbar": vbar, "dim": self.dim}


def exact_solve(g: Grid2D, kappa, F, g_full=None):
    """Direct solve of the full RT0-P0 saddle system (eq. fine_system) with a mean-zero multiplier.

    Returns (u on all faces, physical pressure p with zero mean).
    """
    kinv = 1.0 / np.asarray(kappa, dtype=np.float64).ravel()
    A = mass_matrix(g, kinv).tocsr()
    B = div_matrix(g).tocsr()
    I = g.interior_idx
    gb = np.zeros(g.nf) if g_full is None else np.asarray(g_full, dtype=np.float64).copy()
    gb[I] = 0.0
    # The pressure is determined up to a constant: the last cell's pressure is pinned
    # to zero and its (redundant, by compatibility) divergence equation dropped; the
    # pressure is then shifted to zero mean.  Same solution as the mean-zero multiplier.
    AII = A[I][:, I]
    BI = B[:, I]
    K = sp.bmat([[AII, BI[:-1].T], [BI[:-1], None]], format="csc")
    rhs_f = -(A @ gb)[I]
    rhs_c = (np.asarray(F, dtype=np.float64).ravel() - B @ gb)[:-1]
    sol = RefinedLU(K).solve(np.concatenate([rhs_f, rhs_c]))
    u = gb.copy()
    u[I] = sol[: I.size]
    pprime = np.concatenate([sol[I.size:], [0.0]])
    pprime -= pprime.mean()
    return u, -pprime
