"""The paper's algorithm in three dimensions, step by step, in plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The steps and readings are those of ``oracle.solver`` (section 5's Steps 1-4;
snapshots and the local spectral problem of section 4; the smoother on K_i^+ =
K_i + overlap, eq. smooth; the coarse correction, eq. coarsepre; PCG with the
residual kept in ker B and stopped on the preconditioned residual), on the
unit cube (the paper's models 2 and 3).  A coarse face E_i now carries
J_i = (fine faces across it) snapshots, one per fine face, and its basis
functions live on the two blocks sharing it.

The Euclidean projection onto ker B and the least-squares pressure need the
cell Laplacian B_I B_I^T, which on a uniform grid is the constant-coefficient
Neumann Laplacian sum_a |e_a|^2 (1D Neumann Laplacian along axis a): it is
diagonalised by the orthonormal DCT-II (eigenvalues 2 - 2 cos(pi m / n) per
axis), so both are solved with scipy's DCT (a library primitive) instead of a
sparse factorisation.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp

from .grid3d import Grid3D, div_matrix, mass_matrix
from .local import BorderedSaddle, RefinedLU
from .solver import OracleSolver, bordered_dense_or_sparse


def face_geometry(g: Grid3D, face):
    """Blocks K1 (low side), K2 (high side) and the fine faces of coarse face (axis a, I).

    The fine faces of E are ordered with the lower tangential axis fastest.  Returns
    (K1, K2, e (full indices), e_area, left cells, right cells).
    """
    a, I = face
    K1 = tuple(I[d] - (d == a) for d in range(3))
    K2 = tuple(I)
    t = [d for d in range(3) if d != a]
    lo = [I[d] * g.b[d] for d in range(3)]
    c1, c2 = np.meshgrid(np.arange(g.b[t[0]]), np.arange(g.b[t[1]]), indexing="xy")
    c1, c2 = c1.ravel(), c2.ravel()
    idx = [None, None, None]
    idx[a] = np.full(c1.size, lo[a])
    idx[t[0]] = lo[t[0]] + c1
    idx[t[1]] = lo[t[1]] + c2
    e = g.face(a, *idx)
    left = list(idx)
    left[a] = idx[a] - 1
    area = g.cell_vol / g.h[a]
    return K1, K2, e, np.full(e.size, area), g.cell(*left), g.cell(*idx)


def snapshots(g: Grid3D, A, B, block_solver, face):
    """Snapshot matrix Psi (faces of omega x J) for one coarse face (eq. snapshot_eqn): on
    each block K of omega, v . n = delta_l on E, zero flux on the rest of dK and div v =
    the outward flux / |K| (alpha_K, + in K1, - in K2)."""
    K1, K2, e, e_area, _, _ = face_geometry(g, face)
    parts = []
    for K, sign in ((K1, 1.0), (K2, -1.0)):
        bs = block_solver(K)
        vol_K = bs.cells.size * g.cell_vol
        alpha = sign * e_area / vol_K
        rhs_f = -A[bs.faces][:, e].toarray()
        rhs_c = alpha[None, :] * g.cell_vol - B[bs.cells][:, e].toarray()
        v, _ = bs.solve(rhs_f, rhs_c)
        parts.append((bs.faces, v))
    faces = np.concatenate([parts[0][0], parts[1][0], e])
    Psi = np.vstack([parts[0][1], parts[1][1], np.eye(e.size)])
    return faces, Psi


def pencil(g: Grid3D, A, B, kinv_cells, face, faces, Psi, s_scale=1.0):
    """Diagonal a-form and s-form on span(Psi) (eq. spectral_eqn), prefactor 1/s_scale
    (None: the printed 1/H with H = |K|^(1/3))."""
    K1, K2, e, e_area, left, right = face_geometry(g, face)
    Dg = e_area * 0.5 * (kinv_cells[left] + kinv_cells[right])
    cells = np.concatenate([g.cells_in(*g.block_box(K1)), g.cells_in(*g.block_box(K2))])
    M = A[faces][:, faces]
    divs = B[cells][:, faces] @ Psi
    H = (g.bx * g.h[0] * g.by * g.h[1] * g.bz * g.h[2]) ** (1.0 / 3.0) if s_scale is None else s_scale
    S = (Psi.T @ (M @ Psi) + divs.T @ (divs / g.cell_vol)) / H
    return Dg, 0.5 * (S + S.T)


def coarse_rt0_interpolation(g: Grid3D) -> sp.csr_matrix:
    """Coarse RT0 face functions interpolated on the fine faces: the function of coarse face
    (a, I) is 1 - |x_a - X|/H_a in the normal direction on its two blocks (constant across)."""
    rows, cols, vals = [], [], []
    for col, (a, I) in enumerate(g.coarse_faces()):
        t = [d for d in range(3) if d != a]
        ia = np.arange((I[a] - 1) * g.b[a], (I[a] + 1) * g.b[a] + 1)
        w = 1.0 - np.abs(ia - I[a] * g.b[a]) / g.b[a]
        r1 = np.arange(I[t[0]] * g.b[t[0]], (I[t[0]] + 1) * g.b[t[0]])
        r2 = np.arange(I[t[1]] * g.b[t[1]], (I[t[1]] + 1) * g.b[t[1]])
        A_, T1, T2 = np.meshgrid(ia, r1, r2, indexing="ij")
        W = np.broadcast_to(w[:, None, None], A_.shape)
        idx = [None, None, None]
        idx[a], idx[t[0]], idx[t[1]] = A_.ravel(), T1.ravel(), T2.ravel()
        rows.append(g.face(a, *idx))
        vals.append(W.ravel())
        cols.append(np.full(A_.size, col))
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.nf, len(g.coarse_faces())))
    R.eliminate_zeros()
    return R


class CellLaplacian:
    """Solves (B_I B_I^T) q = b (consistent b, mean-zero q) by the orthonormal DCT-II."""

    def __init__(self, g: Grid3D):
        self.shape = (g.nz, g.ny, g.nx)  # arrays are [k][j][i]
        lam = np.zeros(self.shape)
        for a, n in enumerate(g.n):
            area2 = (g.cell_vol / g.h[a]) ** 2
            l1 = 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)
            sh = [1, 1, 1]
            sh[2 - a] = n
            lam = lam + area2 * l1.reshape(sh)
        lam[0, 0, 0] = 1.0
        self.lam = lam

    def __call__(self, b):
        bh = sfft.dctn(np.asarray(b, dtype=np.float64).reshape(self.shape), type=2, norm="ortho")
        bh /= self.lam
        bh[0, 0, 0] = 0.0
        return sfft.idctn(bh, type=2, norm="ortho").ravel()


class OracleSolver3D(OracleSolver):
    """Setup and solve on the unit cube; the Krylov and two-grid methods are the 2D oracle's."""

    def __init__(self, g: Grid3D, kappa, eig_tol, eta=0.2, overlap=2, s_scale=1.0, basis="gmsfem",
                 m_pre=1, m_post=1, additive=False):
        self.g = g
        self.kappa = np.asarray(kappa, dtype=np.float64).reshape(g.nz, g.ny, g.nx)
        if not np.all(np.isfinite(self.kappa)) or np.any(self.kappa <= 0):
            raise ValueError("permeability must be finite and positive")
        if overlap < 1:
            raise ValueError("overlap must be at least 1 (oversampled smoother domains)")
        self.kinv = (1.0 / self.kappa).ravel()
        self.eig_tol, self.eta, self.overlap = float(eig_tol), float(eta), int(overlap)
        self.m_pre, self.m_post, self.additive = int(m_pre), int(m_post), bool(additive)
        self.A = mass_matrix(g, self.kinv).tocsr()
        self.B = div_matrix(g).tocsr()
        self.mask = g.interior.astype(np.float64)
        self._blocks = {}
        self._lap = CellLaplacian(g)
        self.faces = g.coarse_faces()
        self.omega_faces, self.Psi, self.eigs, self.counts, self.Phi_local = [], [], [], [], []
        if basis == "rt0":
            self.Phi = coarse_rt0_interpolation(g)
            self.counts = np.ones(len(self.faces), dtype=np.int64)
        else:
            for face in self.faces:
                fa, Psi = snapshots(g, self.A, self.B, self.block, face)
                Dg, S = pencil(g, self.A, self.B, self.kinv, face, fa, Psi, s_scale)
                lam, V = sla.eigh(np.diag(Dg), S)
                cnt = max(1, int(np.count_nonzero(lam < self.eig_tol)))
                Vk = np.ones((Psi.shape[1], 1)) if basis == "msfem" else V[:, :cnt]
                if basis == "msfem":
                    cnt = 1
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
        self.RQ = sp.csr_matrix((np.ones(g.nc), (g.block_of_cells(), np.arange(g.nc))),
                                shape=(g.Nx * g.Ny * g.Nz, g.nc))
        AH = (self.Phi.T @ self.A @ self.Phi).toarray()
        BH = (self.RQ @ self.B @ self.Phi).toarray()
        self.coarse_lu, self.nH, self.mH = bordered_dense_or_sparse(AH, BH)
        self.dim = int(self.counts.sum()) + g.Nx * g.Ny * g.Nz + 1
        self.patches = [BorderedSaddle(self.A, self.B, g.faces_in(*g.block_box(I, self.overlap)),
                                       g.cells_in(*g.block_box(I, self.overlap))) for I in g.blocks()]

    def update_mobility(self, lam):
        """The mobility update of section 6.2 with the basis kept, on the cube: A from
        kappa^{-1} / lam, the coarse operator over the same Phi, the blocks and the smoother
        patches factorised again (OracleSolver.update_mobility in three dimensions)."""
        g = self.g
        lam = np.asarray(lam, dtype=np.float64).ravel()
        if lam.size != g.nc or not np.all(np.isfinite(lam)) or np.any(lam <= 0):
            raise ValueError("mobility must be finite and positive on every cell")
        self.A = mass_matrix(g, self.kinv / lam).tocsr()
        AH = (self.Phi.T @ self.A @ self.Phi).toarray()
        BH = (self.RQ @ self.B @ self.Phi).toarray()
        self.coarse_lu, self.nH, self.mH = bordered_dense_or_sparse(AH, BH)
        self._blocks = {}
        self.patches = [BorderedSaddle(self.A, self.B, g.faces_in(*g.block_box(I, self.overlap)),
                                       g.cells_in(*g.block_box(I, self.overlap))) for I in g.blocks()]

    def block(self, I) -> BorderedSaddle:
        """L_K = R_K L R_K^T on coarse block K (faces strictly inside K, cells of K)."""
        I = tuple(I)
        if I not in self._blocks:
            lo, hi = self.g.block_box(I)
            self._blocks[I] = BorderedSaddle(self.A, self.B, self.g.faces_in(lo, hi), self.g.cells_in(lo, hi))
        return self._blocks[I]

    def project(self, r):
        """Euclidean projection of a face vector onto ker B (interior faces)."""
        q = self._lap(self.B @ (self.mask * r))
        return self.mask * (r - self.B.T @ q)

    def preprocess(self, F, g_full=None):
        """Section 3: coarse RT0 solve, then one local correction per block (eq. subproblem)."""
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
        for I in g.blocks():
            bs = self.block(I)
            v, _ = bs.solve(-AvH[bs.faces], res[bs.cells])
            vbar[bs.faces] += v
        return vbar, gb, Fp

    def pressure(self, u_full):
        """p = argmin ||B_I^T p - (A u)_I||_2 with zero mean (physical sign: A v = B^T p)."""
        I = self.g.interior_idx
        a = np.zeros(self.g.nf)
        a[I] = (self.A @ u_full)[I]
        p = self._lap(self.B @ a)
        return p - p.mean()


def exact_solve(g: Grid3D, kappa, F):
    """Direct solve of the full RT0-P0 saddle system (eq. fine_system), no-flow boundary:
    (u on all faces, physical pressure with zero mean)."""
    kinv = 1.0 / np.asarray(kappa, dtype=np.float64).ravel()
    A = mass_matrix(g, kinv).tocsr()
    B = div_matrix(g).tocsr()
    I = g.interior_idx
    AII, BI = A[I][:, I], B[:, I]
    K = sp.bmat([[AII, BI[:-1].T], [BI[:-1], None]], format="csc")
    rhs = np.concatenate([np.zeros(I.size), np.asarray(F, dtype=np.float64).ravel()[:-1]])
    sol = RefinedLU(K).solve(rhs)
    u = np.zeros(g.nf)
    u[I] = sol[: I.size]
    pp = np.concatenate([sol[I.size:], [0.0]])
    pp -= pp.mean()
    return u, -pp
