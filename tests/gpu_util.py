"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on the same inputs."""
import functools
import warnings

import numpy as np
import torch

warnings.filterwarnings("ignore", category=Warning, module="scipy")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@functools.lru_cache(maxsize=8)
def oracle_for(nx, ny, bx, by, key, tol):
    from oracle import Grid2D, OracleSolver
    kappa = KAPPAS[key]
    return OracleSolver(Grid2D(nx, ny, bx, by), kappa, tol)


KAPPAS = {}


def register(key, kappa):
    KAPPAS[key] = np.asarray(kappa, dtype=np.float64)
    return key


def eig_bound(kappa, bx, by, lam):
    """Relative tolerance for the local eigenvalues lambda of one coarse face.

    The snapshots enter S through the kappa^{-1}-weighted mass Gram; their accuracy in
    that norm is limited by eps times the condition number of the local stream-function
    matrices, about contrast * (block cells per side)^2 (a factor 100 of margin).  The
    pencil's largest eigenvalue mu = 1/lambda_min carries that error, which reaches
    lambda_k as a relative eps * lambda_k / lambda_min on top.
    """
    eps = np.finfo(np.float64).eps
    kappa = np.asarray(kappa)
    contrast = float(kappa.max() / kappa.min())
    base = 100.0 * eps * contrast * max(bx, by) ** 2
    return max(base, 1e-12) + 100.0 * eps * lam / lam.min()


def oracle_face(kappa, bx, by, fid):
    """The oracle's pencil of coarse face fid (x-faces first, then y-faces, each row
    by row): returns (T = D^{-1/2} S D^{-1/2}, D, S)."""
    from oracle.discretization import Grid2D, div_matrix, mass_matrix
    from oracle.local import BorderedSaddle
    from oracle.spectral import block_rect, pencil, snapshots
    ny, nx = kappa.shape
    g = Grid2D(nx, ny, bx, by)
    Nx = nx // bx
    nex = (Nx - 1) * (ny // by)
    if fid < nex:
        face = ("x", fid % (Nx - 1) + 1, fid // (Nx - 1))
    else:
        f = fid - nex
        face = ("y", f % Nx, f // Nx + 1)
    kinv = (1.0 / kappa).ravel()
    A, B = mass_matrix(g, kinv).tocsr(), div_matrix(g).tocsr()

    def block(I, J):
        r = block_rect(g, I, J)
        return BorderedSaddle(A, B, g.faces_in(*r), g.cells_in(*r))
    fa, Psi = snapshots(g, A, B, block, face)
    Dg, S = pencil(g, A, B, kinv, face, fa, Psi)
    d = 1.0 / np.sqrt(Dg)
    return d[:, None] * S * d[None, :], Dg, S
