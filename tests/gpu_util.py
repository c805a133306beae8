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
