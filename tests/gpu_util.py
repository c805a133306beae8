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
