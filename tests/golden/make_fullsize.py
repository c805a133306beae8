"""Write the oracle's results on the full-size 2D workloads (run by hand; minutes per workload).

For each workload: the adaptive basis counts and Dim, the eigenvalues of a seeded
sample of coarse faces, the PCG iteration count, relative residual and Lanczos
Cond at rtol 1e-8, and -- from a solve at rtol 1e-12, where the iterate equals
the discrete solution to well below 1e-10 -- the velocity on a seeded sample of
faces, the pressure on a seeded sample of cells and the full vectors' 2-norms.
It also records how far that iterate lies from the direct solve of
the full saddle system (the attainable FP64 accuracy of the problem).  Only the
oracle and the seeded input generators are called.  Output:
tests/golden/fullsize_<workload>.npz (numpy, no pickled objects).

    python tests/golden/make_fullsize.py [workload ...]
"""
from __future__ import annotations

import os
import sys
import time
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Grid2D, OracleSolver  # noqa: E402
from oracle.solver import exact_solve  # noqa: E402
from workloads import configs  # noqa: E402

WORKLOADS = ["darcy2d_256_b16", "darcy2d_1024_b16", "darcy2d_1024_b8"]
N_FACE_SAMPLES = 65536
N_CELL_SAMPLES = 32768
N_EIG_FACES = 256


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded sample of k distinct indices in [0, n) (all of them when k >= n), sorted."""
    if k >= n:
        return np.arange(n)
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def make(name: str) -> str:
    w = configs.get(name)
    kappa, F = w.make_inputs()
    g = Grid2D(w.nx, w.ny, w.bx, w.by)
    t0 = time.time()
    o = OracleSolver(g, kappa, w.eig_tol)
    t_setup = time.time() - t0
    print(f"{name}: setup {t_setup:.1f} s, Dim {o.dim}", flush=True)
    r8 = o.solve(F.ravel(), rtol=1e-8, maxit=2000)
    print(f"{name}: rtol 1e-8 {r8['iters']} iterations, Cond {r8['cond']:.4g}", flush=True)
    r12 = o.solve(F.ravel(), rtol=1e-12, maxit=4000)
    print(f"{name}: rtol 1e-12 {r12['iters']} iterations", flush=True)
    # attainable FP64 accuracy of the problem: the distance of the converged iterate to the
    # direct solve of the full saddle system (a few minutes at 1024^2)
    floor_u = floor_p = np.float64(np.nan)
    if g.nc <= 1024 * 1024:
        ue, pe = exact_solve(g, kappa, F.ravel())
        floor_u = np.linalg.norm(r12["u"] - ue) / np.linalg.norm(ue)
        floor_p = np.linalg.norm(r12["p"] - pe) / np.linalg.norm(pe)
        print(f"{name}: rtol 1e-12 iterate vs direct solve: u {floor_u:.2e}, p {floor_p:.2e}", flush=True)
    fidx = sample_indices(g.nf, N_FACE_SAMPLES, 1)
    cidx = sample_indices(g.nc, N_CELL_SAMPLES, 2)
    eidx = sample_indices(len(o.faces), N_EIG_FACES, 3)
    jmax = max(w.bx, w.by)
    eigs = np.zeros((eidx.size, jmax))
    for k, f in enumerate(eidx):
        eigs[k, : o.eigs[f].size] = o.eigs[f]
    out = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(
        out, counts=o.counts.astype(np.int16), dim=np.int64(o.dim), eig_faces=eidx, eigs=eigs,
        iters_1e8=np.int64(r8["iters"]), relres_1e8=np.float64(r8["relres"]), cond_1e8=np.float64(r8["cond"]),
        iters_1e12=np.int64(r12["iters"]), face_idx=fidx, u_1e12=r12["u"][fidx], cell_idx=cidx,
        p_1e12=r12["p"][cidx], u_norm=np.float64(np.linalg.norm(r12["u"])),
        p_norm=np.float64(np.linalg.norm(r12["p"])), floor_u=np.float64(floor_u), floor_p=np.float64(floor_p),
        seconds=np.float64(time.time() - t0))
    print(f"{name}: wrote {out} after {time.time() - t0:.0f} s", flush=True)
    return out


if __name__ == "__main__":
    warnings.filterwarnings("ignore")
    for name in (sys.argv[1:] or WORKLOADS):
        make(name)
