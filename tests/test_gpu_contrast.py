"""Robustness over contrast on the GPU (section 6's protocol; needs an MI355X): a binary
medium, background 1 and channels / inclusions at 10^-6 .. 10^6, on 128 x 128 cells in
16 x 16 blocks at the paper's tolerance 10.  The adaptive space keeps the iteration
count flat (the paper's tables spread by about 2); the MsFEM space (one function per
face, the sum of its snapshots) degrades at high contrast.  Iteration counts at three
contrasts are checked against the oracle."""
import numpy as np
import pytest

from workloads import fields

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]
torch = pytest.importorskip("torch")

from gpu_util import dev  # noqa: E402

N, B, TOL = 128, 16, 10.0
EXPS = (-6, -4, -2, 0, 2, 4, 6)


def test_iterations_flat_over_contrast():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_07220_amd as tg
    from oracle import OracleSolver
    from oracle.discretization import Grid2D
    F = fields.corner_source(N, N)
    its, its_ms = {}, {}
    for e in EXPS:
        kappa = fields.field_binary(N, N, 7, 10.0 ** e)
        s = tg.Solver(dev(kappa), B, B, TOL)
        its[e] = s.solve(dev(F), rtol=1e-8)["iters"]
        s.close()
        if e >= 2:
            s = tg.Solver(dev(kappa), B, B, TOL, coarse_space="msfem")
            its_ms[e] = s.solve(dev(F), rtol=1e-8, maxit=3000)["iters"]
            s.close()
    print(f"GMsFEM iterations over contrast {its}; MsFEM {its_ms}")
    assert max(its.values()) - min(its.values()) <= 4, its
    assert max(its_ms.values()) > max(its.values()) + 4, (its, its_ms)
    g = Grid2D(N, N, B, B)
    for e in (-6, 0, 6):
        kappa = fields.field_binary(N, N, 7, 10.0 ** e)
        ref = OracleSolver(g, kappa, TOL).solve(F.ravel(), rtol=1e-8)["iters"]
        assert abs(its[e] - ref) <= 1, (e, its[e], ref)
    kappa = fields.field_binary(N, N, 7, 1e6)
    ref_ms = OracleSolver(g, kappa, TOL, basis="msfem").solve(F.ravel(), rtol=1e-8, maxit=3000)["iters"]
    assert abs(its_ms[6] - ref_ms) <= 1, (its_ms[6], ref_ms)
