"""The coarse space kept under changing mobility (section 6.2) at the workloads' sizes
(needs an MI355X): the library's update_mobility (basis of the initial permeability kept;
operator, coarse matrix, coarse RT0 system and smoother rebuilt) against a setup whose
coarse space is built anew for lambda * kappa, over a sequence of front positions."""
import numpy as np
import pytest

from workloads import configs, fields

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_util import dev, host  # noqa: E402


@pytest.mark.parametrize("name", ["darcy2d_256_b16", "darcy2d_1024_b16"])
def test_kept_coarse_space_costs_at_most_two_iterations(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_07220_amd as tg
    w = configs.get(name)
    kappa, F = w.make_inputs()
    Fd = dev(F)
    s = tg.Solver(dev(kappa), w.bx, w.by, w.eig_tol)
    try:
        for t in (0.25, 0.5, 0.75, 1.0, 1.25):
            lam = fields.mobility_front(w.nx, w.ny, t)
            s.update_mobility(dev(lam))
            kept = s.solve(Fd, rtol=w.rtol, maxit=2000)
            f = tg.Solver(dev(kappa * lam), w.bx, w.by, w.eig_tol)
            fresh = f.solve(Fd, rtol=w.rtol, maxit=2000)
            dim_fresh = f.info()["dim"]
            f.close()
            print(f"{name} front {t}: kept basis {kept['iters']} iterations, new basis {fresh['iters']} "
                  f"(Dim {s.info()['dim']} kept, {dim_fresh} new)")
            assert kept["converged"] and fresh["converged"]
            assert kept["iters"] <= fresh["iters"] + 2
            # the same discrete solution, to the accuracy of the stopping test
            ea = np.linalg.norm(host(kept["p"]) - host(fresh["p"])) / np.linalg.norm(host(fresh["p"]))
            assert ea <= 1e-5
    finally:
        s.close()
