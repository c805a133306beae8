"""Section 5's controls on the GPU against the oracle (needs an MI355X): smoothing steps
m1 = m2 > 1, the two-level additive Schwarz form, the smoother weight eta, the
oversampling and the eigenvalue tolerance (basis counts and Dim)."""
import numpy as np
import pytest

from workloads import configs, fields

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from gpu_util import dev, host, rel  # noqa: E402


def _kappa(name):
    if name == "cfg32":
        return configs.get("darcy2d_32_b8").make_inputs()[0], 8, 0.5
    return fields.field_channelized(64, 64, 11, contrast=1e6), 8, 2.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", [{"smooth_steps": 2}, {"smooth_steps": 3}, {"additive": True}])
@pytest.mark.parametrize("name", ["cfg32", "chan64"])
def test_cycle_variants_match_oracle(name, variant, precision):
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    kappa, b, tol = _kappa(name)
    n = kappa.shape[0]
    kw = {"m_pre": variant.get("smooth_steps", 1), "m_post": variant.get("smooth_steps", 1),
          "additive": variant.get("additive", False)}
    o = OracleSolver(Grid2D(n, n, b, b), kappa, tol, **kw)
    s = tg.Solver(dev(kappa), b, b, tol, precision=precision, **variant)
    r = np.random.default_rng(9).standard_normal(o.g.nf) * o.mask
    z = host(s.apply_precond("twogrid", dev(r)))
    e = rel(z, o.twogrid(r))
    F = fields.corner_source(n, n).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10, maxit=2000), o.solve(F, rtol=1e-10, maxit=2000)
    du = host(res["u"]) - ro["u"]
    ea = np.sqrt(du @ (o.A @ du)) / np.sqrt(ro["u"] @ (o.A @ ro["u"]))
    print(f"{name} {variant} {precision}: two-grid {e:.2e}, iters {res['iters']} / {ro['iters']}, u (energy) {ea:.2e}")
    assert res["converged"]
    if precision == "fp64":
        assert e < 1e-8 and abs(res["iters"] - ro["iters"]) <= 1 and ea <= 1e-10
    else:
        assert e < 1e-4 and ea <= 1e-8


def test_eta_and_overlap_match_oracle():
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    kappa, b, tol = _kappa("chan64")
    F = fields.corner_source(64, 64).ravel()
    for eta, ov in ((0.1, 2), (0.24, 2), (0.2, 1), (0.2, 3)):
        o = OracleSolver(Grid2D(64, 64, b, b), kappa, tol, eta=eta, overlap=ov)
        s = tg.Solver(dev(kappa), b, b, tol, eta=eta, overlap=ov)
        res, ro = s.solve(dev(F), rtol=1e-10), o.solve(F, rtol=1e-10)
        print(f"eta {eta} overlap {ov}: iters {res['iters']} / {ro['iters']}")
        assert abs(res["iters"] - ro["iters"]) <= 1
        assert np.linalg.norm(host(res["p"]) - ro["p"]) <= 1e-10 * np.linalg.norm(ro["p"])


def test_tolerance_sweep_dim_matches_oracle():
    """The tolerance trades the coarse dimension against the iteration count (section
    4.2): at every tolerance the counts and Dim equal the oracle's and the iterations agree."""
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    kappa, b, _ = _kappa("chan64")
    F = fields.corner_source(64, 64).ravel()
    prev_dim = 0
    for tol in (0.5, 2.0, 8.0, 20.0):
        o = OracleSolver(Grid2D(64, 64, b, b), kappa, tol)
        s = tg.Solver(dev(kappa), b, b, tol)
        near = np.array([np.any(np.abs(e - tol) <= 1e-8 * tol) for e in o.eigs])
        assert np.array_equal(s.counts()[~near], o.counts[~near]) and s.info()["dim"] == o.dim
        res, ro = s.solve(dev(F), rtol=1e-8), o.solve(F, rtol=1e-8)
        print(f"tol {tol}: Dim {o.dim}, iters {res['iters']} / {ro['iters']}, Cond {ro['cond']:.3g}")
        assert abs(res["iters"] - ro["iters"]) <= 1 and o.dim >= prev_dim
        prev_dim = o.dim
