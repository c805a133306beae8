"""The solver on the unit cube (needs an MI355X) against the 3D oracle (oracle/solver3d.py),
element by element on small seeded grids that span several blocks and patches, including
non-cubic blocks, overlap 1 and 2, and the three coarse spaces.

Bars (the same algorithm on both sides, rounding apart): basis counts equal, eigenvalues
to 1e-9 relative, operator and preconditioner probes to 1e-10 relative (in the 2-norm of
the output), PCG iteration counts within one, velocity and pressure to 1e-10 relative.
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]
torch = pytest.importorskip("torch")

from gpu_util import dev, host  # noqa: E402

CASES = {
    # name: (cells, block, overlap, eigen tolerance, log-permeability scale)
    "cube12_b4_ov2": ((12, 12, 12), (4, 4, 4), 2, 2.0, 2.0),
    "box15x12x9_b5x4x3_ov1": ((15, 12, 9), (5, 4, 3), 1, 2.0, 2.0),
    "box20x20x10_b5_ov2": ((20, 20, 10), (5, 5, 5), 2, 2.0, 3.0),
}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(name, seed=5):
    from oracle.grid3d import Grid3D
    dims, b, ov, tol, scale = CASES[name]
    g = Grid3D(*dims, *b)
    rng = np.random.default_rng(seed)
    kappa = np.exp(scale * rng.standard_normal(g.nc))
    F = np.zeros(g.nc)
    F[0], F[-1] = 1.0, -1.0
    return g, kappa, F, ov, tol


def _pair(name, basis="gmsfem"):
    import paper_1807_07220_amd as tg
    from oracle.solver3d import OracleSolver3D
    g, kappa, F, ov, tol = _inputs(name)
    o = OracleSolver3D(g, kappa, tol, overlap=ov, basis=basis)
    nx, ny, nz = g.n
    s = tg.Solver(dev(kappa.reshape(nz, ny, nx)), g.bx, g.by, tol, bz=g.bz, overlap=ov, coarse_space=basis)
    return g, kappa, F, o, s


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_operator_and_setup(name):
    """A x on the interior faces; basis counts and every eigenvalue of every face."""
    _need_gpu()
    g, kappa, F, o, s = _pair(name)
    try:
        x = np.random.default_rng(1).standard_normal(g.nf)
        y = host(s.apply_A(dev(x)))
        np.testing.assert_allclose(y, o.apply_A(x), rtol=0, atol=1e-12 * np.abs(o.apply_A(x)).max())
        counts = np.array(s.counts())
        np.testing.assert_array_equal(counts, o.counts)
        E = s.eigs()
        for i, lam in enumerate(o.eigs):
            np.testing.assert_allclose(E[i, :lam.size], lam, rtol=1e-9)
        assert s.info()["dim"] == o.dim
    finally:
        s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_preprocess_and_preconditioner(name):
    """vbar of section 3; smoother, coarse correction and two-grid cycle on a random
    residual (boundary entries zero)."""
    _need_gpu()
    g, kappa, F, o, s = _pair(name)
    try:
        vbar, _, _ = o.preprocess(F)
        got = host(s.preprocess(dev(F)))
        assert _rel(got, vbar) <= 1e-10
        r = np.random.default_rng(2).standard_normal(g.nf) * o.mask
        for which, fn in (("smoother", o.smooth), ("coarse", o.coarse), ("twogrid", o.twogrid)):
            z = host(s.apply_precond(which, dev(r)))
            ref = fn(r)
            print(f"{name} {which}: rel {_rel(z, ref):.2e}")
            assert _rel(z, ref) <= 1e-10, which
    finally:
        s.close()


@pytest.mark.parametrize("name,basis", [(n, "gmsfem") for n in CASES] +
                         [("cube12_b4_ov2", "msfem"), ("cube12_b4_ov2", "rt0"), ("box15x12x9_b5x4x3_ov1", "rt0")])
def test_solve(name, basis):
    _need_gpu()
    g, kappa, F, o, s = _pair(name, basis)
    try:
        ref = o.solve(F, rtol=1e-8)
        got = s.solve(dev(F), rtol=1e-8)
        eu, ep = _rel(host(got["u"]), ref["u"]), _rel(host(got["p"]), ref["p"])
        print(f"{name} {basis}: iterations {got['iters']} (oracle {ref['iters']}), u {eu:.2e}, p {ep:.2e}")
        assert got["converged"]
        assert abs(got["iters"] - ref["iters"]) <= 1
        assert eu <= 1e-10 and ep <= 1e-10
        # div u = F: the preprocessing meets it to round-off; each PCG correction is
        # divergence-free to about eps cond(S) of the local Schur complements (applied as
        # explicit inverses; the oracle's refined sparse LU reaches eps), so the bound is
        # relative to the largest sum of |flux| over a cell's faces and allows for the
        # conditioning at these contrasts (permeability ratio up to 1e9)
        uh = host(got["u"])
        scale = (abs(o.B) @ np.abs(uh)).max()
        derr = np.abs(o.B @ uh - F).max()
        print(f"  max |B u - F| {derr:.1e} (flux scale {scale:.2e})")
        assert derr <= 1e-9 * scale
    finally:
        s.close()


def test_update_mobility_keeps_the_basis():
    """Section 6.2 on the cube: the operator of lambda kappa over the initial basis."""
    _need_gpu()
    name = "cube12_b4_ov2"
    g, kappa, F, o, s = _pair(name)
    try:
        lam = np.exp(np.random.default_rng(7).uniform(-1.0, 1.0, g.nc))
        o.update_mobility(lam)
        s.update_mobility(dev(lam))
        ref = o.solve(F, rtol=1e-8)
        got = s.solve(dev(F), rtol=1e-8)
        assert abs(got["iters"] - ref["iters"]) <= 1
        assert _rel(host(got["u"]), ref["u"]) <= 1e-10
        assert np.array_equal(np.array(s.counts()), o.counts)
    finally:
        s.close()


def test_transport_and_impes_on_the_cube():
    """The cube's transport step against the oracle's (velocity from the oracle's direct
    solve), then the IMPES loop with the kept coarse space against the oracle's loop."""
    _need_gpu()
    import paper_1807_07220_amd as tg
    from oracle.solver3d import OracleSolver3D, exact_solve
    from oracle.transport import impes, transport_step
    g, kappa, F, ov, tol = _inputs("box20x20x10_b5_ov2")
    nx, ny, nz = g.n
    u, _ = exact_solve(g, kappa, F)
    s0 = np.zeros(g.nc)
    s_o, it_o = transport_step(g, u, F, s0, 0.002, max_newton=2000)
    s_g, outer, res = tg.transport_step(dev(u), dev(F), dev(s0.reshape(nz, ny, nx)), 0.002)
    err = np.abs(host(s_g).ravel() - s_o).max()
    print(f"cube transport: {outer} tile launches (oracle {it_o} Newton iterations), max diff {err:.2e}")
    assert err <= 2 * (nx + ny + nz) * 1e-12
    o = OracleSolver3D(g, kappa, tol, overlap=ov)
    s_ref, its = impes(o, F, np.zeros(g.nc), steps=4, dt=0.002, pressure_every=2, rtol=1e-10)
    sv = tg.Solver(dev(kappa.reshape(nz, ny, nx)), g.bx, g.by, tol, bz=g.bz, overlap=ov)
    try:
        r = sv.impes(dev(F), dev(np.zeros((nz, ny, nx))), steps=4, dt=0.002, pressure_every=2, rtol=1e-10)
    finally:
        sv.close()
    err = np.abs(host(r["s"]).ravel() - s_ref).max()
    print(f"cube IMPES: PCG {r['pcg_iters']} (oracle {its}), max |s diff| {err:.2e}")
    assert all(abs(a - b) <= 1 for a, b in zip(r["pcg_iters"], its))
    assert err <= 1e-7
