"""Two-phase transport and the IMPES loop on the GPU (section 6.2; needs an MI355X) against
the oracle's transport (oracle/transport.py), on the same seeded permeability, sources and
oracle velocity.

Tolerance of one transport step: both sides stop at max_i |R_i| <= 1e-12 (the oracle by
global Newton, the GPU by tile-wise nonlinear Gauss-Seidel), and the step's solution is
unique.  The Jacobian dR/ds is an M-matrix whose columns are diagonally dominant with
margin >= 1, and along an upwind path each cell passes on at most the share it receives,
so a residual r moves the saturation by at most |r| times the number of cells on the
longest upwind path (<= nx + ny for the flows here): 2 (nx + ny) 1e-12 bounds the
difference.
"""
import numpy as np
import pytest

from workloads import fields

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]
torch = pytest.importorskip("torch")

from gpu_util import dev, host  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flow(nx, ny, seed):
    """Seeded log-normal permeability, quarter-five-spot sources and the oracle's exact velocity."""
    from oracle.discretization import Grid2D
    from oracle.solver import exact_solve
    rng = np.random.default_rng(seed)
    kappa = np.exp(fields.gaussian_field_2d(nx, ny, 0.1, rng))
    F = fields.corner_source(nx, ny)
    g = Grid2D(nx, ny)
    u, _ = exact_solve(g, kappa, F)
    return g, kappa, F, u


@pytest.mark.parametrize("nx,ny,seed", [(48, 48, 1), (100, 70, 2), (17, 33, 3)])
def test_transport_step_matches_oracle(nx, ny, seed):
    """Several steps from s = 0 (long steps: the cell of the injector sees a Courant number
    in the hundreds), then one from a random saturation; the GPU's tile Gauss-Seidel
    against the oracle's global Newton, and the water balance of every GPU step."""
    _need_gpu()
    import paper_1807_07220_amd as tg
    from oracle.transport import fractional_flow, transport_step
    g, kappa, F, u = _flow(nx, ny, seed)
    phi, dt = 0.2, 0.004
    tol = 2 * (nx + ny) * 1e-12
    s_o = np.zeros(g.nc)
    s_g = dev(np.zeros((ny, nx)))
    ud, Fd = dev(u), dev(F)
    for step in range(4):
        s_o_new, it_o = transport_step(g, u, F, s_o, dt, phi, max_newton=2000)
        s_g_new, outer, res = tg.transport_step(ud, Fd, s_g, dt, phi=phi)
        got = host(s_g_new).ravel()
        err = np.abs(got - s_o_new).max()
        print(f"{nx}x{ny} step {step}: {outer} tile launches (oracle: {it_o} Newton iterations), "
              f"max |R| {res:.1e}, max |s_gpu - s_oracle| {err:.2e}")
        assert res <= 1e-12
        assert err <= tol
        assert got.min() >= 0.0 and got.max() <= 1.0
        # water balance: the upwind fluxes cancel in the sum over cells
        f, _ = fractional_flow(got)
        gain = phi * g.cell_area * np.sum(got - host(s_g).ravel())
        assert abs(gain - dt * (np.sum(np.maximum(F, 0)) + np.sum(f * np.minimum(F.ravel(), 0)))) < 1e-11
        s_o, s_g = s_o_new, s_g_new
    assert s_o.max() > 0.5
    s0 = np.random.default_rng(seed + 10).uniform(0.0, 1.0, g.nc)
    s_o_new, _ = transport_step(g, u, F, s0, 0.01, phi, max_newton=2000)
    s_g_new, _, _ = tg.transport_step(ud, Fd, dev(s0.reshape(ny, nx)), 0.01, phi=phi)
    assert np.abs(host(s_g_new).ravel() - s_o_new).max() <= tol


def _residual_bound(a_max, tol=1e-12):
    """The GPU stops at max |R_i| <= tol in its own rounding; the oracle's recomputation of
    R_i = s_i + a_i f_w(s_i) - b_i differs by a few ulps of its largest term (1 + a_i)."""
    return tol + 64 * np.finfo(np.float64).eps * (1.0 + a_max)


def test_transport_step_256():
    """The pressure workload's 256^2 grid (16 x 16 tiles, upwind paths across many tiles):
    from a random saturation element by element against the oracle's Newton; from s = 0
    (the oracle's Newton needs about 80 iterations there) through the defining equations:
    the oracle's residual of the GPU's saturation."""
    _need_gpu()
    import paper_1807_07220_amd as tg
    from oracle.transport import face_fluxes, transport_residual, transport_step
    nx = ny = 256
    g, kappa, F, u = _flow(nx, ny, 7)
    s0 = np.random.default_rng(3).uniform(0.0, 1.0, g.nc)
    s_o, it_o = transport_step(g, u, F, s0, 0.004)
    s_g, outer, res = tg.transport_step(dev(u), dev(F), dev(s0.reshape(ny, nx)), 0.004)
    err = np.abs(host(s_g).ravel() - s_o).max()
    print(f"256^2 random start: {outer} tile launches (oracle: {it_o} Newton iterations), max diff {err:.2e}")
    assert err <= 2 * (nx + ny) * 1e-12
    out, nb = face_fluxes(g, u)
    coef = 0.004 / (0.2 * g.cell_area)
    a_max = coef * (np.maximum(out, 0).sum(1) + np.maximum(-F.ravel(), 0)).max()
    z = np.zeros(g.nc)
    s_g, outer, res = tg.transport_step(dev(u), dev(F), dev(z.reshape(ny, nx)), 0.004)
    r = transport_residual(host(s_g).ravel(), z, out, nb, F.ravel(), coef, 1.0, 5.0)
    print(f"256^2 from s = 0: {outer} tile launches, oracle max |R| {np.abs(r).max():.2e}")
    assert np.abs(r).max() <= _residual_bound(a_max)


def test_transport_step_1024_residual():
    """1024^2 (the size of the large pressure workloads) with a seeded gradient flow whose
    sources match its divergence: three steps from s = 0, each checked through the oracle's
    residual of the defining equations and the saturation bounds."""
    _need_gpu()
    import paper_1807_07220_amd as tg
    from oracle.discretization import Grid2D
    from oracle.transport import face_fluxes, transport_residual
    nx = ny = 1024
    g = Grid2D(nx, ny)
    u, q = fields.gradient_flow(nx, ny, 21)
    out, nb = face_fluxes(g, u)
    dt = 0.01
    coef = dt / (0.2 * g.cell_area)
    a_max = coef * (np.maximum(out, 0).sum(1) + np.maximum(-q.ravel(), 0)).max()
    s = np.zeros(g.nc)
    ud, qd = dev(u), dev(q)
    sd = dev(s.reshape(ny, nx))
    for step in range(3):
        sd_new, outer, res = tg.transport_step(ud, qd, sd, dt)
        s_new = host(sd_new).ravel()
        r = transport_residual(s_new, s, out, nb, q.ravel(), coef, 1.0, 5.0)
        print(f"1024^2 step {step}: {outer} tile launches, GPU max |R| {res:.1e}, oracle {np.abs(r).max():.1e}")
        assert np.abs(r).max() <= _residual_bound(a_max)
        assert s_new.min() >= 0.0 and s_new.max() <= 1.0
        s, sd = s_new, sd_new
    assert s.max() > 0.5


def test_total_mobility():
    _need_gpu()
    import paper_1807_07220_amd as tg
    s = np.random.default_rng(5).uniform(0, 1, (33, 19))
    lam = host(tg.total_mobility(dev(s), mu_w=0.5, mu_o=3.0))
    np.testing.assert_allclose(lam, s * s / 0.5 + (1 - s) ** 2 / 3.0, rtol=1e-15, atol=0)


def test_transport_rejects_bad_parameters():
    _need_gpu()
    import paper_1807_07220_amd as tg
    u = dev(np.zeros(tg.nfaces(8, 8)))
    q = dev(np.zeros((8, 8)))
    s = dev(np.zeros((8, 8)))
    for kw in ({"phi": 0.0}, {"mu_w": -1.0}, {"tol": 0.0}, {"max_outer": -1}):
        with pytest.raises(tg.TgmsError) as e:
            tg.transport_step(u, q, s, 0.1, **kw)
        assert e.value.status == "INVAL"
    with pytest.raises(tg.TgmsError):
        tg.transport_step(u, q, s, -0.1)


@pytest.mark.parametrize("coarse_space", ["gmsfem", "rt0"])
def test_impes_matches_oracle(coarse_space):
    """Section 6.2's loop (mobility of the current saturation, pressure by the two-grid PCG
    with the initial coarse space kept, one transport step) against the oracle's loop:
    PCG iteration counts within one, and the final saturations.  The pressure solves stop
    at rtol 1e-10 on both sides; their velocities then agree to about 1e-9 relative, which
    bounds the saturations' difference at about 1e-7 after a few steps."""
    _need_gpu()
    import paper_1807_07220_amd as tg
    from oracle import OracleSolver
    from oracle.discretization import Grid2D
    from oracle.transport import impes
    nx = ny = 64
    rng = np.random.default_rng(11)
    kappa = np.exp(2.0 * fields.gaussian_field_2d(nx, ny, 0.1, rng))
    F = fields.corner_source(nx, ny)
    o = OracleSolver(Grid2D(nx, ny, 8, 8), kappa, 4.0, basis=coarse_space)
    s_o, its_o = impes(o, F.ravel(), np.zeros(nx * ny), steps=6, dt=0.005, pressure_every=2, rtol=1e-10)
    sv = tg.Solver(dev(kappa), 8, 8, 4.0, coarse_space=coarse_space)
    try:
        r = sv.impes(dev(F), dev(np.zeros((ny, nx))), steps=6, dt=0.005, pressure_every=2, rtol=1e-10)
    finally:
        sv.close()
    err = np.abs(host(r["s"]).ravel() - s_o).max()
    print(f"IMPES {coarse_space}: PCG {r['pcg_iters']} (oracle {its_o}), max |s diff| {err:.2e}")
    assert len(r["pcg_iters"]) == 3
    assert all(abs(a - b) <= 1 for a, b in zip(r["pcg_iters"], its_o))
    assert err <= 1e-7
    assert s_o.max() > 0.5
