"""Pins of the oracle's two-phase transport (section 6.2, CPU): conservation, the bounds
of the saturation, the Newton Jacobian, and convergence to the Buckley-Leverett solution."""
import numpy as np
import pytest

from oracle.discretization import Grid2D
from oracle.transport import (face_fluxes, fractional_flow, impes, total_mobility, transport_jacobian,
                              transport_residual, transport_step)
from workloads import fields

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _flow(n=16, seed=3):
    """A divergence-free-plus-sources face flux from an oracle pressure solve."""
    from oracle import OracleSolver
    g = Grid2D(n, n, n // 4, n // 4)
    kappa = np.exp(np.random.default_rng(seed).standard_normal((n, n)))
    F = fields.corner_source(n, n).ravel()
    o = OracleSolver(g, kappa, 0.5)
    return g, o, o.solve(F, rtol=1e-12)["u"], F


def test_fractional_flow_and_mobility():
    s = np.linspace(0, 1, 11)
    f, df = fractional_flow(s, 1.0, 5.0)
    assert f[0] == 0.0 and f[-1] == 1.0 and np.all(np.diff(f) > 0)
    h = 1e-6
    fd = (fractional_flow(s[1:-1] + h)[0] - fractional_flow(s[1:-1] - h)[0]) / (2 * h)
    assert np.allclose(df[1:-1], fd, rtol=1e-7)
    assert np.allclose(total_mobility(s), s ** 2 + (1 - s) ** 2 / 5.0)


def test_step_conserves_water_and_stays_in_bounds():
    """Summed over the cells the upwind fluxes cancel: the water volume changes by exactly
    dt (sum q^+ + sum f_w(s_i) q^-); the saturation stays in [0, 1]."""
    g, o, u, F = _flow()
    s = np.zeros(g.nc)
    dt, phi = 0.02, 0.2
    for _ in range(5):
        s_new, it = transport_step(g, u, F, s, dt, phi)
        f, _ = fractional_flow(s_new)
        gain = phi * g.cell_area * np.sum(s_new - s)
        assert abs(gain - dt * (np.sum(np.maximum(F, 0)) + np.sum(f * np.minimum(F, 0)))) < 1e-12
        assert s_new.min() >= 0.0 and s_new.max() <= 1.0 and it <= 40
        s = s_new
    assert s.max() > 0.3


def test_jacobian_against_finite_differences():
    g, o, u, F = _flow(n=8)
    out, nb = face_fluxes(g, u)
    s = np.random.default_rng(1).uniform(0.1, 0.9, g.nc)
    s0 = s.copy()
    coef = 0.05 / (0.2 * g.cell_area)
    Jm = transport_jacobian(s, out, nb, F, coef, 1.0, 5.0).toarray()
    h = 1e-7
    for j in range(0, g.nc, 7):
        e = np.zeros(g.nc)
        e[j] = h
        col = (transport_residual(s + e, s0, out, nb, F, coef, 1.0, 5.0)
               - transport_residual(s - e, s0, out, nb, F, coef, 1.0, 5.0)) / (2 * h)
        assert np.allclose(Jm[:, j], col, atol=1e-6 * np.abs(Jm).max())


def test_converges_to_buckley_leverett():
    """A 1D strip with uniform injection at the left: the implicit upwind saturation at
    t approaches the Buckley-Leverett profile, whose front (Welge tangent) travels at
    f_w(s_f) / s_f with f_w'(s_f) = f_w(s_f) / s_f; the L1 error falls with the grid."""
    phi, t_end = 1.0, 0.3
    s_grid = np.linspace(1e-6, 1, 200001)
    f, df = fractional_flow(s_grid)
    sf = s_grid[np.argmax(f / s_grid)]  # the tangent from the origin touches f_w at its largest f_w / s
    errs = []
    for n in (100, 200, 400):
        g = Grid2D(n, 1, n, 1)
        # unit flux to the right through every interior x-face, source +1 / sink -1
        u = np.zeros(g.nf)
        u[g.xf(np.arange(1, n), 0)] = 1.0 / g.hy
        F = np.zeros(n)
        F[0], F[-1] = 1.0, -1.0
        s = np.zeros(n)
        steps = n // 2
        for _ in range(steps):
            s, _ = transport_step(g, u, F, s, t_end / steps, phi)
        x = (np.arange(n) + 0.5) / n
        # exact profile: s(x) with f_w'(s) = x / t behind the front, 0 ahead of it
        exact = np.zeros(n)
        behind = x < t_end * df[np.searchsorted(s_grid, sf)]
        for i in np.flatnonzero(behind):
            cand = np.flatnonzero((df[::-1] >= x[i] / t_end))
            exact[i] = s_grid[::-1][cand[0]] if cand.size else 1.0
        exact[behind] = np.maximum(exact[behind], sf)
        errs.append(np.mean(np.abs(s - exact)))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 0.03, errs


def test_impes_loop_with_kept_coarse_space():
    """The coupled loop: pressure with the previous mobility (basis of the initial
    permeability kept), then transport; the water front moves from the injector and
    every pressure solve converges."""
    g, o, u, F = _flow()
    s, its = impes(o, F, np.zeros(g.nc), steps=6, dt=0.02, pressure_every=2)
    assert len(its) == 3 and max(its) < 40
    assert s[0] > 0.5 and s[-1] < s[0]


def test_cube_step_along_each_axis_matches_the_strip():
    """The cube's six-sided fluxes: a column of n cells along x, y or z with a unit flux
    through its interior faces gives the saturation of the same strip on the square."""
    from oracle.grid3d import Grid3D
    n, dt = 12, 0.05
    g2 = Grid2D(n, 1, n, 1)
    u2 = np.zeros(g2.nf)
    u2[g2.xf(np.arange(1, n), 0)] = 1.0 / g2.hy
    F = np.zeros(n)
    F[0], F[-1] = 1.0, -1.0
    s2, _ = transport_step(g2, u2, F, np.zeros(n), dt, 1.0)
    for a in range(3):
        dims = [1, 1, 1]
        dims[a] = n
        g3 = Grid3D(*dims)
        u3 = np.zeros(g3.nf)
        area = g3.cell_vol / g3.h[a]
        for t in range(1, n):
            q = [0, 0, 0]
            q[a] = t
            u3[g3.face(a, *q)] = 1.0 / area
        s3, _ = transport_step(g3, u3, F, np.zeros(n), dt, 1.0)
        np.testing.assert_allclose(s3, s2, rtol=0, atol=1e-13)
