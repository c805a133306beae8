"""Pins of the oracle's discretisation against brute force and closed forms (CPU)."""
import numpy as np
import pytest

from oracle.discretization import Grid2D, div_matrix, dof_count, mass_matrix
from oracle.solver import exact_solve

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _basis_value(g, face, x, y):
    """RT0 basis function of a full-numbered face evaluated at (x, y) (brute force)."""
    if face < g.n_xf:
        j, i = divmod(face, g.nx + 1)
        xf = i * g.hx
        if not (j * g.hy <= y <= (j + 1) * g.hy):
            return np.zeros(2)
        if xf - g.hx <= x <= xf:
            return np.array([(x - (xf - g.hx)) / g.hx, 0.0])
        if xf <= x <= xf + g.hx:
            return np.array([((xf + g.hx) - x) / g.hx, 0.0])
        return np.zeros(2)
    f = face - g.n_xf
    j, i = divmod(f, g.nx)
    yf = j * g.hy
    if not (i * g.hx <= x <= (i + 1) * g.hx):
        return np.zeros(2)
    if yf - g.hy <= y <= yf:
        return np.array([0.0, (y - (yf - g.hy)) / g.hy])
    if yf <= y <= yf + g.hy:
        return np.array([0.0, ((yf + g.hy) - y) / g.hy])
    return np.zeros(2)


def test_mass_matrix_matches_gauss_quadrature():
    """A_ij = int kinv phi_i.phi_j by 2-point Gauss per cell (exact for these polynomials)."""
    g = Grid2D(4, 3)
    rng = np.random.default_rng(0)
    kinv = rng.uniform(0.1, 5.0, size=g.nc)
    A = mass_matrix(g, kinv).toarray()
    gp = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    Ab = np.zeros((g.nf, g.nf))
    for j in range(g.ny):
        for i in range(g.nx):
            c = g.cell(i, j)
            faces = [g.xf(i, j), g.xf(i + 1, j), g.yf(i, j), g.yf(i, j + 1)]
            for a in gp:
                for b in gp:
                    x, y = (i + a) * g.hx, (j + b) * g.hy
                    vals = [_basis_value(g, f, x, y) for f in faces]
                    w = 0.25 * g.cell_area * kinv[c]
                    for p, fp in enumerate(faces):
                        for q, fq in enumerate(faces):
                            Ab[fp, fq] += w * vals[p] @ vals[q]
    assert np.allclose(A, Ab, rtol=1e-13, atol=1e-15)
    assert np.allclose(A, A.T)
    assert np.all(np.linalg.eigvalsh(A) > 0)


def test_div_matrix_is_boundary_flux():
    """B_cf = int_c div phi_f equals the outward flux of phi_f through dc."""
    g = Grid2D(3, 5)
    B = div_matrix(g).toarray()
    for j in range(g.ny):
        for i in range(g.nx):
            c = g.cell(i, j)
            for f in range(g.nf):
                # outward flux = sum over the 4 edges of (phi_f . n) * edge length, at edge midpoints
                x0, x1, y0, y1 = i * g.hx, (i + 1) * g.hx, j * g.hy, (j + 1) * g.hy
                xm, ym = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
                eps = 1e-12
                flux = (_basis_value(g, f, x1 - eps, ym)[0] - _basis_value(g, f, x0 + eps, ym)[0]) * g.hy
                flux += (_basis_value(g, f, xm, y1 - eps)[1] - _basis_value(g, f, xm, y0 + eps)[1]) * g.hx
                assert abs(B[c, f] - flux) < 1e-9


def test_dof_counts_match_paper():
    """Section 6 quotes the unknown counts of its two 3D fine grids and the RT0
    coarse dimensions; with no-flow boundaries each is interior faces + cells +
    1 (the mean-zero pressure multiplier).  Values in tests/golden/paper_counts.json."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")) as fh:
        gold = json.load(fh)
    for rec in gold["fine_dof"]:
        assert dof_count(rec["cells"]) == rec["dof"]
    for rec in gold["rt0_coarse_dim"]:
        assert dof_count(rec["blocks"]) == rec["dim"]


def _manufactured(n, k0=2.5):
    """p = cos(pi x) cos(pi y), v = -k0 grad p, f = 2 k0 pi^2 p, v.n = 0 on dD."""
    g = Grid2D(n, n)
    x = np.arange(n + 1) * g.hx
    s = np.sin(np.pi * x)
    F = 2 * k0 * np.outer(s[1:] - s[:-1], s[1:] - s[:-1])   # int_c f, [j, i]
    u, p = exact_solve(g, np.full((n, n), k0), F)
    return g, u, p, k0


def _l2_errors(g, u, p, k0):
    gp = np.array([0.5 - np.sqrt(0.15), 0.5, 0.5 + np.sqrt(0.15)])
    gw = np.array([5, 8, 5]) / 18.0
    ev2 = ep2 = 0.0
    n = g.nx
    for j in range(n):
        for i in range(n):
            ul, ur = u[g.xf(i, j)], u[g.xf(i + 1, j)]
            vb, vt = u[g.yf(i, j)], u[g.yf(i, j + 1)]
            pc = p[g.cell(i, j)]
            for a, wa in zip(gp, gw):
                for b, wb in zip(gp, gw):
                    x, y = (i + a) * g.hx, (j + b) * g.hy
                    vx = k0 * np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
                    vy = k0 * np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
                    vhx = ul + a * (ur - ul)
                    vhy = vb + b * (vt - vb)
                    w = wa * wb * g.cell_area
                    ev2 += w * ((vx - vhx) ** 2 + (vy - vhy) ** 2)
                    ep2 += w * (np.cos(np.pi * x) * np.cos(np.pi * y) - pc) ** 2
    return np.sqrt(ev2), np.sqrt(ep2)


def test_manufactured_solution_first_order():
    """L2 errors of v and p fall as O(h) (observed order >= 0.9 over 16 -> 64)."""
    errs = []
    for n in (16, 32, 64):
        errs.append(_l2_errors(*_manufactured(n)))
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders >= 0.9), orders


def test_manufactured_superconvergence_at_faces():
    """Face-centre normal velocities and cell-centre pressures converge as O(h^2)."""
    out = []
    for n in (16, 32, 64):
        g, u, p, k0 = _manufactured(n)
        # face-midpoint values of the exact normal velocity
        ex = np.zeros(g.nf)
        for j in range(n):
            y = (j + 0.5) * g.hy
            for i in range(n + 1):
                ex[g.xf(i, j)] = k0 * np.pi * np.sin(np.pi * i * g.hx) * np.cos(np.pi * y)
        for j in range(n + 1):
            for i in range(n):
                x = (i + 0.5) * g.hx
                ex[g.yf(i, j)] = k0 * np.pi * np.cos(np.pi * x) * np.sin(np.pi * j * g.hy)
        xc = (np.arange(n) + 0.5) * g.hx
        pc = np.outer(np.cos(np.pi * xc), np.cos(np.pi * xc)).ravel()
        out.append((np.abs(u - ex).max() / np.abs(ex).max(), np.abs(p - pc).max()))
    out = np.array(out)
    orders = np.log2(out[:-1] / out[1:])
    assert np.all(orders >= 1.8), orders


def test_exact_solve_with_boundary_data():
    """Nonzero normal flux on dD: the discrete solution reproduces a linear pressure exactly.

    p = -x (so v = (kappa, 0) for constant kappa) lies in the discrete spaces'
    reach: with g = v.n on dD and f = 0 the RT0-P0 solution is exact up to
    round-off (constant velocity is in RT0, cell averages of a linear p are
    its cell-centre values).
    """
    n, k0 = 8, 3.0
    g = Grid2D(n, n)
    gf = np.zeros(g.nf)
    for j in range(n):
        gf[g.xf(0, j)] = k0
        gf[g.xf(n, j)] = k0
    u, p = exact_solve(g, np.full((n, n), k0), np.zeros((n, n)), gf)
    assert np.allclose(u[: g.n_xf], k0, atol=1e-12)
    assert np.allclose(u[g.n_xf:], 0.0, atol=1e-12)
    xc = (np.arange(n) + 0.5) * g.hx
    pex = np.tile(-xc, n)
    pex -= pex.mean()
    assert np.allclose(p, pex, atol=1e-12)
