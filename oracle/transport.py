"""Two-phase flow by IMPES (section 6.2): saturation transport, mobility, the coupled loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Equations (section 6.2, eqs. satEq, fraction, mobility, DisSatEq_Implicit,
integralFlux): with quadratic relative permeabilities k_rw = s^2, k_ro = (1-s)^2
  total mobility     lambda(s) = s^2 / mu_w + (1 - s)^2 / mu_o,
  fractional flow    f_w(s) = (s^2 / mu_w) / lambda(s),
and the backward-Euler upwind finite-volume step for every cell i
  phi |Omega_i| (s_i - s_i^n) / dt = q_i^+ - sum_j f_w(s_up(ij)) u_ij + f_w(s_i) q_i^-,
with u_ij the total flux out of i through face ij, s_up(ij) the saturation of the
cell the flux leaves (upstream weighting), q^+ = max(q, 0) (water injected) and
q^- = min(q, 0) (fluid produced at the cell's fractional flow).  Readings: the printed
step has no porosity (|Omega_i| alone); the saturation equation's phi is kept, so
phi = 1 gives the printed form.  Each step is solved by Newton's method from s^n,
each update limited to 0.2 per cell and the saturation clipped to [0, 1], until the
largest residual is at most newton_tol; each Newton system is solved directly
(sparse LU).

IMPES: the pressure equation is solved with the mobility of the previous step
(section 6.2), here every `pressure_every` transport steps, with the coarse space of
the initial permeability kept (OracleSolver.update_mobility).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def total_mobility(s, mu_w=1.0, mu_o=5.0):
    s = np.asarray(s, dtype=np.float64)
    return s * s / mu_w + (1.0 - s) ** 2 / mu_o


def fractional_flow(s, mu_w=1.0, mu_o=5.0):
    """f_w and its derivative."""
    s = np.asarray(s, dtype=np.float64)
    a, b = s * s / mu_w, (1.0 - s) ** 2 / mu_o
    lam = a + b
    da, db = 2.0 * s / mu_w, -2.0 * (1.0 - s) / mu_o
    return a / lam, (da * lam - a * (da + db)) / (lam * lam)


def face_fluxes(g, u_full):
    """Per cell and side (W, E, S, N; on the cube also bottom, top) the total flux out of
    the cell and the neighbour across that side (-1 at the boundary of D, where the
    no-flow flux is 0)."""
    u = np.asarray(u_full)
    if hasattr(g, "nz"):
        nx, ny, nz = g.n
        I, J, K = (a.ravel() for a in g._mesh(nx, ny, nz))
        out = np.zeros((g.nc, 6))
        nb = -np.ones((g.nc, 6), dtype=np.int64)
        area = [g.cell_vol / h for h in g.h]
        for a, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            out[:, 2 * a] = -u[g.face(a, I, J, K)] * area[a]
            out[:, 2 * a + 1] = u[g.face(a, I + di, J + dj, K + dk)] * area[a]
            pos = (I, J, K)[a]
            nb[:, 2 * a] = np.where(pos > 0, g.cell(I - di, J - dj, K - dk), -1)
            nb[:, 2 * a + 1] = np.where(pos < g.n[a] - 1, g.cell(I + di, J + dj, K + dk), -1)
        out[nb < 0] = 0.0
        return out, nb
    nx, ny = g.nx, g.ny
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    I, J = I.ravel(), J.ravel()
    out = np.zeros((g.nc, 4))
    nb = -np.ones((g.nc, 4), dtype=np.int64)
    out[:, 0] = -u[g.xf(I, J)] * g.hy
    out[:, 1] = u[g.xf(I + 1, J)] * g.hy
    out[:, 2] = -u[g.yf(I, J)] * g.hx
    out[:, 3] = u[g.yf(I, J + 1)] * g.hx
    nb[:, 0] = np.where(I > 0, g.cell(I - 1, J), -1)
    nb[:, 1] = np.where(I < nx - 1, g.cell(I + 1, J), -1)
    nb[:, 2] = np.where(J > 0, g.cell(I, J - 1), -1)
    nb[:, 3] = np.where(J < ny - 1, g.cell(I, J + 1), -1)
    out[nb < 0] = 0.0
    return out, nb


def transport_residual(s, s_old, out, nb, q, coef, mu_w, mu_o):
    """R_i = s_i - s_i^n - coef (q^+ - sum_j f_w(s_up) u_ij + f_w(s_i) q^-), coef = dt / (phi |Omega_i|)."""
    f, _ = fractional_flow(s, mu_w, mu_o)
    up = np.where(out >= 0.0, f[:, None], np.where(nb >= 0, f[np.maximum(nb, 0)], 0.0))
    flux = np.sum(up * out, axis=1)
    return s - s_old - coef * (np.maximum(q, 0.0) - flux + f * np.minimum(q, 0.0))


def transport_jacobian(s, out, nb, q, coef, mu_w, mu_o) -> sp.csr_matrix:
    _, df = fractional_flow(s, mu_w, mu_o)
    n = s.size
    diag = 1.0 + coef * (np.sum(np.where(out > 0.0, out, 0.0), axis=1) - np.minimum(q, 0.0)) * df
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag]
    for k in range(out.shape[1]):
        m = (out[:, k] < 0.0) & (nb[:, k] >= 0)
        i = np.flatnonzero(m)
        j = nb[i, k]
        rows.append(i); cols.append(j); vals.append(coef * out[i, k] * df[j])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def transport_step(g, u_full, q, s, dt, phi=0.2, mu_w=1.0, mu_o=5.0, newton_tol=1e-12, max_newton=100,
                   max_change=0.2):
    """One backward-Euler upwind step (eq. DisSatEq_Implicit) by Newton: returns (s, iterations).

    The S-shaped f_w makes plain Newton from s^n cycle for long steps (f_w' vanishes at
    s = 0); every update is limited to max_change per cell (an Appleyard chop) before the
    clip to [0, 1]."""
    out, nb = face_fluxes(g, u_full)
    q = np.asarray(q, dtype=np.float64).ravel()
    coef = dt / (phi * (g.cell_vol if hasattr(g, "nz") else g.cell_area))
    s_old = np.asarray(s, dtype=np.float64).ravel().copy()
    s = s_old.copy()
    for it in range(max_newton + 1):
        R = transport_residual(s, s_old, out, nb, q, coef, mu_w, mu_o)
        if np.abs(R).max() <= newton_tol:
            return s, it
        if it == max_newton:
            break
        Jm = transport_jacobian(s, out, nb, q, coef, mu_w, mu_o)
        d = -spla.spsolve(Jm.tocsc(), R)
        s = np.clip(s + np.clip(d, -max_change, max_change), 0.0, 1.0)
    raise RuntimeError("Newton did not converge")


def impes(solver, F, s0, steps, dt, pressure_every=1, phi=0.2, mu_w=1.0, mu_o=5.0, rtol=1e-8):
    """Section 6.2's IMPES loop with the coarse space of the initial permeability kept:
    every `pressure_every` steps the mobility of the current saturation is set and the
    pressure equation solved; then the saturation takes one transport step.  Returns the
    final saturation and per pressure solve the PCG iteration count."""
    s = np.asarray(s0, dtype=np.float64).ravel().copy()
    its, u = [], None
    for k in range(steps):
        if k % pressure_every == 0:
            solver.update_mobility(total_mobility(s, mu_w, mu_o))
            r = solver.solve(F, rtol=rtol)
            u = r["u"]
            its.append(r["iters"])
        s, _ = transport_step(solver.g, u, F, s, dt, phi, mu_w, mu_o)
    return s, its
