"""RT0 x P0 discretisation on a uniform Cartesian grid of the unit square.

Paper section 2, equations "matrixform" and "fine_system": the velocity space
is lowest-order Raviart-Thomas (one normal-velocity unknown per face), the
pressure space is piecewise constant (one unknown per cell),
    A_ij = int_D kappa^{-1} phi_i . phi_j,  B_ij = int_D q_i div phi_j,
    F_i  = int_D f q_i.

Conventions (oracle-internal, "full" face numbering that includes the
boundary faces of D):
  * cell (i, j), 0 <= i < nx, 0 <= j < ny, index c = j*nx + i;
  * x-face at x = i*hx in row j, 0 <= i <= nx, index j*(nx+1) + i;
  * y-face at y = j*hy in column i, 0 <= j <= ny, index (nx+1)*ny + j*nx + i;
  * a face unknown is the normal velocity along +x (x-faces) or +y (y-faces),
    so the basis function phi_e has phi_e . n_e = 1 on face e;
  * q_c is the indicator of cell c.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Grid2D:
    """Fine grid nx x ny on (0,1)^2 with coarse blocks of bx x by cells."""

    def __init__(self, nx: int, ny: int, bx: int | None = None, by: int | None = None):
        self.nx, self.ny = int(nx), int(ny)
        self.hx, self.hy = 1.0 / nx, 1.0 / ny
        self.bx = int(bx) if bx else nx
        self.by = int(by) if by else ny
        if nx % self.bx or ny % self.by:
            raise ValueError("fine grid must be divisible by the coarse block size")
        self.Nx, self.Ny = nx // self.bx, ny // self.by
        self.n_xf = (nx + 1) * ny
        self.n_yf = nx * (ny + 1)
        self.nf = self.n_xf + self.n_yf
        self.nc = nx * ny
        self.cell_area = self.hx * self.hy
        # face length: x-faces are vertical segments of length hy
        self.face_len = np.concatenate([np.full(self.n_xf, self.hy), np.full(self.n_yf, self.hx)])
        self.interior = np.ones(self.nf, dtype=bool)
        jj = np.arange(ny)
        self.interior[jj * (nx + 1)] = False
        self.interior[jj * (nx + 1) + nx] = False
        ii = np.arange(nx)
        self.interior[self.n_xf + ii] = False
        self.interior[self.n_xf + ny * nx + ii] = False
        self.interior_idx = np.flatnonzero(self.interior)
        self.boundary_idx = np.flatnonzero(~self.interior)

    # ---- index helpers -------------------------------------------------
    def xf(self, i, j):
        return np.asarray(j) * (self.nx + 1) + np.asarray(i)

    def yf(self, i, j):
        return self.n_xf + np.asarray(j) * self.nx + np.asarray(i)

    def cell(self, i, j):
        return np.asarray(j) * self.nx + np.asarray(i)

    def cells_in(self, i0, i1, j0, j1):
        """Cells of the rectangle [i0,i1) x [j0,j1) (cell indices)."""
        I, J = np.meshgrid(np.arange(i0, i1), np.arange(j0, j1))
        return self.cell(I.ravel(), J.ravel())

    def faces_in(self, i0, i1, j0, j1):
        """Faces strictly inside the cell rectangle [i0,i1) x [j0,j1).

        These are the faces whose two neighbouring cells both lie in the
        rectangle: the unknowns of V_h cap H_0(div) on that subdomain.
        """
        xi, xj = np.meshgrid(np.arange(i0 + 1, i1), np.arange(j0, j1))
        yi, yj = np.meshgrid(np.arange(i0, i1), np.arange(j0 + 1, j1))
        return np.concatenate([self.xf(xi.ravel(), xj.ravel()), self.yf(yi.ravel(), yj.ravel())])

    def block_of_cells(self):
        """Coarse-block index of every cell."""
        I = np.arange(self.nx) // self.bx
        J = np.arange(self.ny) // self.by
        return (J[:, None] * self.Nx + I[None, :]).ravel()

    # coarse faces strictly inside D: x-faces at X = I*Hx (1 <= I < Nx) for block
    # row J, then y-faces at Y = J*Hy (1 <= J < Ny) for block column I.
    def coarse_faces(self):
        out = []
        for J in range(self.Ny):
            for I in range(1, self.Nx):
                out.append(("x", I, J))
        for J in range(1, self.Ny):
            for I in range(self.Nx):
                out.append(("y", I, J))
        return out


def mass_matrix(g: Grid2D, kinv: np.ndarray) -> sp.csr_matrix:
    """A_ij = int kappa^{-1} phi_i . phi_j over all (full-numbered) faces.

    On cell c = [x0,x1] x [y0,y1] with constant kinv_c, the two x-face basis
    functions restricted to c are ((x - x0)/hx, 0) and ((x1 - x)/hx, 0), whose
    products integrate to |c|/3 (same face) and |c|/6 (opposite faces); the
    x- and y-components are orthogonal.  (Section 2, eq. fine_system.)
    """
    nx, ny = g.nx, g.ny
    k = np.asarray(kinv, dtype=np.float64).reshape(ny, nx)
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    a = g.cell_area * k
    rows, cols, vals = [], [], []
    for lo, hi in ((g.xf(I, J), g.xf(I + 1, J)), (g.yf(I, J), g.yf(I, J + 1))):
        lo, hi = lo.ravel(), hi.ravel()
        av = a.ravel()
        rows += [lo, hi, lo, hi]
        cols += [lo, hi, hi, lo]
        vals += [av / 3.0, av / 3.0, av / 6.0, av / 6.0]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.nf, g.nf))


def div_matrix(g: Grid2D) -> sp.csr_matrix:
    """B_cf = int_c div phi_f: +|f| on the cell's high face, -|f| on its low face."""
    nx, ny = g.nx, g.ny
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    c = g.cell(I, J).ravel()
    rows = np.concatenate([c, c, c, c])
    cols = np.concatenate([g.xf(I + 1, J).ravel(), g.xf(I, J).ravel(), g.yf(I, J + 1).ravel(), g.yf(I, J).ravel()])
    vals = np.concatenate([np.full(c.size, g.hy), np.full(c.size, -g.hy), np.full(c.size, g.hx), np.full(c.size, -g.hx)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.nc, g.nf))


def source_vector(F_cells: np.ndarray) -> np.ndarray:
    """F_c = int_c f; inputs are already cell-integrated, so this flattens."""
    return np.asarray(F_cells, dtype=np.float64).ravel().copy()


def interior_to_full(g: Grid2D, x_int: np.ndarray, g_bnd: np.ndarray | None = None) -> np.ndarray:
    out = np.zeros(g.nf)
    out[g.interior_idx] = x_int
    if g_bnd is not None:
        out[g.boundary_idx] = g_bnd
    return out


def dof_count(n_cells_per_axis) -> int:
    """Unknowns of the RT0-P0 system on a uniform box grid with no-flow boundary.

    Interior faces + cells + 1 (the mean-zero pressure multiplier); valid in
    any dimension.  Section 6 quotes this count for its two 3D fine grids.
    """
    n = [int(v) for v in n_cells_per_axis]
    cells = int(np.prod(n))
    faces = 0
    for a in range(len(n)):
        faces += (n[a] - 1) * cells // n[a]
    return faces + cells + 1
