"""RT0 x P0 discretisation on a uniform Cartesian grid of the unit cube.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper section 2, equations "matrixform" and "fine_system", in three dimensions
(the paper's models 2 and 3): one normal-velocity unknown per face, one
pressure per cell,
    A_ij = int_D kappa^{-1} phi_i . phi_j,  B_ij = int_D q_i div phi_j,
    F_i  = int_D f q_i.

Numbering ("full", boundary faces included):
  * cell (i, j, k), index c = (k*ny + j)*nx + i;
  * x-face at x = i*hx in cell row (j, k), 0 <= i <= nx: index (k*ny + j)*(nx+1) + i;
  * y-face at y = j*hy in column (i, k), 0 <= j <= ny:
    n_xf + (k*(ny+1) + j)*nx + i;
  * z-face at z = k*hz in column (i, j), 0 <= k <= nz:
    n_xf + n_yf + (k*ny + j)*nx + i;
  * a face unknown is the normal velocity along +x, +y or +z.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Grid3D:
    """Fine grid nx x ny x nz on (0,1)^3 with coarse blocks of bx x by x bz cells."""

    def __init__(self, nx, ny, nz, bx=None, by=None, bz=None):
        self.n = (int(nx), int(ny), int(nz))
        self.nx, self.ny, self.nz = self.n
        self.h = tuple(1.0 / v for v in self.n)
        self.b = (int(bx or nx), int(by or ny), int(bz or nz))
        self.bx, self.by, self.bz = self.b
        if any(n % b for n, b in zip(self.n, self.b)):
            raise ValueError("fine grid must be divisible by the coarse block size")
        self.N = tuple(n // b for n, b in zip(self.n, self.b))
        self.Nx, self.Ny, self.Nz = self.N
        nx, ny, nz = self.n
        self.n_xf = (nx + 1) * ny * nz
        self.n_yf = nx * (ny + 1) * nz
        self.n_zf = nx * ny * (nz + 1)
        self.nf = self.n_xf + self.n_yf + self.n_zf
        self.nc = nx * ny * nz
        self.cell_vol = self.h[0] * self.h[1] * self.h[2]
        self.face_area = np.concatenate([np.full(self.n_xf, self.h[1] * self.h[2]),
                                         np.full(self.n_yf, self.h[0] * self.h[2]),
                                         np.full(self.n_zf, self.h[0] * self.h[1])])
        I, J, K = self._mesh(nx, ny, nz)
        bnd = np.concatenate([self.face(0, 0, J, K), self.face(0, nx, J, K),
                              self.face(1, I, 0, K), self.face(1, I, ny, K),
                              self.face(2, I, J, 0), self.face(2, I, J, nz)]).ravel()
        self.interior = np.ones(self.nf, dtype=bool)
        self.interior[bnd] = False
        self.interior_idx = np.flatnonzero(self.interior)
        self.boundary_idx = np.flatnonzero(~self.interior)

    @staticmethod
    def _mesh(a, b, c):
        K, J, I = np.meshgrid(np.arange(c), np.arange(b), np.arange(a), indexing="ij")
        return I, J, K

    # ---- index helpers -------------------------------------------------
    def cell(self, i, j, k):
        return (np.asarray(k) * self.ny + np.asarray(j)) * self.nx + np.asarray(i)

    def face(self, axis, i, j, k):
        """Face of `axis` whose low corner is the vertex (i, j, k)."""
        i, j, k = np.asarray(i), np.asarray(j), np.asarray(k)
        nx, ny, nz = self.n
        if axis == 0:
            return (k * ny + j) * (nx + 1) + i
        if axis == 1:
            return self.n_xf + (k * (ny + 1) + j) * nx + i
        return self.n_xf + self.n_yf + (k * ny + j) * nx + i

    def cells_in(self, lo, hi):
        """Cells of the box [lo, hi) (per axis, in cell indices)."""
        I, J, K = self._mesh(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])
        return self.cell(I + lo[0], J + lo[1], K + lo[2]).ravel()

    def faces_in(self, lo, hi):
        """Faces whose two neighbouring cells both lie in the box [lo, hi)."""
        out = []
        for a in range(3):
            l2, h2 = list(lo), list(hi)
            l2[a] += 1  # faces strictly between cells along a
            if h2[a] - l2[a] < 1:
                continue
            I, J, K = self._mesh(h2[0] - l2[0], h2[1] - l2[1], h2[2] - l2[2])
            out.append(self.face(a, I + l2[0], J + l2[1], K + l2[2]).ravel())
        return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)

    def block_box(self, I, pad=0):
        """Cell box of coarse block I = (Ix, Iy, Iz), enlarged by pad cells and clipped to D."""
        lo = [max(I[a] * self.b[a] - pad, 0) for a in range(3)]
        hi = [min((I[a] + 1) * self.b[a] + pad, self.n[a]) for a in range(3)]
        return lo, hi

    def blocks(self):
        return [(ix, iy, iz) for iz in range(self.Nz) for iy in range(self.Ny) for ix in range(self.Nx)]

    def block_of_cells(self):
        I, J, K = self._mesh(*self.n)
        return ((K // self.bz * self.Ny + J // self.by) * self.Nx + I // self.bx).ravel()

    def coarse_faces(self):
        """Interior coarse faces (axis, I) with I the coarse vertex at the face's low corner:
        x-faces (X = Ix, 1 <= Ix < Nx), then y-faces, then z-faces, each in block order."""
        out = []
        for a in range(3):
            for iz in range(self.Nz + (a == 2)):
                for iy in range(self.Ny + (a == 1)):
                    for ix in range(self.Nx + (a == 0)):
                        I = (ix, iy, iz)
                        if 1 <= I[a] < self.N[a]:
                            out.append((a, I))
        return out


def mass_matrix(g: Grid3D, kinv) -> sp.csr_matrix:
    """A over all faces: per cell and axis, |c| kinv_c / 3 on the two faces of that axis
    and |c| kinv_c / 6 between them (exact integrals of the RT0 basis on a box; no
    coupling across axes for scalar kappa)."""
    kv = np.asarray(kinv, dtype=np.float64).ravel() * g.cell_vol
    I, J, K = g._mesh(*g.n)
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    rows, cols, vals = [], [], []
    for a, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        lo = g.face(a, I, J, K)
        hi = g.face(a, I + di, J + dj, K + dk)
        rows += [lo, hi, lo, hi]
        cols += [lo, hi, hi, lo]
        vals += [kv / 3.0, kv / 3.0, kv / 6.0, kv / 6.0]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(g.nf, g.nf))


def div_matrix(g: Grid3D) -> sp.csr_matrix:
    """B_cf = int_c div phi_f: +|f| on the cell's high face of each axis, -|f| on its low face."""
    I, J, K = g._mesh(*g.n)
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    c = g.cell(I, J, K)
    rows, cols, vals = [], [], []
    for a, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        area = g.cell_vol / g.h[a]
        rows += [c, c]
        cols += [g.face(a, I + di, J + dj, K + dk), g.face(a, I, J, K)]
        vals += [np.full(c.size, area), np.full(c.size, -area)]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(g.nc, g.nf))
