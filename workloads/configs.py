"""Named synthetic workloads (the unit square or cube, uniform Cartesian grids).

Each workload fixes the fine grid, the coarse block size, the permeability
generator and its seed, the source, the eigenvalue tolerance and the
precision of the preconditioner.  ``make_inputs`` returns the permeability
and the cell-integrated source as float64 arrays of shape (ny, nx), or
(nz, ny, nx) on the cube.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fields


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    bx: int
    by: int
    generator: str
    seed: int
    eig_tol: float
    rtol: float = 1e-8
    precision: str = "fp64"  # "fp64" or "mixed"
    contrast: float = 1e6

    nz: int = 0  # > 0: the unit cube
    bz: int = 0

    def make_inputs(self):
        if self.generator == "layered3d":
            return (fields.field_layered_3d(self.nx, self.ny, self.nz, self.seed, contrast=self.contrast),
                    fields.well_pattern_3d(self.nx, self.ny, self.nz))
        if self.generator == "straight":
            kappa = fields.field_straight(self.nx, self.ny, self.seed, contrast=self.contrast)
        elif self.generator == "channelized":
            kappa = fields.field_channelized(self.nx, self.ny, self.seed, contrast=self.contrast)
        else:
            raise ValueError(self.generator)
        return kappa, fields.corner_source(self.nx, self.ny)


WORKLOADS = {
    # 32x32 fine, 4x4 coarse, GRF(var 1, len 0.1) + 3 straight channels at 1e4, tol 0.5.
    "darcy2d_32_b8": Workload("darcy2d_32_b8", 32, 32, 8, 8, "straight", 1, 0.5, contrast=1e4),
    # 256x256 fine, 16x16 coarse, GRF(var 2, len 0.05) + 20 curved channels + 40 inclusions at 1e6, tol 0.2.
    "darcy2d_256_b16": Workload("darcy2d_256_b16", 256, 256, 16, 16, "channelized", 2, 0.2),
    # 1024x1024 fine, 64x64 coarse, same generator, FP32 preconditioner inside flexible FP64 PCG.
    "darcy2d_1024_b16_mixed": Workload("darcy2d_1024_b16_mixed", 1024, 1024, 16, 16, "channelized", 3, 0.2,
                                       precision="mixed"),
    "darcy2d_1024_b16": Workload("darcy2d_1024_b16", 1024, 1024, 16, 16, "channelized", 3, 0.2),
    # 1024x1024 fine, 128x128 coarse (8x8 blocks).
    "darcy2d_1024_b8": Workload("darcy2d_1024_b8", 1024, 1024, 8, 8, "channelized", 5, 0.2),
    # the cube: 60x220x85 cells in 5x11x5 blocks, layered (35 smooth log-normal layers of
    # log-variance 3 over 50 fluvial layers, contrast 1e7), five-spot wells through the
    # thickness; and a 15x33x15 cut of the same shape (3x3x3 blocks, the same patch size)
    "darcy3d_60x220x85_b5x11x5": Workload("darcy3d_60x220x85_b5x11x5", 60, 220, 5, 11, "layered3d", 7, 3.0,
                                          contrast=1e7, nz=85, bz=5),
    "darcy3d_15x33x15_b5x11x5": Workload("darcy3d_15x33x15_b5x11x5", 15, 33, 5, 11, "layered3d", 8, 3.0,
                                         contrast=1e7, nz=15, bz=5),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]
