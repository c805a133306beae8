"""Seeded synthetic permeability fields and sources.

These generators produce inputs only: a cell-wise permeability array and a
cell-integrated source.  They hold none of the solver's arithmetic and are
shared by the oracle tests, the GPU tests and the benchmark.

The paper's own fields (a 2D channel/inclusion model, a 3D inclusion model
and the SPE10 layers; section 6, figure "Permeability fields") are not
available, so these generators stand in for them with the same ingredients:
a log-normal background plus high-permeability channels and inclusions whose
permeability equals the contrast value.

All geometry is expressed in physical coordinates of the unit square, so a
seed yields the same geometry at every resolution.  Arrays are indexed
``[j, i]`` (row j along y, column i along x, x fastest in memory).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_field_2d(nx: int, ny: int, corr_len: float, rng: np.random.Generator) -> np.ndarray:
    """Unit-variance Gaussian field with exponential covariance exp(-r/corr_len).

    Sampled exactly on the cell centres by circulant embedding on a torus
    padded to twice the domain in each direction; negative circulant
    eigenvalues (if any) are clipped to zero.
    """
    px, py = 2 * nx, 2 * ny
    hx, hy = 1.0 / nx, 1.0 / ny
    dx = np.minimum(np.arange(px), px - np.arange(px)) * hx
    dy = np.minimum(np.arange(py), py - np.arange(py)) * hy
    r = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2)
    cov = np.exp(-r / corr_len)
    lam = np.fft.fft2(cov).real
    lam = np.clip(lam, 0.0, None)
    xi = rng.standard_normal((py, px)) + 1j * rng.standard_normal((py, px))
    g = np.fft.fft2(np.sqrt(lam / (px * py)) * xi)
    return np.ascontiguousarray(g.real[:ny, :nx])


def _cell_centres(nx: int, ny: int):
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    return np.meshgrid(x, y)  # X[j,i], Y[j,i]


def straight_channels(nx, ny, count, width, rng):
    """Boolean mask of ``count`` straight channels through random points."""
    X, Y = _cell_centres(nx, ny)
    mask = np.zeros((ny, nx), dtype=bool)
    for _ in range(count):
        px, py = rng.uniform(0.0, 1.0, size=2)
        ang = rng.uniform(0.0, np.pi)
        nxv, nyv = -np.sin(ang), np.cos(ang)
        dist = np.abs((X - px) * nxv + (Y - py) * nyv)
        mask |= dist <= 0.5 * width
    return mask


def curved_channels(nx, ny, count, rng, amp=(0.02, 0.08), wavelen=(0.2, 0.6), width=(0.006, 0.016)):
    """Boolean mask of sinuous channels.

    Each channel follows y' = y0 + A sin(2 pi x'/L + phi) in a frame rotated by
    a random angle about a random centre; a cell belongs to the channel when
    its distance to that curve (first-order, normal to the curve) is at most
    half the width.
    """
    X, Y = _cell_centres(nx, ny)
    mask = np.zeros((ny, nx), dtype=bool)
    for _ in range(count):
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        ang = rng.uniform(0.0, np.pi)
        a = rng.uniform(*amp)
        lw = rng.uniform(*wavelen)
        phi = rng.uniform(0.0, 2 * np.pi)
        w = rng.uniform(*width)
        c, s = np.cos(ang), np.sin(ang)
        xr = (X - cx) * c + (Y - cy) * s
        yr = -(X - cx) * s + (Y - cy) * c
        k = 2 * np.pi / lw
        centre = a * np.sin(k * xr + phi)
        slope = a * k * np.cos(k * xr + phi)
        dist = np.abs(yr - centre) / np.sqrt(1.0 + slope ** 2)
        mask |= dist <= 0.5 * w
    return mask


def rect_inclusions(nx, ny, count, rng, side=(0.01, 0.05)):
    """Boolean mask of ``count`` axis-aligned rectangles."""
    X, Y = _cell_centres(nx, ny)
    mask = np.zeros((ny, nx), dtype=bool)
    for _ in range(count):
        wx, wy = rng.uniform(*side, size=2)
        x0 = rng.uniform(0.0, 1.0 - wx)
        y0 = rng.uniform(0.0, 1.0 - wy)
        mask |= (X >= x0) & (X <= x0 + wx) & (Y >= y0) & (Y <= y0 + wy)
    return mask


def field_straight(nx, ny, seed, log_var=1.0, corr_len=0.1, n_channels=3, width=None, contrast=1e4):
    """Log-normal background plus straight channels at permeability ``contrast``."""
    rng = _rng(seed)
    g = gaussian_field_2d(nx, ny, corr_len, rng)
    kappa = np.exp(np.sqrt(log_var) * g)
    w = width if width is not None else 1.0 / 32.0
    mask = straight_channels(nx, ny, n_channels, w, rng)
    kappa[mask] = contrast
    return kappa


def field_channelized(nx, ny, seed, log_var=2.0, corr_len=0.05, n_channels=20, n_incl=40, contrast=1e6):
    """Log-normal background plus curved channels and rectangular inclusions."""
    rng = _rng(seed)
    g = gaussian_field_2d(nx, ny, corr_len, rng)
    kappa = np.exp(np.sqrt(log_var) * g)
    mask = curved_channels(nx, ny, n_channels, rng) | rect_inclusions(nx, ny, n_incl, rng)
    kappa[mask] = contrast
    return kappa


def field_binary(nx, ny, seed, value, n_channels=3, n_incl=6):
    """Binary medium: 1 in the background, ``value`` in channels and inclusions.

    Used for contrast sweeps (the paper varies the channel/inclusion value over
    1e-6 .. 1e6 with the background fixed at 1); the geometry depends only on
    the seed, so every value in a sweep sees the same channels.
    """
    rng = _rng(seed)
    mask = straight_channels(nx, ny, n_channels, 1.5 / nx if nx >= 32 else 1.0 / nx, rng)
    mask |= rect_inclusions(nx, ny, n_incl, rng, side=(0.06, 0.12))
    kappa = np.ones((ny, nx))
    kappa[mask] = value
    return kappa


def corner_source(nx, ny):
    """Cell-integrated source: +1 in cell (0,0), -1 in cell (nx-1, ny-1)."""
    f = np.zeros((ny, nx))
    f[0, 0] = 1.0
    f[ny - 1, nx - 1] = -1.0
    return f


def random_source(nx, ny, seed):
    """Zero-sum random cell-integrated source (for parity tests)."""
    rng = _rng(seed)
    f = rng.standard_normal((ny, nx))
    return f - f.mean()


def mobility_front(nx, ny, t, mu_ratio=5.0, width=0.05):
    """Total mobility of a water front advancing from the cell-(0,0) corner.

    Water saturation s = 1 / (1 + exp((r - t) / width)) with r the distance of the
    cell centre from (0, 0) and t in [0, sqrt(2)] the front position; quadratic
    relative permeabilities k_w = s^2, k_o = (1 - s)^2 and viscosities 1 (water)
    and mu_ratio (oil): lambda = s^2 + (1 - s)^2 / mu_ratio (a synthetic stand-in for
    the mobility of a transport step).
    """
    x, y = _cell_centres(nx, ny)
    r = np.sqrt(x ** 2 + y ** 2)
    s = 1.0 / (1.0 + np.exp(np.clip((r - t) / width, -60.0, 60.0)))
    return s ** 2 + (1.0 - s) ** 2 / mu_ratio


def gradient_flow(nx, ny, seed, corr_len=0.1):
    """A total velocity and matching sources for transport tests on any grid.

    Face normal velocities (full face numbering: (nx+1)*ny x-faces, row j first, then
    nx*(ny+1) y-faces) are minus the difference of a seeded smooth potential (a Gaussian
    field plus a diagonal tilt) across the face times a seeded positive face weight, zero
    on the boundary of the square; the cell-integrated source is each cell's net outflow,
    so the pair is consistent.  Scaled so that the sources sum to 1 over the injecting
    cells.  Returns (u, q) with q indexed [j, i].
    """
    rng = _rng(seed)
    x, y = _cell_centres(nx, ny)
    phi = gaussian_field_2d(nx, ny, corr_len, rng) * 0.2 - 2.0 * (x + y)
    w = np.exp(0.5 * gaussian_field_2d(nx + 1, ny + 1, corr_len, rng))
    ux = np.zeros((ny, nx + 1))
    ux[:, 1:nx] = -(phi[:, 1:] - phi[:, :-1]) * nx * w[:ny, 1:nx]
    uy = np.zeros((ny + 1, nx))
    uy[1:ny, :] = -(phi[1:, :] - phi[:-1, :]) * ny * w[1:ny, :nx]
    q = (ux[:, 1:] - ux[:, :-1]) / ny + (uy[1:, :] - uy[:-1, :]) / nx
    scale = 1.0 / np.sum(np.maximum(q, 0.0))
    return np.concatenate([ux.ravel(), uy.ravel()]) * scale, q * scale


def field_layered_3d(nx, ny, nz, seed, n_smooth=None, log_var=3.0, corr_len=0.1, n_channels=6, contrast=1e7):
    """Layered permeability of the cube, indexed [k, j, i] (layer k along z, x fastest).

    The top ``n_smooth`` layers (largest k; by default 35 of every 85) are a smooth
    log-normal medium: per layer a
    Gaussian field in the (x, y) plane, correlated between neighbouring layers by an
    AR(1) blend, scaled to log-variance ``log_var``.  The layers below are fluvial: a
    low-permeability log-normal background (log-variance 1) cut by sinuous channels whose
    geometry drifts slowly from layer to layer (a new set every 5 layers), channel and
    background values set ``contrast`` apart.  A stand-in, built from the same
    ingredients, for the layered reservoir models of the paper's experiments.
    """
    rng = _rng(seed)
    if n_smooth is None:
        n_smooth = int(round(nz * 35 / 85))
    kappa = np.empty((nz, ny, nx))
    prev = gaussian_field_2d(nx, ny, corr_len, rng)
    rho = 0.8
    n_fluvial = max(nz - n_smooth, 0)
    for k in range(nz - 1, nz - 1 - min(n_smooth, nz), -1):
        prev = rho * prev + np.sqrt(1.0 - rho * rho) * gaussian_field_2d(nx, ny, corr_len, rng)
        kappa[k] = np.exp(np.sqrt(log_var) * prev)
    mask = None
    bg = gaussian_field_2d(nx, ny, corr_len, rng)
    low = 1.0 / np.sqrt(contrast)
    for k in range(n_fluvial):
        if k % 5 == 0:
            mask = curved_channels(nx, ny, n_channels, rng, width=(0.04, 0.08))
        bg = rho * bg + np.sqrt(1.0 - rho * rho) * gaussian_field_2d(nx, ny, corr_len, rng)
        layer = low * np.exp(bg)
        layer[mask] = low * contrast
        kappa[k] = layer
    return kappa


def well_pattern_3d(nx, ny, nz):
    """Cell-integrated sources of a five-spot through the whole thickness: injectors in the
    four vertical corner columns (total +1), the producer in the central column (-1)."""
    f = np.zeros((nz, ny, nx))
    for (i, j) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
        f[:, j, i] += 0.25 / nz
    f[:, ny // 2, nx // 2] -= 1.0 / nz
    return f
