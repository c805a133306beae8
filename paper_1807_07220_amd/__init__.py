"""Two-grid GMsFEM-preconditioned mixed Darcy solver on AMD MI355X (gfx950).

``Solver(kappa, bx, by, eig_tol)`` runs the setup (adaptive spectral coarse
space, coarse Cholesky, smoother factors) on the GPU; ``Solver.solve(F, g)``
returns velocity, pressure and the PCG iteration count.  All arrays are
float64 torch tensors on the GPU; the work runs in the HIP library
``libtgms.so`` through its C ABI (include/tgms.h).
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import Grid, Info, Options, TgmsError, TransportParams, check, load  # noqa: F401

__all__ = ["Solver", "TgmsError", "nfaces", "total_mobility", "transport_step", "trim_device_cache"]

COARSE_SPACES = {"gmsfem": 0, "msfem": 1, "rt0": 2}


def trim_device_cache():
    """Return the device blocks the library keeps for reuse to the runtime (tgms_trim_device_cache)."""
    load().tgms_trim_device_cache()


def nfaces(nx: int, ny: int, nz: int | None = None) -> int:
    """Length of a full face array: (nx+1)*ny x-faces then nx*(ny+1) y-faces (the square),
    or x-, y- and z-faces of the nx x ny x nz cube."""
    if nz is None:
        return (nx + 1) * ny + nx * (ny + 1)
    return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _transport_params(**kw) -> TransportParams:
    """tgms_transport_params with the library's defaults, overridden by kw."""
    prm = TransportParams()
    load().tgms_default_transport(ctypes.byref(prm))
    for k, v in kw.items():
        if not hasattr(prm, k):
            raise TypeError(f"unknown transport parameter {k}")
        setattr(prm, k, v)
    return prm


def total_mobility(s: torch.Tensor, **params) -> torch.Tensor:
    """lambda(s) = s^2 / mu_w + (1 - s)^2 / mu_o per cell (tgms_total_mobility)."""
    s = s.contiguous()
    lam = torch.empty_like(s)
    prm = _transport_params(**params)
    check(load().tgms_total_mobility(_ptr(s), s.numel(), ctypes.byref(prm), _ptr(lam),
                                     ctypes.c_void_p(torch.cuda.current_stream(s.device).cuda_stream)))
    return lam


def transport_step(u: torch.Tensor, q: torch.Tensor, s: torch.Tensor, dt: float, **params):
    """One implicit upwind saturation step (tgms_transport_step) on the (ny, nx) grid of s
    (or the (nz, ny, nx) grid of the cube).

    Returns (s_new, tile launches, final max |R_i|); s is not modified."""
    nz, ny, nx = s.shape if s.dim() == 3 else (1, *s.shape)
    s_new = s.contiguous().clone()
    prm = _transport_params(**params)
    outer, res = ctypes.c_longlong(0), ctypes.c_double(0.0)
    check(load().tgms_transport_step(nx, ny, nz if s.dim() == 3 else 1, _ptr(u.contiguous()), _ptr(q.contiguous().reshape(-1)), _ptr(s_new),
                                     float(dt), ctypes.byref(prm),
                                     ctypes.c_void_p(torch.cuda.current_stream(s.device).cuda_stream),
                                     ctypes.byref(outer), ctypes.byref(res)))
    return s_new, outer.value, res.value


class Solver:
    """Setup on construction; see include/tgms.h for the definitions."""

    def __init__(self, kappa: torch.Tensor, bx: int, by: int, eig_tol: float, eta: float = 0.2, overlap: int = 2,
                 precision: str = "fp64", s_scale: float = 1.0, stream: torch.cuda.Stream | None = None,
                 graphs: bool = True, autotune: bool = True, tune_cache: str | None = None,
                 warm_start: str = "exact", cnn_weights: torch.Tensor | None = None, rq_tol: float = 1e-6,
                 smoother_staging: int = -1, rows_per_thread: int = 0, force_counts=None,
                 coarse_space: str = "gmsfem", coarse_factor: str = "auto", smooth_steps: int = 1,
                 additive: bool = False, bz: int | None = None, _restore: str | None = None):
        lib = load()
        if kappa is not None and kappa.dim() not in (2, 3):
            raise ValueError("kappa must be (ny, nx) or (nz, ny, nx)")
        self.dim = 3 if kappa is not None and kappa.dim() == 3 else 2
        self.nz, self.bz = 1, 1
        self.device = kappa.device if kappa is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        opt = Options()
        lib.tgms_default_options(ctypes.byref(opt))
        opt.eta, opt.overlap, opt.s_scale = float(eta), int(overlap), float(s_scale)
        opt.precision = {"fp64": 0, "mixed": 1}[precision]
        opt.stream = ctypes.c_void_p(self.stream.cuda_stream)
        opt.graphs = 1 if graphs else 0
        opt.autotune = 1 if autotune else 0
        self._tune_cache = None if tune_cache is None else str(tune_cache).encode()
        opt.tune_cache = self._tune_cache
        opt.smoother_staging = int(smoother_staging)
        opt.rows_per_thread = int(rows_per_thread)
        opt.coarse_space = COARSE_SPACES[coarse_space]
        opt.coarse_factor = {"auto": 0, "dense": 1, "bcr": 2}[coarse_factor]
        opt.smooth_steps = int(smooth_steps)
        opt.additive = 1 if additive else 0
        if _restore is not None:
            handle = ctypes.c_void_p()
            check(lib.tgms_load(str(_restore).encode(), ctypes.byref(opt), ctypes.byref(handle)))
            self._h = handle
            self._from_info()
            return
        if self.dim == 3:
            self.nz, self.ny, self.nx = kappa.shape
            if bz is None:
                raise ValueError("a cube needs bz")
            self.bz = int(bz)
        else:
            self.ny, self.nx = kappa.shape
        self.bx, self.by = int(bx), int(by)
        if force_counts is not None:
            import numpy as np
            self._force = np.ascontiguousarray(force_counts, dtype=np.int32)
            opt.force_counts = self._force.ctypes.data_as(ctypes.c_void_p)
        opt.warm_start = {"exact": 0, "dct": 1, "cnn": 2}[warm_start]
        if cnn_weights is not None:
            if not (cnn_weights.is_cuda and cnn_weights.dtype == torch.float32 and cnn_weights.is_contiguous()):
                raise ValueError("cnn_weights must be a contiguous float32 CUDA tensor")
            opt.cnn_weights = ctypes.c_void_p(cnn_weights.data_ptr())
        opt.rq_tol = float(rq_tol)
        grid = Grid(self.dim, self.nx, self.ny, self.nz, self.bx, self.by, self.bz)
        handle = ctypes.c_void_p()
        kappa = kappa.contiguous()
        check(lib.tgms_setup(ctypes.byref(grid), _ptr(kappa), float(eig_tol), ctypes.byref(opt),
                             ctypes.byref(handle)))
        self._h = handle
        self.precision = precision

    @classmethod
    def load(cls, path: str, stream: torch.cuda.Stream | None = None, graphs: bool = True, autotune: bool = True,
             tune_cache: str | None = None, smoother_staging: int = -1, rows_per_thread: int = 0) -> "Solver":
        """Restore a context written by save() (tgms_load): the coarse space is read, not solved for."""
        return cls(None, 0, 0, 0.0, stream=stream, graphs=graphs, autotune=autotune, tune_cache=tune_cache,
                   smoother_staging=smoother_staging, rows_per_thread=rows_per_thread, _restore=path)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nfaces(self) -> int:
        return nfaces(self.nx, self.ny, self.nz if self.dim == 3 else None)

    def _from_info(self):
        inf = self.info()
        self.nx, self.ny, self.bx, self.by = inf["nx"], inf["ny"], inf["bx"], inf["by"]
        self.precision = "mixed" if inf["precision"] else "fp64"

    def save(self, path: str):
        """Write the setup artefact (tgms_save)."""
        check(load().tgms_save(self._h, str(path).encode()))

    def probe_pencil(self):
        """Per coarse face the a-form diagonal D [faces][jmax] and s-form S [faces][jmax][jmax] (GPU)."""
        n = self.info()["n_coarse_faces"]
        jmax = max(self.bx, self.by)
        D = torch.empty((n, jmax), dtype=torch.float64, device=self.device)
        S = torch.empty((n, jmax, jmax), dtype=torch.float64, device=self.device)
        check(load().tgms_probe_pencil(self._h, _ptr(D), _ptr(S)))
        return D, S

    # ---- results ----------------------------------------------------------
    def solve(self, F: torch.Tensor, g: torch.Tensor | None = None, rtol: float = 1e-8, maxit: int = 1000,
              pressure: bool = True):
        lib = load()
        F = F.contiguous().reshape(-1)
        u = torch.empty(self.nfaces, dtype=torch.float64, device=self.device)
        p = torch.empty(self.ncells, dtype=torch.float64, device=self.device) if pressure else None
        it, rel = ctypes.c_int(0), ctypes.c_double(0.0)
        code = lib.tgms_solve(self._h, _ptr(F), _ptr(g), float(rtol), int(maxit), _ptr(u), _ptr(p),
                              ctypes.byref(it), ctypes.byref(rel))
        converged = code == 0
        if code not in (0, -3):
            check(code)
        return {"u": u, "p": p, "iters": it.value, "relres": rel.value, "converged": converged}

    def impes(self, F: torch.Tensor, s0: torch.Tensor, steps: int, dt: float, pressure_every: int = 1,
              rtol: float = 1e-8, maxit: int = 1000, **params):
        """Section 6.2's IMPES loop with this context's coarse space kept (tgms_impes).

        Returns {"s": final saturation (ny, nx), "u": last velocity, "pcg_iters": per pressure solve}."""
        F = F.contiguous().reshape(-1)
        s = s0.contiguous().clone()
        u = torch.empty(self.nfaces, dtype=torch.float64, device=self.device)
        npres = (steps + pressure_every - 1) // pressure_every
        its = (ctypes.c_int * max(npres, 1))()
        prm = _transport_params(**params)
        check(load().tgms_impes(self._h, _ptr(F), _ptr(s), int(steps), float(dt), int(pressure_every),
                                ctypes.byref(prm), float(rtol), int(maxit), _ptr(u), ctypes.cast(its, ctypes.c_void_p)))
        return {"s": s, "u": u, "pcg_iters": list(its)[:npres]}

    def update_mobility(self, lam: torch.Tensor):
        """Rebuild the operator for the total mobility lam (cells), keeping the coarse basis."""
        lam = lam.contiguous().reshape(-1)
        if lam.numel() != self.ncells or lam.dtype != torch.float64:
            raise ValueError("mobility must be a float64 field of one value per cell")
        check(load().tgms_update_mobility(self._h, _ptr(lam)))

    def info(self) -> dict:
        inf = Info()
        check(load().tgms_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    def counts(self):
        import numpy as np
        n = self.info()["n_coarse_faces"]
        out = np.zeros(n, dtype=np.int32)
        check(load().tgms_get_counts(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def warm_status(self):
        """Per coarse face: the subspace iteration that accepted it, or -1 (dense fallback)."""
        import numpy as np
        out = np.zeros(self.info()["n_coarse_faces"], dtype=np.int32)
        check(load().tgms_get_warm_status(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def cnn_samples(self):
        """Network inputs [faces][2b][b] and target eigenvectors [faces][8][b] (float32, GPU)."""
        b = self.bx
        n = self.info()["n_coarse_faces"]
        X = torch.empty((n, 2 * b, b), dtype=torch.float32, device=self.device)
        V = torch.empty((n, 8, b), dtype=torch.float32, device=self.device)
        check(load().tgms_cnn_samples(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(V.data_ptr())))
        return X, V

    def eigs(self):
        import numpy as np
        n = self.info()["n_coarse_faces"]
        jm = max(self.bx, self.by) if self.dim == 2 else max(self.by * self.bz, self.bx * self.bz, self.bx * self.by)
        out = np.zeros((n, jm), dtype=np.float64)
        check(load().tgms_get_eigs(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def cond(self) -> float:
        c = ctypes.c_double(0.0)
        check(load().tgms_last_cond(self._h, ctypes.byref(c)))
        return c.value

    # ---- per-kernel event timing ------------------------------------------
    KERNELS = {"smoother": 0, "dir_apply": 1, "gather_restrict": 2, "coarse_prolong": 3}

    def profile(self, enable: bool = True):
        check(load().tgms_profile(self._h, 1 if enable else 0))

    def profile_get(self, kernel: str):
        n, t = ctypes.c_int(0), ctypes.c_double(0.0)
        check(load().tgms_profile_get(self._h, self.KERNELS[kernel], ctypes.byref(n), ctypes.byref(t)))
        return n.value, t.value

    def time_smoother(self, reps: int = 200) -> float:
        """Average duration (ms) of one smoother patch-solve launch over `reps`
        back-to-back launches bracketed by one HIP event pair."""
        ms = ctypes.c_double(0.0)
        check(load().tgms_time_smoother(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def time_dir_apply(self, reps: int = 200) -> float:
        """Average duration (ms) of one search-direction update with the operator apply
        (k_dir_apply) over `reps` back-to-back launches between one HIP event pair."""
        ms = ctypes.c_double(0.0)
        check(load().tgms_time_dir_apply(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    # ---- probes -----------------------------------------------------------
    def apply_A(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        check(load().tgms_apply_A(self._h, _ptr(x), _ptr(y)))
        return y

    def preprocess(self, F: torch.Tensor, g: torch.Tensor | None = None) -> torch.Tensor:
        v = torch.empty(self.nfaces, dtype=torch.float64, device=self.device)
        check(load().tgms_preprocess(self._h, _ptr(F.contiguous().reshape(-1)), _ptr(g), _ptr(v)))
        return v

    def apply_precond(self, which: str, r: torch.Tensor) -> torch.Tensor:
        z = torch.empty_like(r)
        check(load().tgms_apply_precond(self._h, {"smoother": 0, "coarse": 1, "twogrid": 2}[which], _ptr(r), _ptr(z)))
        return z

    def close(self):
        if getattr(self, "_h", None):
            load().tgms_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
