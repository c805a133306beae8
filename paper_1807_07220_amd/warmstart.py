"""Learned warm start for the local spectral problems: training and inference helpers.

The network and its training step run in the HIP library (tgms_cnn_* in
include/tgms.h); this module only marshals arguments, gathers training samples
from set-up solvers and keeps the parameters in a .npy file.

Typical use::

    X, V = collect_samples(fields, b=16, eig_tol=0.2)       # exact setups
    w = train(X, V, k=8, steps=2000)                         # Adam on the GPU
    save_weights("warmstart.npy", w)
    s = Solver(kappa, 16, 16, 0.2, warm_start="cnn", cnn_weights=w)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, load


def nparams() -> int:
    return load().tgms_cnn_nparams()


def _fptr(t: torch.Tensor):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def init_weights(seed: int = 0, device="cuda:0", C: int = 16, kout: int = 8) -> torch.Tensor:
    """He-normal weights (the last layer scaled by 0.1, so that the output starts
    near the DCT basis) and zero biases in the library's flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (co, ci) in enumerate([(C, 1), (C, C), (C, C), (kout, C)]):
        parts.append(rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (ci * 9)) * (0.1 if li == 3 else 1.0))
        parts.append(np.zeros(co))
    w = np.concatenate(parts).astype(np.float32)
    if w.size != nparams():
        raise RuntimeError("parameter layout differs from the library's")
    return torch.tensor(w, device=device)


def forward(w: torch.Tensor, X: torch.Tensor, bf16: bool = False) -> torch.Tensor:
    """Network outputs [n][8][W] for inputs X [n][H][W] (float32, GPU); bf16: the
    inference form on the BF16 matrix cores that the warm start uses."""
    n, H, W = X.shape
    X = X.contiguous()
    Y = torch.empty((n, 8, W), dtype=torch.float32, device=X.device)
    stream = torch.cuda.current_stream(X.device).cuda_stream
    fn = load().tgms_cnn_infer if bf16 else load().tgms_cnn_forward
    check(fn(_fptr(w), _fptr(X), n, H, W, _fptr(Y), ctypes.c_void_p(stream)))
    return Y


class Trainer:
    """Adam state and workspace for training steps of one batch shape."""

    def __init__(self, w: torch.Tensor, batch: int, H: int, W: int):
        self.w = w
        self.m = torch.zeros_like(w)
        self.v = torch.zeros_like(w)
        self.t = 0
        self.batch, self.H, self.W = batch, H, W
        nwork = load().tgms_cnn_train_workspace(batch, H, W)
        if nwork == 0:
            raise ValueError("unsupported shape")
        self.work = torch.empty(nwork, dtype=torch.float32, device=w.device)

    def step(self, X: torch.Tensor, V: torch.Tensor, k: int, lr: float) -> float:
        n = X.shape[0]
        if n > self.batch or X.shape[1:] != (self.H, self.W):
            raise ValueError("batch larger than the workspace or a different shape")
        self.t += 1
        loss = ctypes.c_double(0.0)
        stream = torch.cuda.current_stream(X.device).cuda_stream
        check(load().tgms_cnn_train_step(_fptr(self.w), _fptr(self.m), _fptr(self.v), self.t, float(lr),
                                         _fptr(X.contiguous()), _fptr(V.contiguous()), n, self.H, self.W, int(k),
                                         _fptr(self.work), ctypes.byref(loss), ctypes.c_void_p(stream)))
        return loss.value


def collect_samples(fields, b: int, eig_tol: float, device="cuda:0"):
    """Inputs and targets of every interior coarse face of each permeability field
    (exact setups with b x b blocks); returns (X [N][2b][b], V [N][8][b]) on the GPU."""
    from . import Solver
    Xs, Vs = [], []
    for kappa in fields:
        kd = torch.as_tensor(np.ascontiguousarray(kappa), dtype=torch.float64, device=device)
        s = Solver(kd, b, b, eig_tol)
        X, V = s.cnn_samples()
        s.close()
        Xs.append(X)
        Vs.append(V)
    return torch.cat(Xs), torch.cat(Vs)


def train(X: torch.Tensor, V: torch.Tensor, k: int = 8, steps: int = 2000, batch: int = 512, lr: float = 2e-3,
          seed: int = 0, w: torch.Tensor | None = None, log=None):
    """Adam on random mini-batches; the learning rate decays by cosine to lr/20.
    Returns the weights and the per-step losses."""
    n, H, W = X.shape
    if w is None:
        w = init_weights(seed, device=X.device)
    tr = Trainer(w, min(batch, n), H, W)
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (tr.batch,), generator=g).to(X.device)
        a = lr * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * it / max(steps - 1, 1))))
        losses.append(tr.step(X[idx], V[idx], k, a))
        if log and (it % 200 == 0 or it == steps - 1):
            log(f"step {it} loss {losses[-1]:.4f}")
    return tr.w, losses


def save_weights(path: str, w: torch.Tensor):
    np.save(path, w.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load_weights(path: str, device="cuda:0") -> torch.Tensor:
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.ndim != 1 or w.size != nparams():
        raise ValueError(f"{path}: not a warm-start weight vector of {nparams()} float32 values")
    return torch.tensor(w, device=device)
