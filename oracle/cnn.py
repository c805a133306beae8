"""Reference (FP64) of the learned warm start for the local spectral problems.

Test infrastructure only: imported by tests/, the smoke check and the CPU
baseline of the benchmark, never by the library.

The local spectral problem of section 4.2 (the generalized eigenproblem
S_i z = lambda A_i z on the snapshot space, after the diagonal scaling
T = D^{-1/2} S D^{-1/2} and mu = 1/lambda) needs, per coarse face E_i, only the
modes with lambda < tol (mu > 1/tol), and at least one.  Instead of a full
dense eigensolve, a block of k initial vectors is refined by Rayleigh-Ritz
subspace iteration on T and accepted only when the selected modes are certified
(see warm_eigensolve); otherwise the dense solve runs.

The initial vectors come from a DCT-II basis (exact for a homogeneous
permeability up to the end effects) or from a small convolutional network on
the permeability of omega_i = K1 u K2:

  input   X[h][w] = log10(kappa) / 3 on the cells of omega_i, rows h across E
          (H = 2 x block depth), columns w along E (W = J, one per fine face
          of E, in the order of the pencil's index);
  layers  four 3x3 convolutions with zero padding, channels 1 -> C -> C -> C
          -> 8, ReLU after the first three;
  output  the normalised DCT-II basis (see dct_start) plus the mean over the
          rows: 8 vectors of length J (the first k = min(8, J) are used); the
          network learns a correction to the homogeneous-medium start.

Training minimises, per sample, sum_c |y_c / |y_c| - s_c v_c|^2 over the first
k channels, where v_c are the eigenvectors of T for the k largest mu and
s_c = sign(y_c . v_c) (eigenvectors are fixed only up to sign), averaged over
the batch, with Adam.

Parameters are one flat array: for each layer the weights [cout][cin][3][3]
followed by the biases [cout].
"""
from __future__ import annotations

import numpy as np

KOUT = 8        # output channels (block size of the warm start, at most)
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
NORM_EPS = 1e-12  # added to |y_c|^2 before the square root


def layer_shapes(C: int):
    return [(C, 1), (C, C), (C, C), (KOUT, C)]


def nparams(C: int) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(C))


def unpack(theta: np.ndarray, C: int):
    out, o = [], 0
    for co, ci in layer_shapes(C):
        w = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((w, b))
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def init_params(C: int, seed: int = 0) -> np.ndarray:
    """He-normal weights (the last layer scaled by 0.1: the start is close to the DCT
    basis), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for li, (co, ci) in enumerate(layer_shapes(C)):
        scale = np.sqrt(2.0 / (ci * 9)) * (0.1 if li == 3 else 1.0)
        out.append((rng.standard_normal((co, ci, 3, 3)) * scale, np.zeros(co)))
    return pack(out)


def face_window(kappa: np.ndarray, bx: int, by: int, fid: int) -> np.ndarray:
    """Network input of coarse face fid (x-faces first, row by row, then y-faces).

    x-face between K(I-1, J) and K(I, J): rows run along x over the two blocks,
    columns along y.  y-face between K(I, J-1) and K(I, J): rows along y,
    columns along x."""
    ny, nx = kappa.shape
    Nx, Ny = nx // bx, ny // by
    nex = (Nx - 1) * Ny
    lk = np.log10(kappa) / 3.0
    if fid < nex:
        J, I = fid // (Nx - 1), fid % (Nx - 1) + 1
        return lk[J * by:(J + 1) * by, (I - 1) * bx:(I + 1) * bx].T.copy()
    f = fid - nex
    J, I = f // Nx + 1, f % Nx
    return lk[(J - 1) * by:(J + 1) * by, I * bx:(I + 1) * bx].copy()


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[o][h][w] = b[o] + sum_{c,di,dj} w[o][c][di][dj] x[c][h+di-1][w+dj-1],
    with x zero outside [0,H) x [0,W)."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], H, W)) + b[:, None, None]
    for di in range(3):
        for dj in range(3):
            y += np.einsum("oc,chw->ohw", w[:, :, di, dj], xp[:, di:di + H, dj:dj + W])
    return y


def conv3x3_backward(x, w, gy):
    """(dL/dx, dL/dw, dL/db) of conv3x3 given dL/dy."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for di in range(3):
        for dj in range(3):
            gw[:, :, di, dj] = np.einsum("ohw,chw->oc", gy, xp[:, di:di + H, dj:dj + W])
            gxp[:, di:di + H, dj:dj + W] += np.einsum("oc,ohw->chw", w[:, :, di, dj], gy)
    return gxp[:, 1:-1, 1:-1], gw, gy.sum(axis=(1, 2))


def dct_unit(W: int) -> np.ndarray:
    """The first 8 DCT-II columns of length W, unit norm, as rows [8][W] (rows
    beyond W are zero)."""
    D = np.zeros((KOUT, W))
    k = min(KOUT, W)
    B = dct_start(W, k)
    D[:k] = (B / np.linalg.norm(B, axis=0)).T
    return D


def forward(theta: np.ndarray, C: int, x: np.ndarray):
    """x [H][W] -> (y [8][W], cache of (layer input, pre-activation) per layer)."""
    a = x[None, :, :]
    cache = []
    for li, (w, b) in enumerate(unpack(theta, C)):
        z = conv3x3(a, w, b)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if li < 3 else z
    return dct_unit(x.shape[1]) + a.mean(axis=1), cache


def sample_loss(y: np.ndarray, v: np.ndarray, k: int):
    """Loss of one sample and dL/dy; v [k][W] are the target eigenvectors (unit norm)."""
    L = 0.0
    gy = np.zeros_like(y)
    for c in range(k):
        n = np.sqrt(y[c] @ y[c] + NORM_EPS)
        u = y[c] / n
        s = 1.0 if u @ v[c] >= 0 else -1.0
        d = u - s * v[c]
        L += d @ d
        # u = y/n: du/dy = (I - u u^T)/n (up to the eps), so dL/dy = 2 (d - u (u.d)) / n
        gy[c] = (2.0 / n) * (d - u * (u @ d))
    return L, gy


def backward(theta: np.ndarray, C: int, cache, gy_out: np.ndarray) -> np.ndarray:
    """Flat gradient of the loss w.r.t. theta given dL/dy [8][W]."""
    H = cache[0][0].shape[1]
    params = unpack(theta, C)
    g = np.repeat(gy_out[:, None, :] / H, H, axis=1)  # through the mean over rows
    grads = [None] * 4
    for li in range(3, -1, -1):
        a, z = cache[li]
        if li < 3:
            g = g * (z > 0)
        gx, gw, gb = conv3x3_backward(a, params[li][0], g)
        grads[li] = (gw, gb)
        g = gx
    return pack(grads)


def batch_loss_grad(theta, C, X, V, k):
    """Mean loss and gradient over a batch: X [B][H][W], V [B][k][W]."""
    L, G = 0.0, np.zeros_like(theta)
    for x, v in zip(X, V):
        y, cache = forward(theta, C, x)
        l, gy = sample_loss(y, v, k)
        L += l
        G += backward(theta, C, cache, gy)
    return L / len(X), G / len(X)


def adam_step(theta, m, v, g, t: int, lr: float):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = ADAM_B1 * m + (1 - ADAM_B1) * g
    v = ADAM_B2 * v + (1 - ADAM_B2) * g * g
    mh = m / (1 - ADAM_B1 ** t)
    vh = v / (1 - ADAM_B2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


def dct_start(J: int, k: int) -> np.ndarray:
    """J x k DCT-II basis: column c is cos(pi (l + 1/2) c / J)."""
    l = np.arange(J)[:, None] + 0.5
    return np.cos(np.pi * l * np.arange(k)[None, :] / J)


def inertia_count_above(T: np.ndarray, sigma: float):
    """Number of eigenvalues of the symmetric T above sigma: the number of negative
    pivots of the LDL^T factorisation of sigma I - T without pivoting (Sylvester's
    law of inertia); None when a pivot is (relatively) zero."""
    A = sigma * np.eye(T.shape[0]) - T
    scale = np.abs(A).max()
    neg = 0
    for j in range(A.shape[0]):
        d = A[j, j]
        if abs(d) <= 1e-14 * scale:
            return None
        neg += d < 0
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j] / d, A[j, j + 1:])
    return int(neg)


def warm_eigensolve(T: np.ndarray, Y0: np.ndarray, tol: float, rq_tol: float = 1e-6, max_it: int = 8):
    """Rayleigh-Ritz subspace iteration on T from the columns of Y0 (J x k).

    With cnt = the number of eigenvalues of T above sigma = 1/tol (inertia) and
    l = max(1, cnt) selected modes, a face is accepted at the first iteration
    where l < k, exactly cnt Ritz values exceed sigma, the first l Ritz pairs have
    |T u - theta u| / theta <= rq_tol, and, when cnt = 0, exactly one eigenvalue
    lies above theta_1 (1 - 4 rq_tol).  Returns (accepted, iteration, cnt,
    Ritz values descending (k), Ritz vectors J x k)."""
    J, k = Y0.shape
    sigma = 1.0 / tol
    cnt = inertia_count_above(T, sigma)
    if cnt is None or max(cnt, 1) >= k:
        return False, 0, cnt, None, None
    l = max(cnt, 1)
    X = Y0.astype(np.float64).copy()
    for it in range(max_it + 1):
        Q = np.zeros_like(X)  # modified Gram-Schmidt
        for c in range(k):
            q = X[:, c].copy()
            for p in range(c):
                q -= (Q[:, p] @ q) * Q[:, p]
            nq = np.linalg.norm(q)
            if nq <= 1e-12 * max(np.linalg.norm(X[:, c]), 1e-300):
                return False, it, cnt, None, None
            Q[:, c] = q / nq
        W = T @ Q
        Hm = Q.T @ W
        th, Z = np.linalg.eigh(0.5 * (Hm + Hm.T))
        th, Z = th[::-1], Z[:, ::-1]
        U, TU = Q @ Z, W @ Z
        res = np.linalg.norm(TU - U * th, axis=0) / np.abs(th)
        ok = int(np.sum(th > sigma)) == cnt and bool(np.all(res[:l] <= rq_tol))
        if ok and cnt == 0:
            ok = inertia_count_above(T, th[0] * (1.0 - 4.0 * rq_tol)) == 1
        if ok:
            return True, it, cnt, th, U
        X = TU
    return False, max_it, cnt, None, None
