"""Pins of the warm-start oracle (oracle/cnn.py) against independent facts (CPU)."""
import numpy as np
from scipy.signal import correlate2d

from oracle import cnn
from oracle.discretization import Grid2D, div_matrix, mass_matrix
from oracle.local import BorderedSaddle
from oracle.spectral import block_rect, pencil, select, snapshots


def test_conv3x3_is_zero_padded_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 7, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(correlate2d(x[c], w[o, c], mode="same", boundary="fill") for c in range(3))
        assert np.allclose(y[o], ref, rtol=0, atol=1e-13)


def test_sample_loss_sign_and_scale_invariance():
    rng = np.random.default_rng(1)
    v = np.linalg.qr(rng.standard_normal((9, 3)))[0].T        # 3 unit rows
    y = np.zeros((cnn.KOUT, 9))
    y[:3] = np.array([2.5, -0.3, 7.0])[:, None] * v             # scaled, one flipped
    L, g = cnn.sample_loss(y, v, 3)
    assert L < 1e-20 and np.abs(g).max() < 1e-9
    y[0] = np.linalg.qr(np.column_stack([v[0], rng.standard_normal(9)]))[0][:, 1]  # orthogonal to v[0]
    L, _ = cnn.sample_loss(y, v, 1)
    assert abs(L - 2.0) < 1e-10                                  # |u|^2 + |v|^2 with u.v = 0


def _fd_check(f, theta, idx, h=1e-6):
    out = []
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        out.append((f(theta + e) - f(theta - e)) / (2 * h))
    return np.array(out)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    C, H, W, k = 4, 6, 5, 3
    theta = cnn.init_params(C, seed=3)
    theta[-cnn.KOUT:] = rng.standard_normal(cnn.KOUT)           # nonzero output biases
    X = rng.standard_normal((2, H, W))
    V = np.stack([np.linalg.qr(rng.standard_normal((W, k)))[0].T for _ in range(2)])
    L, G = cnn.batch_loss_grad(theta, C, X, V, k)
    idx = rng.choice(theta.size, 40, replace=False)
    fd = _fd_check(lambda t: cnn.batch_loss_grad(t, C, X, V, k)[0], theta, idx)
    assert np.allclose(G[idx], fd, rtol=1e-5, atol=1e-8)
    # every layer's weights and biases receive gradient
    o = 0
    for co, ci in cnn.layer_shapes(C):
        n = co * ci * 9 + co
        assert np.abs(G[o:o + n]).max() > 0
        o += n
    assert o == cnn.nparams(C) == theta.size


def test_zero_network_gives_the_dct_start():
    theta = cnn.init_params(4, seed=0)
    o = sum(co * ci * 9 + co for co, ci in cnn.layer_shapes(4)[:3])
    theta[o:] = 0.0                                     # last layer: zero weights and biases
    x = np.random.default_rng(0).standard_normal((6, 11))
    y, _ = cnn.forward(theta, 4, x)
    D = cnn.dct_start(11, 8)
    assert np.allclose(y, (D / np.linalg.norm(D, axis=0)).T, atol=1e-15)
    y3, _ = cnn.forward(theta, 4, x[:, :3])            # W < 8: the rows beyond W are zero
    assert np.all(y3[3:] == 0.0) and np.allclose(np.linalg.norm(y3[:3], axis=1), 1.0)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = cnn.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01)
    # bias-corrected moments are g and g^2 after one step
    assert np.allclose(th, -0.01 * g / (np.abs(g) + cnn.ADAM_EPS), rtol=1e-14)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_dct_columns_orthogonal():
    D = cnn.dct_start(16, 8)
    Gm = D.T @ D
    assert np.allclose(Gm - np.diag(np.diag(Gm)), 0.0, atol=1e-12)
    assert np.allclose(np.diag(Gm)[1:], 8.0) and abs(Gm[0, 0] - 16.0) < 1e-12


def test_inertia_count_matches_spectrum():
    rng = np.random.default_rng(4)
    for J in (5, 16, 33):
        mu = np.exp(rng.uniform(-3, 3, J))
        Q = np.linalg.qr(rng.standard_normal((J, J)))[0]
        T = (Q * mu) @ Q.T
        for sigma in (0.3, 1.0, 7.0):
            assert cnn.inertia_count_above(T, sigma) == int(np.sum(mu > sigma))


def _spd(rng, mu):
    Q = np.linalg.qr(rng.standard_normal((len(mu), len(mu))))[0]
    return (Q * mu) @ Q.T, Q


def test_warm_eigensolve_recovers_top_modes():
    rng = np.random.default_rng(5)
    mu = np.array([40.0, 9.0, 0.9, 0.5, 0.4, 0.3, 0.2, 0.15, 0.1, 0.08, 0.05, 0.04])
    T, Q = _spd(rng, mu)
    ok, it, cnt, th, U = cnn.warm_eigensolve(T, rng.standard_normal((12, 6)), tol=0.2)
    assert ok and cnt == 2
    assert np.allclose(th[:2], mu[:2], rtol=1e-10)
    for c in range(2):   # eigenvector up to sign
        assert abs(abs(U[:, c] @ Q[:, c]) - 1.0) < 1e-10
    # started on the exact eigenvectors: accepted at once
    ok, it, *_ = cnn.warm_eigensolve(T, Q[:, :6], tol=0.2)
    assert ok and it == 0


def test_warm_eigensolve_certification_rejects_missed_mode():
    rng = np.random.default_rng(6)
    mu = np.array([40.0, 9.0, 0.9, 0.5, 0.4, 0.3, 0.2, 0.15, 0.1, 0.08])
    T, Q = _spd(rng, mu)
    # a block inside the invariant subspace without the top mode never sees it
    for tol in (0.05, 0.2):     # cnt = 1 (mu > 20) and cnt = 2 (mu > 5)
        ok, *_ = cnn.warm_eigensolve(T, Q[:, 1:6], tol=tol)
        assert not ok
    # too many modes for the block: refused
    ok, *_ = cnn.warm_eigensolve(T, rng.standard_normal((10, 3)), tol=3.0)   # cnt = 3 >= k
    assert not ok
    # cnt = 0 keeps the top mode, certified by the count just below theta_1
    mu0 = mu / 100.0
    T0, Q0 = _spd(rng, mu0)
    ok, it, cnt, th, U = cnn.warm_eigensolve(T0, rng.standard_normal((10, 5)), tol=0.2)
    assert ok and cnt == 0 and abs(th[0] - mu0[0]) < 1e-10 * mu0[0]
    ok, *_ = cnn.warm_eigensolve(T0, Q0[:, 1:6], tol=0.2)
    assert not ok


def _face_T(kappa, bx, by, face):
    ny, nx = kappa.shape
    g = Grid2D(nx, ny, bx, by)
    kinv = (1.0 / kappa).ravel()
    A, B = mass_matrix(g, kinv).tocsr(), div_matrix(g).tocsr()

    def block(I, J):
        r = block_rect(g, I, J)
        return BorderedSaddle(A, B, g.faces_in(*r), g.cells_in(*r))
    fa, Psi = snapshots(g, A, B, block, face)
    Dg, S = pencil(g, A, B, kinv, face, fa, Psi)
    d = 1.0 / np.sqrt(Dg)
    return d[:, None] * S * d[None, :], Dg, S


def test_dct_start_exact_for_homogeneous_face():
    T, *_ = _face_T(np.ones((8, 16)), 8, 8, ("x", 1, 0))
    mu, V = np.linalg.eigh(T)
    C = cnn.dct_start(8, 8)
    C /= np.linalg.norm(C, axis=0)
    assert np.allclose(np.abs(np.sum(C * V[:, ::-1], axis=0)), 1.0, atol=1e-8)


def test_warm_eigensolve_matches_dense_selection_on_a_face():
    rng = np.random.default_rng(7)
    kappa = np.exp(2.0 * rng.standard_normal((8, 16)))
    T, Dg, S = _face_T(kappa, 8, 8, ("x", 1, 0))
    lam, Vd, count = select(Dg, S, 0.5)
    ok, it, cnt, th, U = cnn.warm_eigensolve(T, cnn.dct_start(8, 8), tol=0.5)
    assert ok and max(cnt, 1) == count
    assert np.allclose(1.0 / th[:count], lam[:count], rtol=1e-9)
    # same modes: D^{-1/2} U spans the generalized eigenvectors
    Z = U[:, :count] / np.sqrt(Dg)[:, None]
    P = Vd[:, :count]
    cosines = np.linalg.svd(np.linalg.qr(Z)[0].T @ np.linalg.qr(P)[0], compute_uv=False)
    assert np.all(cosines > 1 - 1e-9)


def test_face_window_orientation():
    nx, ny, bx, by = 12, 8, 4, 4
    jj, ii = np.mgrid[0:ny, 0:nx]
    code = lambda i, j: (i + 16.0 * j) / 64.0                  # noqa: E731
    kappa = 10.0 ** (3.0 * code(ii, jj))                       # log10(kappa)/3 = code(i, j)
    # x-face between K(0,1) and K(1,1) (fid = J*(Nx-1) + I-1 = 1*2 + 0)
    X = cnn.face_window(kappa, bx, by, 2)
    assert X.shape == (2 * bx, by)
    assert np.isclose(X[0, 0], code(0, 4)) and np.isclose(X[7, 0], code(7, 4)) and np.isclose(X[0, 3], code(0, 7))
    # y-face between K(2,0) and K(2,1): fid = nex + (J-1)*Nx + I = 4 + 0 + 2
    Y = cnn.face_window(kappa, bx, by, 6)
    assert Y.shape == (2 * by, bx)
    assert np.isclose(Y[0, 0], code(8, 0)) and np.isclose(Y[7, 0], code(8, 7)) and np.isclose(Y[0, 3], code(11, 0))
