"""The solver on the unit cube (needs an MI355X) against the 3D oracle (oracle/solver3d.py),
element by element on small seeded grids that span several blocks and patches, including
non-cubic blocks, overlap 1 and 2, and the three coarse spaces.

Bars (the same algorithm on both sides, rounding apart): basis counts equal, eigenvalues
to 1e-9 relative, operator and preconditioner probes to 1e-10 relative (in the 2-norm of
the output), PCG iteration counts within one, velocity and pressure to 1e-10 relative.
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]
torch = pytest.importorskip("torch")

from gpu_util import dev, host  # noqa: E402

CASES = {
    # name: (cells, block, overlap, eigen tolerance, log-permeability scale)
    "cube12_b4_ov2": ((12, 12, 12), (4, 4, 4), 2, 2.0, 2.0),
    "box15x12x9_b5x4x3_ov1": ((15, 12, 9), (5, 4, 3), 1, 2.0, 2.0),
    "box20x20x10_b5_ov2": ((20, 20, 10), (5, 5, 5), 2, 2.0, 3.0),
    # blocks one cell thick along z (no interior z-faces inside a block, one-cell lines)
    "thin12x12x4_b4x4x1_ov1": ((12, 12, 4), (4, 4, 1), 1, 2.0, 2.0),
    # two blocks per axis with overlap 3: every patch clipped on one side of each axis
    "two8x6x10_b4x3x5_ov3": ((8, 6, 10), (4, 3, 5), 3, 2.0, 2.0),
}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(name, seed=5):
    from oracle.grid3d import Grid3D
    dims, b, ov, tol, scale = CASES[name]
    g = Grid3D(*dims, *b)
    rng = np.random.default_rng(seed)
    kappa = np.exp(scale * rng.standard_normal(g.nc))
    F = np.zeros(g.nc)
    F[0], F[-1] = 1.0, -1.0
    return g, kappa, F, ov, tol


def _pair(name, basis="gmsfem"):
    import paper_1807_07220_amd as tg
    from oracle.solver3d import OracleSolver3D
    g, kappa, F, ov, tol = _inputs(name)
    o = OracleSolver3D(g, kappa, tol, overlap=ov, basis=basis)
    nx, ny, nz = g.n
    s = tg.Solver(dev(kappa.reshape(nz, ny, nx)), g.bx, g.by, tol, bz=g.bz, overlap=ov, coarse_space=basis)
    return g, kappa, F, o, s


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_operator_and_setup(name):
    """A x on the interior faces; basis counts and every eigenvalue of every face."""
    _need_gpu()
    g, kappa, F, o, s = _pair(name)
    try:
        x = np.random.default_rng(1).standard_normal(g.nf)
        y = host(s.apply_A(dev(x)))
        np.testing.assert_allclose(y, o.apply_A(x), rtol=0, atol=1e-12 * np.abs(o.apply_A(x)).max())
        counts = np.array(s.counts())
        np.testing.assert_array_equal(counts, o.counts)
        E = s.eigs()
        for i, lam in enumerate(o.eigs):
            np.testing.assert_allclose(E[i, :lam.size], lam, rtol=1e-9)
        assert s.info()["dim"] == o.dim
    finally:
        s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_preprocess_and_preconditioner(name):
    """vbar of section 3; smoother, coarse correction and two-grid cycle on a random
    residual (boundary entries zero)."""
    _need_gpu()
    g, kappa, F, o, s = _pair(name)
    try:
        vbar, _, _ = o.preprocess(F)
        got = host(s.preprocess(dev(F)))
        assert _rel(got, vbar) <= 1e-10
        r = np.random.default_rng(2).standard_normal(g.nf) * o.mask
        for which, fn in (("smoother", o.smooth), ("coarse", o.coarse), ("twogrid", o.twogrid)):
            z = host(s.apply_precond(which, dev(r)))
            ref = fn(r)
            print(f"{name} {which}: rel {_rel(z, ref):.2e}")
            assert _rel(z, ref) <= 1e-10, which
    finally:
        s.close()


@pytest.mark.parametrize("name,basis", [(n, "gmsfem") for n in CASES] +
                         [("cube12_b4_ov2", "msfem"), ("cube12_b4_ov2", "rt0"), ("box15x12x9_b5x4x3_ov1", "rt0")])
def test_solve(name, basis):
    _need_gpu()
    g, kappa, F, o, s = _pair(name, basis)
    try:
        ref = o.solve(F, rtol=1e-8)
        got = s.solve(dev(F), rtol=1e-8)
        eu, ep = _rel(host(got["u"]), ref["u"]), _rel(host(got["p"]), ref["p"])
        print(f"{name} {basis}: iterations {got['iters']} (oracle {ref['iters']}), u {eu:.2e}, p {ep:.2e}")
        assert got["converged"]
        assert abs(got["iters"] - ref["iters"]) <= 1
        assert eu <= 1e-10 and ep <= 1e-10
        # div u = F: the preprocessing meets it to round-off; each PCG correction is
        # divergence-free to about eps cond(S) of the local Schur complements (applied as
        # explicit inverses; the oracle's refined sparse LU reaches eps), so the bound is
        # relative to the largest sum of |flux| over a cell's faces and allows for the
        # conditioning at these contrasts (permeability ratio up to 1e9)
        uh = host(got["u"])
        scale = (abs(o.B) @ np.abs(uh)).max()
        derr = np.abs(o.B @ uh - F).max()
        print(f"  max |B u - F| {derr:.1e} (flux scale {scale:.2e})")
        assert derr <= 1e-9 * scale
    finally:
        s.close()


def test_update_mobility_keeps_the_basis():
    """Section 6.2 on the cube: the operator of lambda kappa over the initial basis."""
    _need_gpu()
    name = "cube12_b4_ov2"
    g, kappa, F, o, s = _pair(name)
    try:
        lam = np.exp(np.random.default_rng(7).uniform(-1.0, 1.0, g.nc))
        o.update_mobility(lam)
        s.update_mobility(dev(lam))
        ref = o.solve(F, rtol=1e-8)
        got = s.solve(dev(F), rtol=1e-8)
        assert abs(got["iters"] - ref["iters"]) <= 1
        assert _rel(host(got["u"]), ref["u"]) <= 1e-10
        assert np.array_equal(np.array(s.counts()), o.counts)
    finally:
        s.close()


def test_transport_and_impes_on_the_cube():
    """The cube's transport step against the oracle's (velocity from the oracle's direct
    solve), then the IMPES loop with the kept coarse space against the oracle's loop."""
    _need_gpu()
    import paper_1807_07220_amd as tg
    from oracle.solver3d import OracleSolver3D, exact_solve
    from oracle.transport import impes, transport_step
    g, kappa, F, ov, tol = _inputs("box20x20x10_b5_ov2")
    nx, ny, nz = g.n
    u, _ = exact_solve(g, kappa, F)
    s0 = np.zeros(g.nc)
    s_o, it_o = transport_step(g, u, F, s0, 0.002, max_newton=2000)
    s_g, outer, res = tg.transport_step(dev(u), dev(F), dev(s0.reshape(nz, ny, nx)), 0.002)
    err = np.abs(host(s_g).ravel() - s_o).max()
    print(f"cube transport: {outer} tile launches (oracle {it_o} Newton iterations), max diff {err:.2e}")
    assert err <= 2 * (nx + ny + nz) * 1e-12
    o = OracleSolver3D(g, kappa, tol, overlap=ov)
    s_ref, its = impes(o, F, np.zeros(g.nc), steps=4, dt=0.002, pressure_every=2, rtol=1e-10)
    sv = tg.Solver(dev(kappa.reshape(nz, ny, nx)), g.bx, g.by, tol, bz=g.bz, overlap=ov)
    try:
        r = sv.impes(dev(F), dev(np.zeros((nz, ny, nx))), steps=4, dt=0.002, pressure_every=2, rtol=1e-10)
    finally:
        sv.close()
    err = np.abs(host(r["s"]).ravel() - s_ref).max()
    print(f"cube IMPES: PCG {r['pcg_iters']} (oracle {its}), max |s diff| {err:.2e}")
    assert all(abs(a - b) <= 1 for a, b in zip(r["pcg_iters"], its))
    assert err <= 1e-7


def _eig_bound3(kappa, g, face, lam):
    """Relative tolerance of the eigenvalues lambda of one coarse face on the layered
    workloads (permeability ratios up to 1e8 within one block pair).  The snapshots come
    from the blocks' Schur complements applied as explicit inverses, accurate to about eps
    times their condition number, at most the local contrast times (largest block
    extent)^2 (a factor 100 of margin); the largest pencil eigenvalue carries that error,
    which reaches lambda_k as a relative eps lambda_k / lambda_min on top."""
    from oracle.solver3d import face_geometry
    eps = np.finfo(np.float64).eps
    K1, K2, _, _, _, _ = face_geometry(g, face)
    k = np.asarray(kappa).ravel()
    cells = np.concatenate([g.cells_in(*g.block_box(K1)), g.cells_in(*g.block_box(K2))])
    contrast = float(k[cells].max() / k[cells].min())
    base = 100.0 * eps * contrast * max(g.b) ** 2
    return max(base, 1e-12) + 100.0 * eps * lam / lam.min()


def _workload_solver(name):
    import paper_1807_07220_amd as tg
    from workloads import configs
    w = configs.get(name)
    kappa, F = w.make_inputs()
    s = tg.Solver(dev(kappa), w.bx, w.by, w.eig_tol, bz=w.bz)
    return w, kappa, F, s


def test_layered_workload_cut_matches_oracle():
    """The layered workload's 15 x 33 x 15 cut (3 x 3 x 3 blocks of 5 x 11 x 5 cells: the full
    workload's patch size 9 x 15 x 9 and faces of 55 and 25 fine faces) element by element."""
    _need_gpu()
    from oracle.grid3d import Grid3D
    from oracle.solver3d import OracleSolver3D
    w, kappa, F, s = _workload_solver("darcy3d_15x33x15_b5x11x5")
    try:
        g = Grid3D(w.nx, w.ny, w.nz, w.bx, w.by, w.bz)
        o = OracleSolver3D(g, kappa.ravel(), w.eig_tol)
        np.testing.assert_array_equal(np.array(s.counts()), o.counts)
        E = s.eigs()
        worst = 0.0
        for i, lam in enumerate(o.eigs):
            err = np.abs(E[i, :lam.size] - lam) / lam
            bound = _eig_bound3(kappa, g, g.coarse_faces()[i], lam)
            assert np.all(err <= bound), (i, err.max(), bound.min())
            worst = max(worst, err.max())
        print(f"15x33x15 cut: largest relative eigenvalue difference {worst:.1e}")
        ref = o.solve(F.ravel(), rtol=1e-8)
        got = s.solve(dev(F), rtol=1e-8)
        print(f"15x33x15 cut: Dim {s.info()['dim']} (oracle {o.dim}), iterations {got['iters']} "
              f"(oracle {ref['iters']})")
        assert abs(got["iters"] - ref["iters"]) <= 1
        # The permeability spans 1e8 here: at rtol 1e-8 the two iterates may differ in the
        # channels by up to ~rtol sqrt(contrast) in the 2-norm (the energy norm weighs them by
        # kappa^{-1}).  The solutions are compared at rtol 1e-12, in the energy norm to 1e-10,
        # and in the 2-norm to 1e-10 or twice the oracle iterate's own distance to the
        # direct solve, whichever is coarser.
        from oracle.solver3d import exact_solve
        ref = o.solve(F.ravel(), rtol=1e-12, maxit=1000)
        got = s.solve(dev(F), rtol=1e-12, maxit=1000)
        ue, pe = exact_solve(g, kappa.ravel(), F.ravel())
        uh, ph = host(got["u"]), host(got["p"])
        d = uh - ref["u"]
        ea = np.sqrt(d @ (o.A @ d)) / np.sqrt(ref["u"] @ (o.A @ ref["u"]))
        eu, ep = _rel(uh, ref["u"]), _rel(ph, ref["p"])
        fu, fp = _rel(ref["u"], ue), _rel(ref["p"], pe)
        print(f"  rtol 1e-12: u {eu:.2e} (energy {ea:.2e}, oracle vs direct {fu:.2e}), p {ep:.2e} (floor {fp:.2e})")
        assert ea <= 1e-10
        assert eu <= max(1e-10, 2 * fu) and ep <= max(1e-10, 2 * fp)
    finally:
        s.close()


def test_layered_workload_full_size():
    """60 x 220 x 85 cells (4080 blocks, 11456 coarse faces): the local spectral problems of
    sampled faces of every axis against the oracle's (its snapshots of the two blocks, its
    pencil, LAPACK), and the solve through properties that hold at any size: convergence,
    div u = F, and the projected residual P(A u) (zero for the exact discrete solution)
    small next to P(A vbar)."""
    _need_gpu()
    import scipy.linalg as sla
    from oracle.grid3d import Grid3D, div_matrix, mass_matrix
    from oracle.local import BorderedSaddle
    from oracle.solver3d import CellLaplacian, pencil, snapshots
    w, kappa, F, s = _workload_solver("darcy3d_60x220x85_b5x11x5")
    try:
        g = Grid3D(w.nx, w.ny, w.nz, w.bx, w.by, w.bz)
        kinv = 1.0 / kappa.ravel()
        A = mass_matrix(g, kinv).tocsr()
        B = div_matrix(g).tocsr()
        faces = g.coarse_faces()
        counts, E = np.array(s.counts()), s.eigs()
        rng = np.random.default_rng(3)
        axis_of = np.array([a for a, _ in faces])
        sample = np.concatenate([rng.choice(np.flatnonzero(axis_of == a), 4, replace=False) for a in range(3)])

        def block(I):
            lo, hi = g.block_box(I)
            return BorderedSaddle(A, B, g.faces_in(lo, hi), g.cells_in(lo, hi))

        for fid in sample:
            fa, Psi = snapshots(g, A, B, block, faces[fid])
            Dg, S = pencil(g, A, B, kinv, faces[fid], fa, Psi, 1.0)
            # the reference eigenvalues from the symmetric form T = D^{-1/2} S D^{-1/2} of the
            # oracle's pencil (LAPACK): its largest mu = 1/lambda_min are accurate to eps |T|,
            # while the generalised solver factors S, whose condition number reaches 1e6 here
            T = S / np.sqrt(np.outer(Dg, Dg))
            lam = np.sort(1.0 / sla.eigvalsh(0.5 * (T + T.T)))
            err = np.abs(E[fid, :lam.size] - lam) / lam
            bound = _eig_bound3(kappa, g, faces[fid], lam)
            k = int(np.argmax(err / bound))
            print(f"  face {fid} (axis {faces[fid][0]}): worst relative eigenvalue difference {err[k]:.1e} at "
                  f"lambda {lam[k]:.3e} (bound {bound[k]:.1e}, lambda_min {lam[0]:.2e})")
            assert np.all(err <= bound)
            if not np.any(np.abs(lam - w.eig_tol) <= 1e-8 * w.eig_tol):
                assert counts[fid] == max(1, int(np.count_nonzero(lam < w.eig_tol)))
        Fd = dev(F)
        vbar = host(s.preprocess(Fd))
        got = s.solve(Fd, rtol=1e-8)
        u = host(got["u"])
        print(f"60x220x85: Dim {s.info()['dim']}, iterations {got['iters']}, Cond {s.cond():.3g}")
        assert got["converged"]
        assert np.abs(B @ vbar - F.ravel()).max() <= 1e-12 * (abs(B) @ np.abs(vbar)).max()
        assert np.abs(B @ u - F.ravel()).max() <= 1e-9 * (abs(B) @ np.abs(u)).max()
        lap = CellLaplacian(g)
        mask = g.interior.astype(float)

        def proj(r):
            return mask * (r - B.T @ lap(B @ (mask * r)))

        ru, r0 = np.linalg.norm(proj(A @ u)), np.linalg.norm(proj(A @ vbar))
        print(f"  |P A u| / |P A vbar| = {ru / r0:.2e}")
        assert ru <= 1e-6 * r0
    finally:
        s.close()
