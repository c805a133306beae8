"""The C-ABI calls around setup and solve (needs an MI355X): checkpoint and restore of
the setup, the pencil probe, imposed basis counts, the comparator coarse spaces
(MsFEM, RT0) and the grid's dimension check, each against the oracle or bitwise
against the context it came from."""
import ctypes

import numpy as np
import pytest

from workloads import configs, fields

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from gpu_util import dev, host, oracle_face, rel  # noqa: E402

CASES = {
    # name: (kappa, bx, by, tol)
    "cfg32": (lambda: configs.get("darcy2d_32_b8").make_inputs()[0], 8, 8, 0.5),
    "chan64": (lambda: fields.field_channelized(64, 64, 11, contrast=1e6), 8, 8, 2.0),
    "b16_96x64": (lambda: fields.field_channelized(96, 64, 13, contrast=1e6), 16, 16, 0.2),
}


def _oracle(kappa, bx, by, tol, **kw):
    from oracle import Grid2D, OracleSolver
    ny, nx = kappa.shape
    return OracleSolver(Grid2D(nx, ny, bx, by), kappa, tol, **kw)


@pytest.mark.parametrize("name", ["cfg32", "chan64"])
def test_save_load_solves_bitwise(name, tmp_path):
    """tgms_save / tgms_load: the restored context (coarse space read back, not solved
    for) solves bitwise as the saved one, also after a mobility update."""
    import paper_1807_07220_amd as tg
    gen, bx, by, tol = CASES[name]
    kappa = gen()
    ny, nx = kappa.shape
    F = dev(fields.corner_source(nx, ny))
    s = tg.Solver(dev(kappa), bx, by, tol, autotune=False)
    r0 = s.solve(F, rtol=1e-10)
    path = str(tmp_path / "ctx.tgms")
    s.save(path)
    t = tg.Solver.load(path, autotune=False)
    assert (t.nx, t.ny, t.bx, t.by) == (nx, ny, bx, by)
    assert np.array_equal(t.counts(), s.counts()) and np.array_equal(t.eigs(), s.eigs())
    r1 = t.solve(F, rtol=1e-10)
    assert r1["iters"] == r0["iters"]
    assert torch.equal(r1["u"], r0["u"]) and torch.equal(r1["p"], r0["p"])
    lam = dev(fields.mobility_front(nx, ny, 0.6))
    s.update_mobility(lam)
    r2 = s.solve(F, rtol=1e-10)
    s.save(path)
    t2 = tg.Solver.load(path, autotune=False)
    r3 = t2.solve(F, rtol=1e-10)
    assert r3["iters"] == r2["iters"] and torch.equal(r3["u"], r2["u"]) and torch.equal(r3["p"], r2["p"])
    for x in (s, t, t2):
        x.close()


def test_load_rejects_bad_files(tmp_path):
    import paper_1807_07220_amd as tg
    bad = tmp_path / "bad.tgms"
    bad.write_bytes(b"not a context")
    for p in (str(bad), str(tmp_path / "missing.tgms")):
        with pytest.raises(tg.TgmsError) as e:
            tg.Solver.load(p)
        assert e.value.status == "INVAL"
    # a truncated file
    s = tg.Solver(dev(np.ones((32, 32))), 8, 8, 0.5, autotune=False)
    good = tmp_path / "good.tgms"
    s.save(str(good))
    data = good.read_bytes()
    cut = tmp_path / "cut.tgms"
    cut.write_bytes(data[: len(data) // 2])
    with pytest.raises(tg.TgmsError) as e:
        tg.Solver.load(str(cut))
    assert e.value.status == "INVAL"


@pytest.mark.parametrize("name", ["cfg32", "b16_96x64"])
def test_pencil_probe_matches_oracle(name):
    """Each face's pencil (D, S) against the oracle's pencil() on sampled faces: D to
    round-off; S in the norm of T = D^{-1/2} S D^{-1/2} to the accuracy of the snapshot
    solves (eps times the local condition number, as for the eigenvalues)."""
    import paper_1807_07220_amd as tg
    gen, bx, by, tol = CASES[name]
    kappa = gen()
    s = tg.Solver(dev(kappa), bx, by, tol, autotune=False)
    D, S = s.probe_pencil()
    D, S = host(D), host(S)
    n = s.info()["n_coarse_faces"]
    ny, nx = kappa.shape
    nex = (nx // bx - 1) * (ny // by)
    contrast = kappa.max() / kappa.min()
    worst = 0.0
    for fid in sorted(set(np.random.default_rng(0).choice(n, size=min(n, 10), replace=False)) | {0, n - 1}):
        T, Do, So = oracle_face(kappa, bx, by, fid)
        J = Do.size
        assert J == (by if fid < nex else bx)
        assert np.abs(D[fid, :J] - Do).max() <= 1e-15 * np.abs(Do).max()
        d = 1.0 / np.sqrt(Do)
        Tg = d[:, None] * S[fid, :J, :J] * d[None, :]
        err = np.linalg.norm(Tg - T) / np.linalg.norm(T)
        worst = max(worst, err)
        assert np.all(S[fid, J:, :] == 0) and np.all(S[fid, :, J:] == 0)
    print(f"pencil {name}: worst relative T difference {worst:.2e}")
    eps = np.finfo(np.float64).eps
    assert worst <= max(1e-12, 100 * eps * contrast * max(bx, by) ** 2)


def test_forced_counts_match_oracle():
    """Imposed counts (one more mode than the threshold keeps, on every face) give the
    oracle's coarse correction and solve with the same imposed counts."""
    import paper_1807_07220_amd as tg
    gen, bx, by, tol = CASES["chan64"]
    kappa = gen()
    o0 = _oracle(kappa, bx, by, tol)
    force = np.minimum(o0.counts + 1, [e.size for e in o0.eigs]).astype(np.int32)
    o = _oracle(kappa, bx, by, tol, force_counts=force)
    s = tg.Solver(dev(kappa), bx, by, tol, force_counts=force)
    assert np.array_equal(s.counts(), force) and s.info()["dim"] == o.dim
    r = np.random.default_rng(6).standard_normal(o.g.nf) * o.mask
    assert rel(host(s.apply_precond("coarse", dev(r))), o.coarse(r)) < 1e-8
    F = fields.corner_source(64, 64).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10), o.solve(F, rtol=1e-10)
    assert abs(res["iters"] - ro["iters"]) <= 1
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])
    with pytest.raises(tg.TgmsError):
        tg.Solver(dev(kappa), bx, by, tol, force_counts=np.zeros_like(force))


@pytest.mark.parametrize("space", ["msfem", "rt0"])
@pytest.mark.parametrize("name", ["cfg32", "chan64"])
def test_comparator_coarse_spaces_match_oracle(space, name):
    """The paper's comparators (section 6): the same two-grid preconditioner with the
    MsFEM or coarse RT0 space, against the oracle with the same basis."""
    import paper_1807_07220_amd as tg
    gen, bx, by, tol = CASES[name]
    kappa = gen()
    o = _oracle(kappa, bx, by, tol, basis=space)
    s = tg.Solver(dev(kappa), bx, by, tol, coarse_space=space)
    assert s.info()["coarse_space"] == {"msfem": 1, "rt0": 2}[space]
    assert s.info()["dim"] == o.dim
    r = np.random.default_rng(7).standard_normal(o.g.nf) * o.mask
    for which, ref in (("coarse", o.coarse), ("twogrid", o.twogrid)):
        z = host(s.apply_precond(which, dev(r)))
        assert rel(z, ref(r)) < 1e-8, which
    F = fields.corner_source(o.g.nx, o.g.ny).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10, maxit=2000), o.solve(F, rtol=1e-10, maxit=2000)
    print(f"{space} {name}: iters gpu {res['iters']} oracle {ro['iters']}")
    assert res["converged"] and abs(res["iters"] - ro["iters"]) <= 1
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])


def test_grid_dimension_checked():
    from paper_1807_07220_amd import _lib
    lib = _lib.load()
    kappa = dev(np.ones((32, 32)))
    kappa3 = dev(np.ones((4, 32, 32)))
    opt = _lib.Options()
    lib.tgms_default_options(ctypes.byref(opt))
    h = ctypes.c_void_p()
    # dimensions other than 2 and 3, and cubes whose sizes the blocks do not divide or that
    # have fewer than 2 blocks on an axis, are refused before any kernel reads kappa
    for grid, k, status in (((1, 32, 32, 4, 8, 8, 2), kappa, -1), ((4, 32, 32, 4, 8, 8, 2), kappa, -1),
                            ((3, 32, 32, 4, 8, 8, 3), kappa3, -1), ((3, 32, 32, 4, 8, 8, 4), kappa3, -7)):
        g = _lib.Grid(*grid)
        code = lib.tgms_setup(ctypes.byref(g), ctypes.c_void_p(k.data_ptr()), 0.5, ctypes.byref(opt),
                              ctypes.byref(h))
        assert code == status and not h.value, (grid, code)
    g = _lib.Grid(2, 32, 32, 1, 8, 8, 1)
    assert lib.tgms_setup(ctypes.byref(g), ctypes.c_void_p(kappa.data_ptr()), 0.5, ctypes.byref(opt),
                          ctypes.byref(h)) == 0
    inf = _lib.Info()
    assert lib.tgms_info(h, ctypes.byref(inf)) == 0 and inf.eig_unconverged == 0
    lib.tgms_destroy(h)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["cfg32", "chan64", "b16_96x64"])
def test_cyclic_reduction_coarse_factor_matches_oracle(name, precision):
    """The block cyclic-reduction Cholesky of the coarse systems (forced here also where
    the dense inverse would be chosen by size) against the oracle's direct solves: the
    coarse correction and the preprocessing (its coarse RT0 system), and the solve."""
    import paper_1807_07220_amd as tg
    gen, bx, by, tol = CASES[name]
    kappa = gen()
    o = _oracle(kappa, bx, by, tol)
    s = tg.Solver(dev(kappa), bx, by, tol, precision=precision, coarse_factor="bcr")
    inf = s.info()
    assert inf["coarse_block"] > 0 and inf["rt0_block"] == o.g.Nx
    r = np.random.default_rng(8).standard_normal(o.g.nf) * o.mask
    zc = host(s.apply_precond("coarse", dev(r)))
    ec = rel(zc, o.coarse(r))
    F = fields.random_source(o.g.nx, o.g.ny, 5).ravel()
    ev = rel(host(s.preprocess(dev(F))), o.preprocess(F)[0])
    Fc = fields.corner_source(o.g.nx, o.g.ny).ravel()
    res, ro = s.solve(dev(Fc), rtol=1e-10), o.solve(Fc, rtol=1e-10)
    du = host(res["u"]) - ro["u"]
    eu = np.sqrt(du @ (o.A @ du)) / np.sqrt(ro["u"] @ (o.A @ ro["u"]))  # energy norm
    print(f"bcr {name} {precision}: block {inf['coarse_block']}, coarse {ec:.2e}, preprocess {ev:.2e}, "
          f"iters {res['iters']} / {ro['iters']}, u {eu:.2e}")
    assert ev < 1e-8
    if precision == "fp64":
        assert ec < 1e-8 and abs(res["iters"] - ro["iters"]) <= 1 and eu <= 1e-10
    else:
        assert ec < 1e-4 and eu <= 1e-8
