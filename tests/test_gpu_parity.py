"""Parity of the HIP path with the FP64 oracle (needs an MI355X).

Every test compares the library's result with the oracle's on the same
seeded inputs.  Sizes span several coarse blocks and patches, square and
non-square blocks, boundary-clipped patches and nonzero boundary data.
"""
import numpy as np
import pytest

from workloads import configs, fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from gpu_util import dev, eig_bound, host, oracle_for, register, rel  # noqa: E402

# Probe tolerances follow the conditioning of the local and coarse problems:
# two backward-stable solvers of the same system agree to about eps * cond.
# At contrast <= 1e3 that is below 1e-11; at contrast 1e6 the coarse and
# block problems reach cond ~ 1e6 after equilibration, hence 1e-8 there.
# The final velocity and pressure are held to 1e-10 in every case.
PROBE_TOL = {"cfg32": 1e-11, "rect36x24": 1e-11, "chan64": 1e-8, "odd35x21": 1e-11, "b16_128": 2e-9,
             "b16_96x64": 2e-9}

CASES = {
    # name: (nx, ny, bx, by, kappa generator, tol)
    "cfg32": (32, 32, 8, 8, lambda: configs.get("darcy2d_32_b8").make_inputs()[0], 0.5),
    "rect36x24": (36, 24, 6, 4, lambda: np.exp(2.0 * np.random.default_rng(7).standard_normal((24, 36))), 0.5),
    "chan64": (64, 64, 8, 8, lambda: fields.field_channelized(64, 64, 11, contrast=1e6), 2.0),
    # block and patch widths without a fixed-width kernel instantiation (generic paths)
    "odd35x21": (35, 21, 7, 7, lambda: np.exp(1.5 * np.random.default_rng(11).standard_normal((21, 35))), 0.5),
    # the 16 x 16-block kernels of the 256^2 and 1024^2 workloads (interior patches 20 x 20,
    # clipped 18 x 20 and 18 x 18) at contrast 1e6 and their tolerance 0.2: square and
    # non-square grids of blocks
    "b16_128": (128, 128, 16, 16, lambda: fields.field_channelized(128, 128, 19, contrast=1e6), 0.2),
    # (the paper's tolerance 10 here: Cond 9.6 instead of 2e4 at 0.2)
    "b16_96x64": (96, 64, 16, 16, lambda: fields.field_channelized(96, 64, 13, contrast=1e6), 10.0),
}


def case(name, precision="fp64"):
    import paper_1807_07220_amd as tg
    nx, ny, bx, by, gen, tol = CASES[name]
    kappa = gen()
    register(name, kappa)
    s = tg.Solver(dev(kappa), bx, by, tol, precision=precision)
    o = oracle_for(nx, ny, bx, by, name, tol)
    return s, o, kappa


@pytest.mark.parametrize("name", list(CASES))
def test_apply_A(name):
    s, o, _ = case(name)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(o.g.nf) * o.mask
    y = host(s.apply_A(dev(x)))
    assert rel(y, o.apply_A(x)) < 1e-14


@pytest.mark.parametrize("name", list(CASES))
def test_counts_and_eigenvalues(name):
    s, o, kappa = case(name)
    counts = s.counts()
    eigs = s.eigs()
    tol = CASES[name][5]
    near = np.array([np.any(np.abs(e - tol) <= 1e-8 * tol) for e in o.eigs])
    assert np.array_equal(counts[~near], o.counts[~near])
    for k, e in enumerate(o.eigs):
        J = e.size
        bound = eig_bound(kappa, CASES[name][2], CASES[name][3], e)
        assert np.all(np.abs(eigs[k, :J] - e) <= bound * e), (k, eigs[k, :J], e)
    info = s.info()
    assert info["dim"] == o.dim


@pytest.mark.parametrize("name", list(CASES))
def test_preprocessing(name):
    s, o, _ = case(name)
    F = fields.random_source(o.g.nx, o.g.ny, 5).ravel()
    vb = host(s.preprocess(dev(F)))
    vo, _, _ = o.preprocess(F)
    print(f"preprocess {name}: rel {rel(vb, vo):.2e}")
    assert rel(vb, vo) < PROBE_TOL[name]
    assert np.abs(o.B @ vb - F).max() < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("which", ["smoother", "coarse", "twogrid"])
def test_preconditioner(name, which):
    s, o, _ = case(name)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(o.g.nf) * o.mask
    z = host(s.apply_precond(which, dev(r)))
    ref = {"smoother": o.smooth, "coarse": o.coarse, "twogrid": o.twogrid}[which](r)
    print(f"{which} {name}: rel {rel(z, ref):.2e}")
    assert rel(z, ref) < PROBE_TOL[name]


@pytest.mark.parametrize("name", ["chan64", "b16_128", "b16_96x64"])
@pytest.mark.parametrize("which", ["smoother", "coarse", "twogrid"])
def test_preconditioner_fp32(name, which):
    """The FP32 preconditioner (factors, coarse basis and inverse in FP32; the residuals
    between its steps formed in FP64) against the FP64 oracle."""
    s, o, _ = case(name, precision="mixed")
    rng = np.random.default_rng(2)
    r = rng.standard_normal(o.g.nf) * o.mask
    z = host(s.apply_precond(which, dev(r)))
    ref = {"smoother": o.smooth, "coarse": o.coarse, "twogrid": o.twogrid}[which](r)
    print(f"fp32 {which} {name}: rel {rel(z, ref):.2e}")
    # bar: about 1700 FP32 unit roundoffs (6e-8), 25 times the largest difference
    # measured here (4e-6, the FP32 coarse solve of the 96 x 64 grid at tolerance 0.2);
    # the end-to-end FP32 solutions are held to 1e-8 (test_mixed_precision_error and
    # the full-size tests)
    assert rel(z, ref) < 1e-4


@pytest.mark.parametrize("name", list(CASES))
def test_solve(name):
    """Setup + solve against the oracle: iterations to rtol 1e-8 within one where the
    preconditioned system is well conditioned (Cond < 1e4; at the 128^2 grid's Cond 4.5e5
    the count moves with rounding-level differences of the coarse solve: 99 against 104
    with the GPU's coarse correction inside the oracle's own PCG), and at rtol 1e-12 on both sides the velocity in the energy norm (the
    kappa^{-1}-weighted L2 norm the method controls) and the pressure within 1e-10; the
    velocity's 2-norm, dominated at contrast 1e6 by channel faces that the energy norm
    weights by 1e-6, within ten times the oracle iterate's own distance to the direct
    solve of the full saddle system (the attainable FP64 accuracy) where that is larger."""
    from oracle.solver import exact_solve
    s, o, kappa = case(name)
    F = fields.corner_source(o.g.nx, o.g.ny).ravel()
    res = s.solve(dev(F), rtol=1e-8)
    ro = o.solve(F, rtol=1e-8)
    print(f"solve {name}: iters gpu {res['iters']} oracle {ro['iters']}, cond {ro['cond']:.3g}")
    assert res["converged"]
    if ro["cond"] < 1e4:
        assert abs(res["iters"] - ro["iters"]) <= 1
    res = s.solve(dev(F), rtol=1e-12, maxit=2000)
    ro = o.solve(F, rtol=1e-12, maxit=2000)
    ue, pe = exact_solve(o.g, kappa, F)
    floor_u = np.linalg.norm(ro["u"] - ue) / np.linalg.norm(ue)
    floor_p = np.linalg.norm(ro["p"] - pe) / np.linalg.norm(pe)
    du = host(res["u"]) - ro["u"]
    eu = np.linalg.norm(du) / np.linalg.norm(ro["u"])
    ea = np.sqrt(du @ (o.A @ du)) / np.sqrt(ro["u"] @ (o.A @ ro["u"]))
    ep = np.linalg.norm(host(res["p"]) - ro["p"]) / np.linalg.norm(ro["p"])
    print(f"solve {name} at rtol 1e-12: u err {eu:.2e} (oracle vs direct {floor_u:.2e}), energy norm {ea:.2e}, "
          f"p err {ep:.2e} (oracle vs direct {floor_p:.2e})")
    assert ea <= 1e-10 and ep <= max(1e-10, 2 * floor_p)
    assert eu <= max(1e-10, 10 * floor_u)


def test_solve_with_boundary_data():
    s, o, _ = case("rect36x24")
    g = o.g
    rng = np.random.default_rng(3)
    gf = np.zeros(g.nf)
    gf[g.boundary_idx] = rng.standard_normal(g.boundary_idx.size)
    F = fields.random_source(g.nx, g.ny, 4).ravel() + (o.B @ gf).sum() / g.nc
    res = s.solve(dev(F), dev(gf), rtol=1e-10)
    ro = o.solve(F, gf, rtol=1e-10)
    assert abs(res["iters"] - ro["iters"]) <= 1
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])
    assert np.linalg.norm(host(res["p"]) - ro["p"]) <= 1e-10 * np.linalg.norm(ro["p"])


@pytest.mark.parametrize("name", ["cfg32", "chan64"])
def test_mixed_precision_error(name):
    s, o, _ = case(name, precision="mixed")
    F = fields.corner_source(o.g.nx, o.g.ny).ravel()
    res = s.solve(dev(F), rtol=1e-10)
    ro = o.solve(F, rtol=1e-10)
    assert res["converged"]
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-8 * np.linalg.norm(ro["u"])
    assert np.linalg.norm(host(res["p"]) - ro["p"]) <= 1e-8 * np.linalg.norm(ro["p"])


def test_error_paths():
    import paper_1807_07220_amd as tg
    kappa = np.ones((32, 32))
    kappa[3, 4] = 0.0
    with pytest.raises(tg.TgmsError) as e:
        tg.Solver(dev(kappa), 8, 8, 0.5)
    assert e.value.status == "INVAL"
    with pytest.raises(tg.TgmsError) as e:
        tg.Solver(dev(np.ones((30, 32))), 8, 8, 0.5)
    assert e.value.status == "INVAL"
    s = tg.Solver(dev(np.ones((32, 32))), 8, 8, 0.5)
    F = np.zeros((32, 32))
    F[0, 0] = 1.0
    with pytest.raises(tg.TgmsError) as e:
        s.solve(dev(F))
    assert e.value.status == "INCOMPAT"
    F[5, 7] = -1.0
    res = s.solve(dev(F), maxit=1, rtol=1e-14)
    assert not res["converged"] and res["iters"] == 1
    res = s.solve(dev(np.zeros((32, 32))))
    assert res["converged"] and res["iters"] == 0
    assert float(res["u"].abs().max()) == 0.0


def test_solve_256_full_oracle():
    """The 256x256 / 16x16-block workload (tolerance 0.2, contrast 1e6): full solve vs oracle."""
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    w = configs.get("darcy2d_256_b16")
    kappa, F = w.make_inputs()
    s = tg.Solver(dev(kappa), w.bx, w.by, w.eig_tol)
    res = s.solve(dev(F), rtol=w.rtol)
    o = OracleSolver(Grid2D(w.nx, w.ny, w.bx, w.by), kappa, w.eig_tol)
    assert np.array_equal(s.counts(), o.counts)
    ro = o.solve(F.ravel(), rtol=w.rtol, maxit=1000)
    eu = np.linalg.norm(host(res["u"]) - ro["u"]) / np.linalg.norm(ro["u"])
    ep = np.linalg.norm(host(res["p"]) - ro["p"]) / np.linalg.norm(ro["p"])
    print(f"256x256: iters gpu {res['iters']} oracle {ro['iters']}, cond {ro['cond']:.3g}, "
          f"u err {eu:.3e}, p err {ep:.3e}, relres gpu {res['relres']:.3e} oracle {ro['relres']:.3e}")
    print("oracle relres tail", np.array(ro["hist"][-8:]))
    assert res["converged"]
    # Iteration parity: +-1 where the preconditioned system is well conditioned (every
    # other case).  Here Cond ~7e5, and the count is sensitive to rounding in the local
    # solves: the GPU smoother differs from the exact (refined) local solves by ~3e-11
    # relative (FP64 conditioning of the patch problems at contrast 1e6), and the oracle
    # itself, with its smoother output perturbed by random relative noise of that size,
    # needs 174, 175, 175 and 176 iterations (four seeds).  The bound is that spread.
    assert abs(res["iters"] - ro["iters"]) <= (1 if ro["cond"] < 1e4 else 2)
    # At Cond ~7e5 a 1e-10 difference between the two preconditioners (the coarse and
    # local problems' conditioning at contrast 1e6) grows over ~170 iterations, so at
    # rtol 1e-8 the two iterates agree to the rtol level only ...
    assert eu <= 3e-8 and ep <= 3e-8
    # ... and the iterative solution converges to the discrete solution: against the direct
    # solve of the full saddle system the error is bounded by Cond * rtol (PCG error bound).
    from oracle.solver import exact_solve
    ue, pe = exact_solve(Grid2D(w.nx, w.ny, w.bx, w.by), kappa, F.ravel())
    for rt in (1e-8, 1e-12):
        res = s.solve(dev(F), rtol=rt, maxit=2000)
        eu = np.linalg.norm(host(res["u"]) - ue) / np.linalg.norm(ue)
        ep = np.linalg.norm(host(res["p"]) - pe) / np.linalg.norm(pe)
        print(f"256x256 at rtol {rt:g}: iters {res['iters']}, u err vs direct {eu:.3e}, p err {ep:.3e}")
        assert eu <= ro["cond"] * rt and ep <= ro["cond"] * rt


def test_graph_replay_matches_eager():
    """Two PCG iterations are captured once as a HIP graph and replayed; repeated solves
    through the graph must match a context that launches every kernel directly, and a
    profiled solve (direct launches, four iterations queued per check) must count the
    launches of exactly the iterations that ran."""
    import paper_1807_07220_amd as tg
    s, o, kappa = case("chan64")
    F = fields.corner_source(o.g.nx, o.g.ny).ravel()
    r_graph = [s.solve(dev(F), rtol=1e-10) for _ in range(3)]
    assert s.info()["pcg_graph"] == 1
    s.profile(True)
    r_prof = s.solve(dev(F), rtol=1e-10)
    assert s.info()["pcg_graph"] == 0
    n, t = s.profile_get("smoother")
    s.profile(False)
    assert n == 2 * r_prof["iters"] + 2 and t > 0.0  # two per iteration and two for z_0
    r_again = s.solve(dev(F), rtol=1e-10)
    assert s.info()["pcg_graph"] == 1
    e = tg.Solver(dev(kappa), o.g.bx, o.g.by, CASES["chan64"][5], graphs=False)
    r_eager = e.solve(dev(F), rtol=1e-10)
    assert e.info()["pcg_graph"] == 0
    for r in r_graph + [r_prof, r_again]:
        assert r["iters"] == r_eager["iters"]
        assert rel(host(r["u"]), host(r_eager["u"])) < 1e-13


def test_setup_and_solve_deterministic():
    """Two setups and solves of the same input give bitwise identical results (no atomics
    in the assembly, fixed-order reductions)."""
    import paper_1807_07220_amd as tg
    w = configs.get("darcy2d_256_b16")
    kappa, F = w.make_inputs()
    outs = []
    for _ in range(2):
        s = tg.Solver(dev(kappa), w.bx, w.by, w.eig_tol)
        r = s.solve(dev(F), rtol=w.rtol)
        outs.append((r["iters"], host(r["u"]), host(r["p"])))
        s.close()
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("name", ["rect36x24", "chan64"])
def test_mobility_update(name):
    """Mobility update with the coarse space kept: the library and the oracle rebuild
    the same operator, smoother and coarse problem, and give the same solve."""
    from oracle import Grid2D, OracleSolver
    s, _, kappa = case(name)
    nx, ny, bx, by, _, tol = CASES[name]
    o = OracleSolver(Grid2D(nx, ny, bx, by), kappa, tol)  # a fresh oracle: it is modified
    lam = fields.mobility_front(nx, ny, 0.7).ravel()
    s.update_mobility(dev(lam.reshape(ny, nx)))
    o.update_mobility(lam)
    assert np.array_equal(s.counts(), o.counts)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(o.g.nf) * o.mask
    for which, ref in (("smoother", o.smooth), ("coarse", o.coarse), ("twogrid", o.twogrid)):
        z = host(s.apply_precond(which, dev(r)))
        assert rel(z, ref(r)) < PROBE_TOL[name], which
    F = fields.corner_source(nx, ny).ravel()
    res = s.solve(dev(F), rtol=1e-10)
    ro = o.solve(F, rtol=1e-10)
    assert res["converged"] and abs(res["iters"] - ro["iters"]) <= 1
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])
    assert np.linalg.norm(host(res["p"]) - ro["p"]) <= 1e-10 * np.linalg.norm(ro["p"])


def test_mobility_update_unit_is_identity():
    """lambda = 1 rebuilds the same factors: the solve is bitwise unchanged; an
    invalid mobility is rejected."""
    s, o, _ = case("cfg32")
    F = dev(fields.corner_source(32, 32))
    r0 = s.solve(F, rtol=1e-10)
    s.update_mobility(dev(np.ones((32, 32))))
    r1 = s.solve(F, rtol=1e-10)
    assert r1["iters"] == r0["iters"]
    assert torch.equal(r1["u"], r0["u"]) and torch.equal(r1["p"], r0["p"])
    import paper_1807_07220_amd as tg
    bad = np.ones((32, 32))
    bad[3, 4] = -1.0
    with pytest.raises(tg.TgmsError):
        s.update_mobility(dev(bad))
    s.update_mobility(dev(np.ones((32, 32))))
    r2 = s.solve(F, rtol=1e-10)
    assert torch.equal(r2["u"], r0["u"])


def test_autotune_cache(tmp_path):
    """The autotuner times the candidate launch configurations once per shape, keeps
    them in the cache file, and later setups of the shape take them from there; the
    tuned solver still matches the oracle."""
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    nx, ny, bx, by = 40, 24, 8, 8
    kappa = np.exp(np.random.default_rng(21).standard_normal((ny, nx)))
    cache = tmp_path / "tune.txt"
    s1 = tg.Solver(dev(kappa), bx, by, 0.5, tune_cache=str(cache))
    i1 = s1.info()
    assert i1["tuned"] in (1, 2) and i1["nred"] in (64, 128, 256, 512, 1024) and i1["smooth_staged"] in (0, 1)
    assert i1["rows_per_thread"] in (1, 4)
    text = cache.read_text()
    assert "40x24/b8x8" in text
    s2 = tg.Solver(dev(kappa), bx, by, 0.5, tune_cache=str(cache))
    i2 = s2.info()
    assert i2["tuned"] == 2 and i2["nred"] == i1["nred"] and i2["smooth_staged"] == i1["smooth_staged"]
    assert i2["rows_per_thread"] == i1["rows_per_thread"]
    s0 = tg.Solver(dev(kappa), bx, by, 0.5, autotune=False)
    assert s0.info()["tuned"] == 0
    o = OracleSolver(Grid2D(nx, ny, bx, by), kappa, 0.5)
    F = fields.corner_source(nx, ny).ravel()
    ro = o.solve(F, rtol=1e-10)
    for s in (s1, s2, s0):
        r = s.solve(dev(F), rtol=1e-10)
        assert abs(r["iters"] - ro["iters"]) <= 1
        assert np.linalg.norm(host(r["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])


@pytest.mark.parametrize("staging,rpt", [(0, 1), (1, 1), (0, 4), (1, 4)])
def test_launch_variants_match_oracle(staging, rpt):
    """Every launch variant the autotuner can pick (smoother blocks staged in LDS by the
    forward and again by the backward chains, or kept there between them; one or four
    vertex rows per thread in the tiled PCG kernels) gives the oracle's preconditioner
    and solution."""
    import paper_1807_07220_amd as tg
    nx, ny, bx, by, gen, tol = CASES["chan64"]
    kappa = gen()
    register("chan64", kappa)
    o = oracle_for(nx, ny, bx, by, "chan64", tol)
    s = tg.Solver(dev(kappa), bx, by, tol, autotune=False, smoother_staging=staging, rows_per_thread=rpt)
    inf = s.info()
    assert inf["smooth_staged"] == staging and inf["rows_per_thread"] == rpt
    r = np.random.default_rng(3).standard_normal(o.g.nf) * o.mask
    for which in ("smoother", "twogrid"):
        z = host(s.apply_precond(which, dev(r)))
        zo = o.smooth(r) if which == "smoother" else o.twogrid(r)
        assert rel(z * o.mask, zo) <= PROBE_TOL["chan64"]
    F = fields.corner_source(nx, ny).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10), o.solve(F, rtol=1e-10)
    assert abs(res["iters"] - ro["iters"]) <= 1
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])
    s.close()


def test_largest_blocks_many_modes():
    """The largest blocks the local band factors take (20 x 20 cells) with many modes per
    face (tol 50): the per-block coarse assembly at its largest LDS footprint (the
    centre block holds up to 80 coarse unknowns); counts, the two-grid operator and the
    solution match the oracle's."""
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    nx = ny = 60
    bx = by = 20
    kappa = fields.field_channelized(nx, ny, 23, contrast=1e4)
    o = OracleSolver(Grid2D(nx, ny, bx, by), kappa, 50.0)
    s = tg.Solver(dev(kappa), bx, by, 50.0)
    assert np.array_equal(s.counts(), np.asarray(o.counts))
    r = np.random.default_rng(5).standard_normal(o.g.nf) * o.mask
    z = host(s.apply_precond("twogrid", dev(r)))
    assert rel(z * o.mask, o.twogrid(r)) <= 1e-9
    F = fields.random_source(nx, ny, 9).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10), o.solve(F, rtol=1e-10)
    assert abs(res["iters"] - ro["iters"]) <= 1
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_overlap_one_matches_oracle(precision):
    """Overlap 1 (patch widths without a fixed-width smoother kernel) against the
    oracle with the same overlap; mixed precision takes the flexible update."""
    import paper_1807_07220_amd as tg
    from oracle import Grid2D, OracleSolver
    nx, ny, bx, by = 48, 40, 8, 8
    kappa = fields.field_channelized(nx, ny, 17, contrast=1e4)
    o = OracleSolver(Grid2D(nx, ny, bx, by), kappa, 1.0, overlap=1)
    s = tg.Solver(dev(kappa), bx, by, 1.0, overlap=1, precision=precision)
    F = fields.random_source(nx, ny, 5).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10), o.solve(F, rtol=1e-10)
    assert res["converged"] and ro["iters"] > 20
    if precision == "fp64":
        r = np.random.default_rng(4).standard_normal(o.g.nf) * o.mask
        z = host(s.apply_precond("twogrid", dev(r)))
        assert rel(z * o.mask, o.twogrid(r)) <= 1e-9
        assert abs(res["iters"] - ro["iters"]) <= 1
        assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-10 * np.linalg.norm(ro["u"])
    else:
        assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-8 * np.linalg.norm(ro["u"])
    s.close()


def test_overlap_zero_rejected():
    import paper_1807_07220_amd as tg
    with pytest.raises(tg.TgmsError):
        tg.Solver(dev(np.ones((32, 32))), 8, 8, 0.5, overlap=0)


@pytest.mark.parametrize("staging", [0, 1])
def test_mixed_smoother_modes_match_oracle(staging):
    """The FP32 smoother in either staging mode keeps the mixed-precision solution
    within 1e-8 of the FP64 oracle's."""
    import paper_1807_07220_amd as tg
    nx, ny, bx, by, gen, tol = CASES["chan64"]
    kappa = gen()
    register("chan64", kappa)
    o = oracle_for(nx, ny, bx, by, "chan64", tol)
    s = tg.Solver(dev(kappa), bx, by, tol, precision="mixed", autotune=False, smoother_staging=staging)
    F = fields.corner_source(nx, ny).ravel()
    res, ro = s.solve(dev(F), rtol=1e-10), o.solve(F, rtol=1e-10)
    assert res["converged"]
    assert np.linalg.norm(host(res["u"]) - ro["u"]) <= 1e-8 * np.linalg.norm(ro["u"])
    s.close()
