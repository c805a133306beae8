"""The allocation-free solve (tgms_solve_noalloc) against tgms_solve, through the C ABI
(needs an MI355X).  Two calls in a row, the second on a smaller grid: each must give
bitwise the results of tgms_solve on the same context (same kernels, same order of
operations), with the scratch array's leftovers of the first call cleared."""
import ctypes

import numpy as np
import pytest

from workloads import fields

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(lib, fn, h, F, nf, ncell, rtol, maxit):
    from paper_1807_07220_amd import _lib
    u = torch.full((nf,), np.nan, dtype=torch.float64, device="cuda:0")
    p = torch.full((ncell,), np.nan, dtype=torch.float64, device="cuda:0")
    it, rel = ctypes.c_int(-1), ctypes.c_double(-1.0)
    code = getattr(lib, fn)(h, ctypes.c_void_p(F.data_ptr()), None, rtol, maxit, ctypes.c_void_p(u.data_ptr()),
                            ctypes.c_void_p(p.data_ptr()), ctypes.byref(it), ctypes.byref(rel))
    torch.cuda.synchronize()
    return code, u, p, it.value, rel.value


def test_noalloc_solve_matches_solve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_07220_amd import _lib, nfaces
    lib = _lib.load()
    opt = _lib.Options()
    lib.tgms_default_options(ctypes.byref(opt))
    for n, b, tol, seed in ((64, 8, 2.0, 11), (32, 8, 0.5, 12)):  # the second call: a smaller input
        kappa = torch.tensor(fields.field_channelized(n, n, seed, contrast=1e6), device="cuda:0")
        F = torch.tensor(fields.corner_source(n, n), device="cuda:0").reshape(-1).contiguous()
        g = _lib.Grid(2, n, n, 1, b, b, 1)
        h = ctypes.c_void_p()
        assert lib.tgms_setup(ctypes.byref(g), ctypes.c_void_p(kappa.data_ptr()), tol, ctypes.byref(opt),
                              ctypes.byref(h)) == 0
        try:
            ref = _run(lib, "tgms_solve", h, F, nfaces(n, n), n * n, 1e-10, 500)
            got = _run(lib, "tgms_solve_noalloc", h, F, nfaces(n, n), n * n, 1e-10, 500)
            assert ref[0] == 0 and got[0] == 0
            assert got[3] == ref[3] and got[4] == ref[4]
            assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2])
            # sizes beyond the scratch array are refused, and the context still works
            code = _run(lib, "tgms_solve_noalloc", h, F, nfaces(n, n), n * n, 1e-10, 10 ** 6)[0]
            assert code == -1 and b"allocation-free" in lib.tgms_last_error()
            again = _run(lib, "tgms_solve", h, F, nfaces(n, n), n * n, 1e-10, 500)
            assert torch.equal(again[1], ref[1])
        finally:
            lib.tgms_destroy(h)
