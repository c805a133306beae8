"""The C-ABI library loads and exports every entry point declared in include/tgms.h (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgms.h")
LIB = os.path.join(ROOT, "paper_1807_07220_amd", "libtgms.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tgms_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_binding_signatures_cover_header():
    from paper_1807_07220_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_default_options_are_the_papers():
    from paper_1807_07220_amd import _lib
    lib = _lib.load()
    o = _lib.Options()
    lib.tgms_default_options(ctypes.byref(o))
    assert o.eta == 0.2 and o.overlap == 2 and o.precision == 0 and o.s_scale == 1.0
