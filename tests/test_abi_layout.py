"""The ctypes structures of the Python binding match the C layout of include/tgms.h (CPU only).

A small C program (gcc) prints sizeof and offsetof of every field of tgms_grid,
tgms_options, tgms_info_t and tgms_transport_params; the binding's ctypes structures must agree.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_struct_layouts_match_header():
    from paper_1807_07220_amd import _lib
    structs = {"tgms_grid": _lib.Grid, "tgms_options": _lib.Options, "tgms_info_t": _lib.Info,
               "tgms_transport_params": _lib.TransportParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tgms.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == _lib.ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
