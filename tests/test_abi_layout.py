"""The ctypes mirrors of the C-ABI structs (paper_1909_12533_amd/_lib.py) have
the layout the header declares: a small C program built with the host
compiler prints sizeof and offsetof of every field of include/sp2dm.h's
structs, compared field by field with ctypes."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_1909_12533_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [L.sp2_bsr, L.sp2_options, L.sp2_stats, L.sp2_step_info]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sp2dm.h"', "int main(void) {"]
    for S in STRUCTS:
        name = S.__name__
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return table


@pytest.mark.parametrize("S", STRUCTS, ids=lambda S: S.__name__)
def test_ctypes_mirror_matches_header(c_layout, S):
    name = S.__name__
    assert C.sizeof(S) == c_layout[(name, "sizeof")]
    for f, _ in S._fields_:
        assert getattr(S, f).offset == c_layout[(name, f)], f"{name}.{f}"
