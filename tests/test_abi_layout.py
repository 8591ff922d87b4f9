"""The binding's ctypes structures have the layout of the C ABI's structures:
a C program built with gcc from include/chebyprop.h prints the size of
every structure and the offset of every field the binding declares, and
both must agree with ctypes (a field the header lacks fails to compile, a
field the binding lacks changes the size)."""

import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_header(tmp_path):
    from paper_2412_10789_amd import chebyprop as cp

    structs = [cp.cp_query, cp.cp_info, cp.cp_graph_stats, cp.cp_server_stats]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "chebyprop.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            name, key, val = line.split()
            got[(name, key)] = int(val)
    for st in structs:
        name = st.__name__
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert got[(name, field)] == getattr(st, field).offset, (name, field)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_constants_match_header(tmp_path):
    """Every precision, kind, truncation-rule, query and graph flag constant
    of the binding has the header's value."""
    from paper_2412_10789_amd import chebyprop as cp

    names = ["CP_F64", "CP_F32", "CP_BF16", "CP_F32F", "CP_PPR", "CP_HKPR", "CP_K_CERTIFIED", "CP_K_TAIL",
             "CP_K_PAPER", "CP_K_FIXED", "CP_GRAPH_BORROW", "CP_GRAPH_VALIDATE", "CP_GRAPH_REORDER",
             "CP_GRAPH_HOST", "CP_GRAPH_XCD_STRIPES", "CP_GRAPH_HOT_SPLIT", "CP_Q_STATS", "CP_Q_TIMING",
             "CP_Q_PWMETHOD", "CP_Q_CLENSHAW"]
    lines = ['#include <stdio.h>', '#include "chebyprop.h"', "int main(void) {"]
    lines += [f'  printf("{n} %lld\\n", (long long)({n}));' for n in names]
    lines += ['  printf("CP_NOALLOC_SCRATCH_BYTES %zu\\n", CP_NOALLOC_SCRATCH_BYTES);', "  return 0;", "}"]
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for n in names + ["CP_NOALLOC_SCRATCH_BYTES"]:
        assert int(got[n]) == getattr(cp, n), n
    assert cp.PRECS == {"f64": cp.CP_F64, "f32": cp.CP_F32, "f32f": cp.CP_F32F, "bf16": cp.CP_BF16}
