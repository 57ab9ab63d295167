"""The ctypes mirrors of the C ABI's structs (llp_stats, llp_trace_rec,
llp_opts, llp_graph, llp_instance) have the header's size and field offsets:
a small C program built against include/llp.h prints them (no GPU)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2603_13147_amd as llp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [("llp_stats", llp.Stats), ("llp_trace_rec", llp.TraceRec), ("llp_opts", llp.Opts),
         ("llp_graph", llp.Graph), ("llp_instance", llp.Instance)]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "llp.h"', "int main(void) {"]
    for cname, py in PAIRS:
        lines.append(f'    printf("{cname} __sizeof__ %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.parametrize("cname,py", PAIRS, ids=[c for c, _ in PAIRS])
def test_struct_layout(c_layout, cname, py):
    assert c_layout[(cname, "__sizeof__")] == ctypes.sizeof(py)
    for field, _ in py._fields_:
        assert c_layout[(cname, field)] == getattr(py, field).offset, field


def test_trace_dtype_matches_record():
    assert llp.TRACE_DTYPE.itemsize == ctypes.sizeof(llp.TraceRec)
    for field, _ in llp.TraceRec._fields_:
        assert llp.TRACE_DTYPE.fields[field][1] == getattr(llp.TraceRec, field).offset
