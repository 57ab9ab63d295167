"""The C ABI library loads on the CPU and exports every entry point that
include/llp.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "llp.h")
LIB = os.path.join(ROOT, "paper_2603_13147_amd", "libllp.so")



def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(llp_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_solvers():
    names = declared()
    for n in ["llp_solve_sssp", "llp_solve_bfs", "llp_solve_sm", "llp_solve_jobs", "llp_solve_knapsack",
              "llp_solve_batch", "llp_workspace_bytes", "llp_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libllp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libllp.so not built")
def test_host_side_calls_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.llp_version.restype = ctypes.c_char_p
    assert lib.llp_version().startswith(b"libllp")
    lib.llp_workspace_bytes.restype = ctypes.c_size_t
    lib.llp_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    assert lib.llp_workspace_bytes(1, 4096, 36864, None) > 4096 * 8
    # argument errors are reported before any device work
    lib.llp_solve_sssp.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.llp_solve_sssp(None, 0, None, None) == 1
    lib.llp_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.llp_last_error()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2603_13147_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "oracle/" not in text, f
