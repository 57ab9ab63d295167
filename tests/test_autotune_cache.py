"""The autotuner's JSON cache (llp_autotune_save / llp_autotune_load) on the
CPU: neither touches the GPU.  Records of any architecture round-trip; a
malformed or out-of-range file is rejected whole; llp_shutdown forgets every
record."""
import ctypes
import json
import os

import pytest

from conftest import ROOT

LIB = os.path.join(ROOT, "paper_2603_13147_amd", "libllp.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libllp.so not built")

ENTRIES = [
    {"arch": "gfx950", "cus": 256, "kind": "batch", "size_class": 13, "block": 512, "chunk": 1},
    {"arch": "gfx950", "cus": 256, "kind": "sssp", "size_class": 26, "block": 0, "chunk": 2},
    {"arch": "gfx942", "cus": 304, "kind": "bfs", "size_class": 20, "block": 0, "chunk": 3},
]


@pytest.fixture()
def lib():
    L = ctypes.CDLL(LIB)
    L.llp_last_error.restype = ctypes.c_char_p
    L.llp_autotune_save.argtypes = [ctypes.c_char_p]
    L.llp_autotune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
    L.llp_shutdown()
    yield L
    L.llp_shutdown()


def write(path, entries, head='"llp_autotune": 1'):
    with open(path, "w") as f:
        f.write("{%s, \"entries\": [\n" % head + ",\n".join(json.dumps(e) for e in entries) + "\n]}\n")


def load(L, path):
    n = ctypes.c_int32(-1)
    st = L.llp_autotune_load(os.fsencode(path), ctypes.byref(n))
    return st, n.value


def saved(L, path):
    assert L.llp_autotune_save(os.fsencode(path)) == 0, L.llp_last_error()
    with open(path) as f:
        return json.load(f)["entries"]


def key(e):
    return (e["arch"], e["cus"], e["kind"], e["size_class"])


def test_round_trip_keeps_every_architecture(lib, tmp_path):
    src, out = tmp_path / "a.json", tmp_path / "b.json"
    write(src, ENTRIES)
    assert load(lib, src) == (0, 3)
    got = saved(lib, out)
    assert sorted(got, key=key) == sorted(ENTRIES, key=key)
    assert not os.path.exists(str(out) + ".tmp")
    # loading the saved file again changes nothing; a later record of the same key replaces the earlier
    assert load(lib, out) == (0, 3)
    write(src, [dict(ENTRIES[1], chunk=4)])
    assert load(lib, src) == (0, 1)
    got = {key(e): e for e in saved(lib, out)}
    assert len(got) == 3 and got[key(ENTRIES[1])]["chunk"] == 4


def test_shutdown_forgets_records(lib, tmp_path):
    src, out = tmp_path / "a.json", tmp_path / "b.json"
    write(src, ENTRIES)
    assert load(lib, src) == (0, 3)
    lib.llp_shutdown()
    assert saved(lib, out) == []


@pytest.mark.parametrize("bad", [
    [dict(ENTRIES[0], block=100)],                       # batch block not a multiple of 64
    [dict(ENTRIES[1], chunk=5)],                         # graph workgroups per CU above the tuner's 4
    [dict(ENTRIES[1], block=256)],                       # graph records carry no block
    [dict(ENTRIES[0], kind="knapsack")],                 # kind the tuner does not record
    [dict(ENTRIES[0], size_class=63)],
    [{k: v for k, v in ENTRIES[0].items() if k != "cus"}],
    [ENTRIES[0], dict(ENTRIES[1], cus=0)],               # one bad entry rejects the file
    [dict(ENTRIES[0], arch="gfx950 x")],                 # architecture names are plain tokens
    [dict(ENTRIES[0], arch="g" * 65)],
])
def test_malformed_cache_is_rejected_whole(lib, tmp_path, bad):
    src, out = tmp_path / "bad.json", tmp_path / "b.json"
    write(src, bad)
    st, n = load(lib, src)
    assert st == 2 and n == 0   # LLP_E_INPUT
    assert saved(lib, out) == []


def test_missing_or_foreign_file(lib, tmp_path):
    st, n = load(lib, tmp_path / "none.json")
    assert st == 1 and n == 0   # LLP_E_ARG
    other = tmp_path / "other.json"
    other.write_text('{"something": []}')
    assert load(lib, other)[0] == 2
    assert lib.llp_autotune_save(b"") == 1
