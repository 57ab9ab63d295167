"""The seeded generators: splitmix64 against its published first output, stable
checksums, and the structural properties each workload recipe promises."""
import importlib.util
import os

import numpy as np

import llpgen
from conftest import GOLDEN, read_golden


def test_splitmix64_published_vector():
    # first output of splitmix64 seeded with 0 (Steele, Lea, Flood 2014 reference code)
    assert llpgen._load().llpgen_draw(0, 0) == 0xE220A8397B1DCDAF


def test_checksums_stable():
    spec = importlib.util.spec_from_file_location("mk", os.path.join(GOLDEN, "make_gen_checksums.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    want = {r[0]: r[1] for r in read_golden("gen_checksums.txt")}
    got = dict(mk.cases())
    assert got == want


def test_uniform_recipe():
    g = llpgen.uniform_graph(4096, 32768, 1, 100, seed=1)
    assert g.m == 36864
    assert not np.any(g.src == g.dst)
    assert g.w.min() >= 1 and g.w.max() <= 100
    assert np.array_equal(g.src[32768:], np.arange(4096))
    assert np.array_equal(g.dst[32768:], (np.arange(4096) + 1) % 4096)


def test_rmat_recipe():
    g = llpgen.rmat_graph(12, seed=5)
    n = 4096
    assert g.m == n * 16 + n
    assert g.src.min() >= 0 and g.src.max() < n
    assert g.w.min() >= 1 and g.w.max() <= 255
    deg = np.bincount(g.src[: n * 16], minlength=n)
    assert deg.max() > 20 * deg.mean()        # power-law hub
    nr = llpgen.rmat_graph(12, seed=5, relabel=False, cycle=False)
    # without relabelling vertex 0 (all-zero bits, prob a+b per source bit) is the hub
    assert np.argmax(np.bincount(nr.src, minlength=n)) == 0


def test_grid_recipe():
    g = llpgen.grid_graph(3, 4, seed=1)
    assert g.m == 2 * (3 * 3 + 2 * 4)
    pairs = set(zip(g.src.tolist(), g.dst.tolist()))
    for u, v in list(pairs):
        assert (v, u) in pairs
        ru, cu, rv, cv = u // 4, u % 4, v // 4, v % 4
        assert abs(ru - rv) + abs(cu - cv) == 1


def test_sm_recipe():
    mp, wr = llpgen.sm_prefs(64, seed=2)
    for i in range(64):
        assert sorted(mp[i].tolist()) == list(range(64))
        assert sorted(wr[i].tolist()) == list(range(64))


def test_dag_recipe():
    pp, pi, du = llpgen.job_dag(20000, seed=4)
    child = np.repeat(np.arange(20000), np.diff(pp))
    assert np.all(pi < child)                    # parents precede children
    assert abs(np.diff(pp)[100:].mean() - 8.0) < 0.2
    for j in range(0, 20000, 997):
        seg = pi[pp[j]:pp[j + 1]]
        assert len(set(seg.tolist())) == len(seg)
    assert du.min() >= 1 and du.max() <= 1000


def test_knapsack_recipe():
    for i in range(50):
        wt, val, W = llpgen.knapsack(i, seed=5)
        assert 16 <= len(wt) <= 256 and 256 <= W <= 4096
        assert wt.min() >= 1 and wt.max() <= W // 4
        assert val.min() >= 1 and val.max() <= 1000
