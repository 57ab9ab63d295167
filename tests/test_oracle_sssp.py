"""Pins of the SSSP / BFS oracle (Section 5.2, Section 5.3) against values the
paper prints, library shortest paths, brute force and invariants."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra, shortest_path

import llpgen
import oracle
from oracle.schedules import INF, relax_arc, sssp_pull_async, sssp_push_bag_interleaved
from conftest import read_golden

I32 = oracle.INF32


def _worked_example():
    rows = read_golden("sssp_worked_example.txt")
    edges = {r[1]: (int(r[2]), int(r[3]), int(r[4])) for r in rows if r[0] == "edge"}
    final = [int(x) for r in rows if r[0] == "final" for x in r[1:]]
    paths = [r[1:] for r in rows if r[0] == "path"]
    return edges, final, paths


def _undirected(edges):
    src, dst, w = [], [], []
    for (u, v, ww) in edges.values():
        src += [u, v]; dst += [v, u]; w += [ww, ww]
    return np.array(src), np.array(dst), np.array(w)


def test_worked_example_fixpoint():
    edges, final, _ = _worked_example()
    src, dst, w = _undirected(edges)
    for bag in (False, True):
        assert oracle.sssp(4, src, dst, w, 0, bag=bag).tolist() == final


def test_worked_example_lattice_paths():
    """Single-edge relaxations in the edge orders of Figure 3 visit exactly the
    printed intermediate states and end at C_F."""
    edges, final, paths = _worked_example()
    for p in paths:
        sep = p.index(":")
        labels, states = p[:sep], p[sep + 1:]
        d = [0, INF, INF, INF]
        for lab, st in zip(labels, states):
            u, v, ww = edges[lab]
            # an undirected edge relaxes whichever endpoint it improves
            d2 = relax_arc(d, u, v, ww)
            if d2 == d:
                d2 = relax_arc(d, v, u, ww)
            d = d2
            want = [INF if x == "inf" else int(x) for x in st.split("=")[1].split(",")]
            assert d == want, (p, lab)
        assert d == final


def test_race_example_join_vs_overwrite():
    rows = {r[0]: r[1:] for r in read_golden("race_examples.txt")}
    edges, _, _ = _worked_example()
    arcs = []
    for (u, v, w) in edges.values():
        arcs += [(u, v, w), (v, u, w)]
    state = [INF if x == "inf" else int(x) for x in rows["sssp_state"]]
    bag = [(0, 3, 3), (2, 3, 3)]          # T1 via edge b, T2 via edge d
    store = sssp_push_bag_interleaved(4, arcs, 0, apply="store", init_state=state, init_bag=bag)
    join = sssp_push_bag_interleaved(4, arcs, 0, apply="join", init_state=state, init_bag=bag)
    assert store[3] == int(rows["sssp_overwrite"][0])
    assert join[3] == int(rows["sssp_correct"][0])
    join_rev = sssp_push_bag_interleaved(4, arcs, 0, apply="join", init_state=state, init_bag=bag[::-1])
    assert join_rev[3] == int(rows["sssp_correct"][0])


def test_bfs_race_example():
    rows = {r[0]: r[1:] for r in read_golden("race_examples.txt")}
    a = [int(x) for x in rows["bfs_arcs"]]
    src, dst = a[0::2], a[1::2]
    lev = oracle.bfs(4, src, dst, 0)
    assert lev[3] == int(rows["bfs_correct_level3"][0])
    arcs = [(u, v, 1) for u, v in zip(src, dst)]
    # T1 relaxes 3 from 0, T2 from 2 (level 1) using the stale read level(3) = inf
    store = sssp_push_bag_interleaved(4, arcs, 0, apply="store", init_state=[0, INF, 1, INF],
                                      init_bag=[(0, 3, 1), (2, 3, 1)])
    assert store[3] == int(rows["bfs_overwrite_level3"][0])


def _scipy_dist(n, src, dst, w, s, unweighted=False):
    A = sp.coo_matrix((np.ones(len(src)) if unweighted else np.asarray(w, np.float64),
                       (src, dst)), shape=(n, n)).tocsr()
    # duplicate arcs: keep the cheapest (coo->csr would sum them)
    if not unweighted:
        A = sp.csr_matrix((n, n))
        order = np.lexsort((w, dst, src))
        s_, d_, w_ = np.asarray(src)[order], np.asarray(dst)[order], np.asarray(w)[order]
        first = np.ones(len(s_), bool)
        first[1:] = (s_[1:] != s_[:-1]) | (d_[1:] != d_[:-1])
        # callers pass weights >= 1: a zero entry would vanish from the sparse matrix
        A = sp.coo_matrix((w_[first].astype(np.float64), (s_[first], d_[first])), shape=(n, n)).tocsr()
        D = dijkstra(A, directed=True, indices=s)
    else:
        A.data[:] = 1.0
        D = shortest_path(A, directed=True, unweighted=True, indices=s)
    return np.where(np.isinf(D), I32, D).astype(np.int64)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_uniform_vs_dijkstra(seed):
    g = llpgen.uniform_graph(4096, 32768, 1, 100, seed=seed)
    want = _scipy_dist(g.n, g.src, g.dst, g.w, 0)
    for bag in (False, True):
        got = oracle.sssp(g.n, g.src, g.dst, g.w, 0, bag=bag)
        assert np.array_equal(got, want)


def test_rmat_vs_dijkstra_and_bfs():
    g = llpgen.rmat_graph(13, seed=7)
    s = llpgen.max_outdeg_source(g)
    want = _scipy_dist(g.n, g.src, g.dst, g.w, s)
    assert np.array_equal(oracle.sssp(g.n, g.src, g.dst, g.w, s, bag=True), want)
    assert np.array_equal(oracle.sssp(g.n, g.src, g.dst, g.w, s), want)
    wantb = _scipy_dist(g.n, g.src, g.dst, None, s, unweighted=True)
    assert np.array_equal(oracle.bfs(g.n, g.src, g.dst, s), wantb)
    assert np.array_equal(oracle.bfs(g.n, g.src, g.dst, s, bag=True), wantb)


def test_grid_vs_dijkstra():
    g = llpgen.grid_graph(40, 50, 1, 1000, seed=100)
    s = llpgen.max_outdeg_source(g)
    assert s == 51   # vertex (1,1): first vertex with 4 neighbours
    want = _scipy_dist(g.n, g.src, g.dst, g.w, s)
    assert np.array_equal(oracle.sssp(g.n, g.src, g.dst, g.w, s, bag=True), want)


def _brute_force(n, arcs, s):
    """Minimum over all simple paths from s (exponential; n <= 7)."""
    best = [INF] * n
    best[s] = 0
    adj = {}
    for u, v, w in arcs:
        adj.setdefault(u, []).append((v, w))

    def dfs(u, seen, dist):
        for v, w in adj.get(u, []):
            if v in seen:
                continue
            if dist + w < best[v]:
                best[v] = dist + w
            dfs(v, seen | {v}, dist + w)
    dfs(s, {s}, 0)
    return [I32 if x == INF else x for x in best]


@pytest.mark.parametrize("seed", range(25))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    m = int(rng.integers(0, 3 * n))
    src = rng.integers(0, n, m); dst = rng.integers(0, n, m); w = rng.integers(0, 20, m)
    s = int(rng.integers(0, n))
    want = _brute_force(n, list(zip(src.tolist(), dst.tolist(), w.tolist())), s)
    assert oracle.sssp(n, src, dst, w, s).tolist() == want
    assert oracle.sssp(n, src, dst, w, s, bag=True).tolist() == want


def test_invariants_uniform():
    g = llpgen.uniform_graph(2000, 9000, 0, 50, seed=11)
    d = oracle.sssp(g.n, g.src, g.dst, g.w, 5).astype(np.int64)
    assert d[5] == 0
    reach_u = d[g.src] < I32
    # d(v) <= d(u) + w on every arc out of a reached vertex
    assert np.all(d[g.dst][reach_u] <= d[g.src][reach_u] + g.w[reach_u])
    # every reached v != s has a tight in-arc
    tight = np.zeros(g.n, bool)
    t = reach_u & (d[g.dst] == d[g.src] + g.w)
    tight[g.dst[t]] = True
    reached = d < I32
    reached[5] = False
    assert np.all(tight[reached])


def test_schedule_independence_orders_and_jacobi():
    g = llpgen.uniform_graph(500, 3000, 1, 30, seed=4)
    ref = oracle.sssp(g.n, g.src, g.dst, g.w, 0)
    for k in range(4):
        order = llpgen.permutation(g.n, seed=k)
        assert np.array_equal(oracle.sssp(g.n, g.src, g.dst, g.w, 0, order=order), ref)
        assert np.array_equal(oracle.sssp(g.n, g.src, g.dst, g.w, 0, order=order, jacobi=True), ref)


@pytest.mark.parametrize("seed", range(10))
def test_schedule_independence_async_stale(seed):
    rng = np.random.default_rng(100 + seed)
    n = 12
    m = 30
    arcs = list(zip(rng.integers(0, n, m).tolist(), rng.integers(0, n, m).tolist(),
                    rng.integers(1, 9, m).tolist()))
    ref = oracle.sssp(n, [a[0] for a in arcs], [a[1] for a in arcs], [a[2] for a in arcs], 0).tolist()
    conv = lambda d: [I32 if x == INF else x for x in d]
    assert conv(sssp_pull_async(n, arcs, 0, seed=seed)) == ref
    for g in (2, 3, 5):
        assert conv(sssp_push_bag_interleaved(n, arcs, 0, apply="join", seed=seed, group=g)) == ref


def test_chain_state_selection_claim():
    """Claim 1 (Section 4.2): on the chain 0->1->...->n-1 a round-robin sweep that
    meets the chain in the wrong order needs n passes (O(n^2) examinations);
    informed selection (the bag) evaluates each vertex once (O(n))."""
    n = 300
    src = np.arange(n - 1); dst = np.arange(1, n); w = np.ones(n - 1, np.int32)
    info = {}
    d = oracle.sssp(n, src, dst, w, 0, order=np.arange(n)[::-1].copy(), info=info)
    assert d.tolist() == list(range(n))
    assert info["count"] == n          # n-1 advancing passes + one clean pass
    info = {}
    oracle.sssp(n, src, dst, w, 0, info=info)
    assert info["count"] == 2          # index order follows the chain: 1 pass + clean pass
    info = {}
    oracle.sssp(n, src, dst, w, 0, jacobi=True, info=info)
    assert info["count"] == n
    info = {}
    oracle.sssp(n, src, dst, w, 0, bag=True, info=info)
    assert info["count"] == n - 1


def test_errors():
    st, _ = oracle.sssp(3, [0, 1], [1, 2], [1, -1], 0, check=False)
    assert st == oracle.E_INPUT
    st, _ = oracle.sssp(3, [0, 1], [1, 5], [1, 1], 0, check=False)
    assert st == oracle.E_INPUT
    st, d = oracle.sssp(3, [0, 1], [1, 2], [2**30, 2**30], 0, check=False)
    assert st == oracle.E_OVERFLOW
    st, d = oracle.sssp(3, [0, 1], [1, 2], [2**30, 2**30 - 2], 0, check=False)
    assert st == oracle.OK and d[2] == 2**31 - 2
    st, _ = oracle.sssp(3, [0], [1], [1], 7, check=False)
    assert st == oracle.E_ARG
    st, d = oracle.sssp(400, np.arange(399), np.arange(1, 400), np.ones(399), 0,
                        order=np.arange(400)[::-1].copy(), max_passes=3, check=False)
    assert st == oracle.E_NOT_CONVERGED
    assert d[1] == 1 and d[399] == I32


def test_zero_weights_selfloops_duplicates():
    src = [0, 0, 1, 1, 2, 2, 3]
    dst = [1, 1, 1, 2, 3, 3, 0]
    w = [5, 3, 0, 0, 7, 2, 1]
    assert oracle.sssp(4, src, dst, w, 0).tolist() == [0, 3, 3, 5]
