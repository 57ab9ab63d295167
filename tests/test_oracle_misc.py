"""Pins of the knapsack (Section 5.8), transitive closure (Section 5.7) and
reduction (Section 5.6) oracles."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import llpgen
import oracle


# ------------------------------------------------------------------ knapsack
def brute_knapsack(wt, val, W):
    best = 0
    n = len(wt)
    for mask in range(1 << n):
        tw = tv = 0
        for i in range(n):
            if mask >> i & 1:
                tw += wt[i]; tv += val[i]
        if tw <= W and tv > best:
            best = tv
    return best


@pytest.mark.parametrize("seed", range(20))
def test_knapsack_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 13))
    W = int(rng.integers(0, 60))
    wt = rng.integers(0, 25, n); val = rng.integers(0, 100, n)
    best, row = oracle.knapsack(wt, val, W, row=True)
    assert best == brute_knapsack(wt.tolist(), val.tolist(), W)
    # the last row holds the optimum for every capacity c <= W
    for c in range(0, W + 1, max(1, W // 7)):
        assert row[c] == brute_knapsack(wt.tolist(), val.tolist(), c)


def test_knapsack_properties_generated():
    for inst in range(3):
        wt, val, W = llpgen.knapsack(inst, seed=5)
        best, row = oracle.knapsack(wt, val, W, row=True)
        assert best == row[W]
        assert np.all(np.diff(row) >= 0)                       # non-decreasing in c
        assert best <= val.sum()
        fits = val[wt <= W]
        assert best >= (fits.max() if fits.size else 0)
        # items heavier than W never fit: appending one changes nothing
        assert oracle.knapsack(np.append(wt, W + 1), np.append(val, 10**5), W) == best
        # doubling every value doubles the optimum
        assert oracle.knapsack(wt, 2 * val, W) == 2 * best
    # every item fits: the optimum takes them all
    assert oracle.knapsack([1, 2, 3], [4, 5, 6], 6) == 15
    assert oracle.knapsack([7, 8], [4, 5], 6) == 0
    assert oracle.knapsack([], [], 10) == 0


def test_knapsack_errors():
    st, _ = oracle.knapsack([1, -2], [1, 1], 5, check=False)
    assert st == oracle.E_INPUT
    st, _ = oracle.knapsack([1, 1], [2**30, 2**30], 5, check=False)
    assert st == oracle.E_OVERFLOW


# ------------------------------------------------------------------ transitive closure
def closure_by_bfs(n, src, dst):
    A = sp.coo_matrix((np.ones(len(src)), (src, dst)), shape=(n, n)).tocsr()
    R = np.zeros((n, n), bool)
    for u in range(n):
        # vertices reachable by >= 1 arc: BFS from each out-neighbour
        for x in A.indices[A.indptr[u]:A.indptr[u + 1]]:
            R[u, breadth_first_order(A, x, directed=True, return_predecessors=False)] = True
    return R


def unpack(bits, n):
    out = np.zeros((n, n), bool)
    for v in range(n):
        out[:, v] = (bits[:, v >> 5] >> np.uint32(v & 31)) & np.uint32(1)
    return out


@pytest.mark.parametrize("n,m,seed", [(1, 1, 0), (5, 6, 1), (33, 40, 2), (70, 150, 3), (100, 90, 4)])
def test_tc_vs_bfs(n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m); dst = rng.integers(0, n, m)
    got = unpack(oracle.transitive_closure(n, src, dst), n)
    assert np.array_equal(got, closure_by_bfs(n, src, dst))


def test_tc_brute_paths_tiny():
    rng = np.random.default_rng(7)
    for _ in range(10):
        n = int(rng.integers(1, 7))
        arcs = set(zip(rng.integers(0, n, 8).tolist(), rng.integers(0, n, 8).tolist()))
        want = np.zeros((n, n), bool)
        # a path of length <= n reaches everything reachable
        for L in range(1, n + 1):
            for walk in itertools.product(range(n), repeat=L + 1):
                if all((walk[i], walk[i + 1]) in arcs for i in range(L)):
                    want[walk[0], walk[-1]] = True
        src = [a for a, _ in arcs]; dst = [b for _, b in arcs]
        assert np.array_equal(unpack(oracle.transitive_closure(n, src, dst), n), want)


def test_tc_dag_chain_and_cycle():
    n = 10
    bits = unpack(oracle.transitive_closure(n, np.arange(n - 1), np.arange(1, n)), n)
    assert np.array_equal(bits, np.triu(np.ones((n, n), bool), 1))
    bits = unpack(oracle.transitive_closure(n, np.arange(n), (np.arange(n) + 1) % n), n)
    assert bits.all()      # on a cycle every pair, diagonal included, is reachable


# ------------------------------------------------------------------ reduction
def test_reduce_closed_forms():
    n = 100000
    x = np.arange(n, dtype=np.uint64)
    assert oracle.reduce_sum(x) == n * (n - 1) // 2
    assert oracle.reduce_sum(np.array([2**64 - 1, 2], np.uint64)) == 1
    assert oracle.reduce_sum(np.full(4, 2**63, np.uint64)) == 0
    y = llpgen.u64_words(4096, seed=3)
    neg = (np.uint64(0) - y)
    assert oracle.reduce_sum(np.concatenate([y, neg])) == 0
    p = llpgen.permutation(4096, seed=1)
    assert oracle.reduce_sum(y[p]) == oracle.reduce_sum(y)
    assert oracle.reduce_sum(np.zeros(0, np.uint64)) == 0
