"""Pins of the job-scheduling oracle (Section 5.5): Kahn longest path, path
enumeration, the race example of Section 4.2, invariants, cycle detection."""
import numpy as np
import pytest

import llpgen
import oracle
from conftest import read_golden


def kahn_longest_start(pred_ptr, pred_idx, dur):
    """Textbook critical-path pass in topological order (Kahn 1962)."""
    n = len(dur)
    succ = [[] for _ in range(n)]
    indeg = np.diff(pred_ptr).astype(np.int64)
    for j in range(n):
        for k in range(pred_ptr[j], pred_ptr[j + 1]):
            succ[pred_idx[k]].append(j)
    S = np.zeros(n, np.int64)
    q = [j for j in range(n) if indeg[j] == 0]
    i = 0
    while i < len(q):
        p = q[i]; i += 1
        for c in succ[p]:
            S[c] = max(S[c], S[p] + dur[p])
            indeg[c] -= 1
            if indeg[c] == 0:
                q.append(c)
    return S


def test_race_example():
    rows = {r[0]: r[1:] for r in read_golden("race_examples.txt")}
    c1, c2 = (int(x) for x in rows["jobs_pred_completion"])
    tj = int(rows["jobs_tj"][0])
    # p1 (duration c1) and p2 (duration c2) start at 0; j depends on both
    S = oracle.jobs([0, 0, 0, 2], [0, 1], [c1, c2, tj])
    assert S[2] + tj == int(rows["jobs_correct_completion"][0])
    assert S[2] + tj != int(rows["jobs_overwrite_completion"][0])


@pytest.mark.parametrize("n,seed", [(100, 1), (5000, 2), (50000, 4)])
def test_vs_kahn(n, seed):
    pp, pi, du = llpgen.job_dag(n, seed=seed)
    want = kahn_longest_start(pp, pi, du)
    for bag in (False, True):
        assert np.array_equal(oracle.jobs(pp, pi, du, bag=bag), want)


def _all_paths_start(n, preds, dur):
    """Start time = max over all paths p0 -> ... -> j of the durations before j
    (explicit enumeration; tiny DAGs only)."""
    best = [0] * n

    def walk(j, acc):
        best[j] = max(best[j], acc)
    for j in range(n):
        # enumerate every path ending at j backwards
        stack = [(j, 0)]
        while stack:
            v, acc = stack.pop()
            walk(j, acc)
            for p in preds[v]:
                stack.append((p, acc + dur[p]))
    return best


@pytest.mark.parametrize("seed", range(15))
def test_path_enumeration_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 11))
    preds = [sorted(set(rng.integers(0, j, rng.integers(0, j + 1)).tolist())) if j else [] for j in range(n)]
    # relabel by a random permutation so the DAG is not index-ordered
    perm = rng.permutation(n)
    inv = np.argsort(perm)
    preds_p = [None] * n
    for j in range(n):
        preds_p[perm[j]] = [int(perm[p]) for p in preds[j]]
    dur = rng.integers(0, 50, n)
    pp = np.zeros(n + 1, np.int64)
    pp[1:] = np.cumsum([len(x) for x in preds_p])
    pi = np.array([p for x in preds_p for p in x], np.int64)
    want = _all_paths_start(n, preds_p, dur)
    assert oracle.jobs(pp, pi, dur).tolist() == want
    assert oracle.jobs(pp, pi, dur, bag=True).tolist() == want
    del inv


def test_invariants():
    pp, pi, du = llpgen.job_dag(20000, seed=8)
    S = oracle.jobs(pp, pi, du).astype(np.int64)
    child = np.repeat(np.arange(20000), np.diff(pp))
    assert np.all(S[child] >= S[pi] + du[pi])
    tight = np.zeros(20000, bool)
    tight[child[S[child] == S[pi] + du[pi]]] = True
    has_pred = np.diff(pp) > 0
    assert np.all(tight[has_pred])
    assert np.all(S[~has_pred] == 0)


def test_cycle_and_errors():
    # 0 -> 1 -> 2 -> 0
    st, _ = oracle.jobs([0, 1, 2, 3], [2, 0, 1], [1, 1, 1], check=False)
    assert st == oracle.E_CYCLE
    st, _ = oracle.jobs([0, 1, 2, 3], [2, 0, 1], [1, 1, 1], bag=True, check=False)
    assert st == oracle.E_CYCLE
    st, _ = oracle.jobs([0, 0, 1], [0], [1, -1], check=False)
    assert st == oracle.E_INPUT
    st, _ = oracle.jobs([0, 0, 1, 2], [0, 1], [2**30, 2**30, 5], check=False)
    assert st == oracle.E_OVERFLOW
