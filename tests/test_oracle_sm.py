"""Pins of the stable-marriage oracle (Section 5.4): man-proposing Gale-Shapley,
brute force over all matchings, stability invariants, scan vs per-woman table."""
import itertools
from collections import deque

import numpy as np
import pytest

import llpgen
import oracle


def gale_shapley(mpref, wrank):
    """Textbook man-proposing deferred acceptance (Gale and Shapley 1962)."""
    n = len(mpref)
    nxt = [0] * n
    holder = [-1] * n
    free = deque(range(n))
    while free:
        m = free.popleft()
        w = int(mpref[m][nxt[m]])
        nxt[m] += 1
        h = holder[w]
        if h < 0:
            holder[w] = m
        elif wrank[w][m] < wrank[w][h]:
            holder[w] = m
            free.append(h)
        else:
            free.append(m)
    wife = [0] * n
    for w, m in enumerate(holder):
        wife[m] = w
    return wife


def is_stable(mpref, wrank, wife):
    n = len(wife)
    husband = {w: m for m, w in enumerate(wife)}
    mrank = np.argsort(mpref, axis=1)
    for m in range(n):
        for w in range(n):
            if mrank[m][w] < mrank[m][wife[m]] and wrank[w][m] < wrank[w][husband[w]]:
                return False
    return True


def test_random_vs_gale_shapley():
    for n, seed in [(1, 1), (2, 2), (50, 3), (300, 4)]:
        mp, wr = llpgen.sm_prefs(n, seed)
        want = gale_shapley(mp, wr)
        wife, prop = oracle.stable_marriage(mp, wr)
        assert wife.tolist() == want
        assert all(mp[m, prop[m]] == wife[m] for m in range(n))
        if n <= 300:
            wife2, prop2 = oracle.stable_marriage(mp, wr, scan=True)
            assert np.array_equal(wife, wife2) and np.array_equal(prop, prop2)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_man_optimal(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    mp = np.array([rng.permutation(n) for _ in range(n)], np.int16)
    wl = [rng.permutation(n) for _ in range(n)]
    wr = np.zeros((n, n), np.int16)
    for w in range(n):
        wr[w, wl[w]] = np.arange(n)
    stable = [p for p in itertools.permutations(range(n)) if is_stable(mp, wr, list(p))]
    assert stable
    mrank = np.argsort(mp, axis=1)
    # man-optimal: every man gets his best partner over all stable matchings
    best = [min(mrank[m][p[m]] for p in stable) for m in range(n)]
    wife, _ = oracle.stable_marriage(mp, wr, scan=True)
    assert [mrank[m][wife[m]] for m in range(n)] == best
    assert tuple(wife.tolist()) in stable
    wife2, _ = oracle.stable_marriage(mp, wr)
    assert np.array_equal(wife, wife2)


def test_invariants_n1000():
    mp, wr = llpgen.sm_prefs(1000, 9)
    wife, prop = oracle.stable_marriage(mp, wr)
    assert sorted(wife.tolist()) == list(range(1000))
    assert is_stable(mp[:1000], wr, wife.tolist())


def test_identical_lists_worst_case():
    """All men share one list and all women rank men 0..n-1 identically: man i
    ends with the i-th woman of the common list (ranks i on it)."""
    n = 40
    common = np.random.default_rng(0).permutation(n)
    mp = np.tile(common, (n, 1)).astype(np.int16)
    wr = np.tile(np.arange(n), (n, 1)).astype(np.int16)
    wife, prop = oracle.stable_marriage(mp, wr, scan=True)
    assert prop.tolist() == list(range(n))
    assert wife.tolist() == common.tolist()


def test_bad_input():
    mp = np.array([[0, 5], [1, 0]], np.int16)
    wr = np.array([[0, 1], [1, 0]], np.int16)
    st, _ = oracle.stable_marriage(mp, wr, check=False)
    assert st == oracle.E_INPUT
