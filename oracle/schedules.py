"""Pure-Python schedule simulators for tiny inputs -- TEST INFRASTRUCTURE ONLY.

They exercise the paper's claim that any fair schedule of monotone advances
reaches the same least fixpoint (Background: Algorithm LLP, Definition 3 and
Lemma 1; Section 4.2: requirements for a correct implementation), and that an
overwrite computed from a stale read does not (Section 4.2, Claim 2).  Natural
domain: distances are Python ints, ``INF`` is float('inf').
"""
from __future__ import annotations

import random

INF = float("inf")


def relax_arc(d, u, v, w):
    """Single-edge relaxation, a partial advance of v (Definition 3: the value
    d(u) + w bounds v from one in-arc): d(v) := min(d(v), d(u) + w)."""
    d = list(d)
    if d[u] != INF and d[u] + w < d[v]:
        d[v] = d[u] + w
    return d


def sssp_alpha(d, in_arcs, v):
    """alpha of Section 5.2: min of d(v) and d(u) + w over every in-arc (u, v, w)."""
    best = d[v]
    for u, w in in_arcs[v]:
        if d[u] != INF and d[u] + w < best:
            best = d[u] + w
    return best


def sssp_pull_async(n, arcs, source, *, seed=0, stale_depth=4, steps=2000):
    """Randomised asynchronous pull schedule with stale reads, applied with the
    lattice join (d only moves forward: min on distances, atomicMax on an
    order-reversed encoding).  Each step picks a random vertex and computes its
    alpha from a snapshot up to ``stale_depth`` steps old.  Fairness: afterwards
    every vertex is re-evaluated against fresh state until a pass changes
    nothing."""
    rng = random.Random(seed)
    in_arcs = [[] for _ in range(n)]
    for u, v, w in arcs:
        in_arcs[v].append((u, w))
    d = [INF] * n
    d[source] = 0
    history = [list(d)]
    for _ in range(steps):
        v = rng.randrange(n)
        if v == source:
            continue
        snap = history[max(0, len(history) - 1 - rng.randrange(stale_depth))]
        a = sssp_alpha(snap, in_arcs, v)
        if a < d[v]:
            d[v] = a
        history.append(list(d))
    while True:
        changed = False
        for v in range(n):
            if v != source:
                a = sssp_alpha(d, in_arcs, v)
                if a < d[v]:
                    d[v] = a
                    changed = True
        if not changed:
            return d


def sssp_push_bag_interleaved(n, arcs, source, *, apply="join", seed=None, group=2,
                              init_state=None, init_bag=None):
    """Push-style bag solver in which ``group`` workers pop arcs together, all
    read the state, then write one after the other (the interleaving of
    Section 4.2, Claim 2).  A work item is an arc (u, v, w); its candidate is
    d(u) + w, compared with the read value of d(v).

    apply="join":  d(v) := min(d(v), cand)   (monotone, what atomicMax gives)
    apply="store": d(v) := cand when cand < the (possibly stale) read of d(v)

    Every successful write pushes v's out-arcs (the successor set of Section
    4.2).  The bag is processed in FIFO order, or in a random order when seed
    is given.  Returns the state when the bag is empty."""
    rng = random.Random(seed) if seed is not None else None
    out_arcs = [[] for _ in range(n)]
    for u, v, w in arcs:
        out_arcs[u].append((u, v, w))
    d = list(init_state) if init_state is not None else [INF] * n
    if init_state is None:
        d[source] = 0
    bag = list(init_bag) if init_bag is not None else list(out_arcs[source])
    while bag:
        take = []
        for _ in range(min(group, len(bag))):
            k = rng.randrange(len(bag)) if rng else 0
            take.append(bag.pop(k))
        reads = [(u, v, w, d[u], d[v]) for (u, v, w) in take]
        for u, v, w, du, dv in reads:
            if du == INF:
                continue
            cand = du + w
            if apply == "join":
                if cand < d[v]:
                    d[v] = cand
                    bag.extend(out_arcs[v])
            else:
                if cand < dv:
                    d[v] = cand
                    bag.extend(out_arcs[v])
    return d
