"""Train the learned per-round scheduler on the GPU from the sweep's own traces.

For each training graph several behaviour schedules (plain, push, random and
the frontier-width hybrid) are run once with LLP_TRACE; the round features
come from the trace (llp_trace_features, the same function the sweep
evaluates when it decides a round, the hybrid's own code for the round among
them).  A sample of rounds is labelled by measurement: for round r and every
candidate round code a (push / pull / dense x delta class), the solve is
re-run with the script schedule (the behaviour's codes for rounds < r, a for
rounds r .. r+h-1, the hybrid's choice afterwards) and timed on the device;
the label is the fastest code, the hybrid's own choice whenever it is within
2% of the fastest.  The network is then fitted with the library's own
forward, loss, backward and Adam kernels (full batch), and the FP32 master
weights are saved as .npy.

Usage (on a machine with an MI355X):
    python -m paper_2603_13147_amd.train_sched --out sched_weights.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import llpgen  # noqa: E402
import paper_2603_13147_amd as llp  # noqa: E402

PLAIN = llp.round_code(llp.MODE_PULL, llp.DCLASS_NONE)
PUSH = llp.round_code(llp.MODE_PUSH, llp.DCLASS_NONE)
# candidate round codes, in order of preference when their costs tie (within
# TIE of the best): no buckets before buckets, push before pull before dense
ACTIONS = [PUSH, PLAIN, llp.round_code(llp.MODE_DENSE, llp.DCLASS_NONE),
           llp.round_code(llp.MODE_PUSH, llp.DCLASS_WIDE), llp.round_code(llp.MODE_PUSH, llp.DCLASS_BASE),
           llp.round_code(llp.MODE_PULL, llp.DCLASS_WIDE), llp.round_code(llp.MODE_PULL, llp.DCLASS_BASE)]
TIE = 0.02
HYBRID = 3   # script code: the round the frontier-width hybrid would run


def hybrid_of(f5):
    """The hybrid's round code from its feature (0 push, 0.5 push with wide
    buckets, 0.25 pull, 1 dense)."""
    if f5 >= 0.75:
        return llp.round_code(llp.MODE_DENSE, llp.DCLASS_NONE)
    if f5 >= 0.375:
        return llp.round_code(llp.MODE_PUSH, llp.DCLASS_WIDE)
    if f5 >= 0.125:
        return PLAIN
    return PUSH

def init_params(seed=0):
    """He-uniform weights, zero biases (float32[LLP_MLP_PARAMS])."""
    rng = np.random.default_rng(seed)
    shapes = [(64, 12), (64,), (64, 64), (64,), (5, 64), (5,)]
    parts = []
    for s in shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def solve_fn(kind):
    return llp.sssp if kind == "sssp" else llp.bfs


def timed(fn, dg, source, ws, out, reps, **kw):
    """Smallest device time (ms) of `reps` solves."""
    import torch
    ts = []
    flags = kw.pop("flags", 0) | llp.TIMING
    for _ in range(reps):
        st = llp.Stats()
        fn(dg, source, out=out, ws=ws, stats=st, flags=flags, **kw)
        ts.append(st.device_ms)
    torch.cuda.synchronize()
    return float(np.min(ts))


def behaviours(seed):
    """Schedules whose rounds are labelled: their histories are what the
    network sees as features when it runs (plain, push and a random mix)."""
    return [("plain", dict(sched=llp.SCHED_PLAIN)), ("push", dict(sched=llp.SCHED_FIXED, flags=llp.PUSH)),
            ("random", dict(sched=llp.SCHED_RANDOM, seed=seed)), ("hybrid", dict(sched=llp.SCHED_HYBRID))]


def label_graph(name, g, kinds, max_rows, horizon, reps, log, seed=0):
    """Features and labels of sampled rounds of several schedules on g.

    Round r of a behaviour schedule is labelled with the round code a whose
    rollout -- the behaviour's own codes for rounds < r, a for rounds
    r .. r+h-1, the hybrid's choice afterwards -- reaches the fixpoint in the
    least device time (the hybrid's own code for round r when it is within
    TIE of the least)."""
    import torch
    s = llpgen.max_outdeg_source(g)
    csr = llpgen.CSRGraph(g, weighted=True, out_weights=True)
    dg = llp.DeviceGraph(csr)
    ws = llp.workspace(llp.KIND_SSSP, g.n, g.m)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    X, Y = [], []
    for kind in kinds:
        fn = solve_fn(kind)
        for bname, bkw in behaviours(seed):
            cap = min(4 * g.n + 64, 1 << 20)
            trace = llp.trace_buffer(cap)
            st = llp.Stats()
            k = dict(bkw)
            k["flags"] = k.get("flags", 0) | llp.TRACE
            fn(dg, s, out=out, ws=ws, stats=st, trace=trace, **k)
            R = int(st.rounds)
            rec = llp.trace_records(trace, R)
            codes = [int(c) for c in rec["mode"]]
            F = llp.trace_features(trace, R, g.n, g.m, llp.KIND_BFS if kind == "bfs" else llp.KIND_SSSP)
            F = F.cpu().numpy()
            rows = np.arange(1, R + 1) if R <= max_rows else np.unique(np.linspace(1, R, max_rows).astype(int))
            tail = [HYBRID] * (2 * R + 20000)   # longer than any rollout: the hybrid to the end
            t0 = time.time()
            counts = {}
            for r in rows:
                costs = []
                for a in ACTIONS:
                    plan = torch.tensor(codes[:int(r) - 1] + [a] * horizon + tail, dtype=torch.int32,
                                        device="cuda")
                    costs.append(timed(fn, dg, s, ws, out, reps, sched=llp.SCHED_SCRIPT, plan=plan))
                best = min(costs)
                hyb = hybrid_of(float(F[r - 1][5]))
                near = [a for a, c in zip(ACTIONS, costs) if c <= best * (1 + TIE)]
                lab = hyb if hyb in near else near[0]
                X.append(F[r - 1])
                Y.append(lab)
                counts[lab] = counts.get(lab, 0) + 1
            log(f"{name} {kind} under {bname}: n={g.n} m={g.m} rounds={R} labelled={len(rows)} "
                f"in {time.time() - t0:.1f}s labels={counts}")
    return X, Y


def fit(X, Y, steps, lr, seed, log):
    import torch
    x = torch.tensor(np.asarray(X, np.float32), device="cuda")
    y = torch.tensor(np.asarray(Y, np.int32), device="cuda")
    p = torch.tensor(init_params(seed), device="cuda")
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    grad = torch.zeros_like(p)
    for step in range(1, steps + 1):
        logits, act = llp.mlp_forward(p, x)
        loss, dl = llp.mlp_loss(logits, y)
        grad.zero_()
        llp.mlp_backward(p, x, act, dl, grad)
        llp.mlp_adam(grad, p, m1, m2, step, lr)
        if step % 500 == 0 or step == 1:
            log(f"step {step} loss {float(loss.item()):.4f}")
    logits, _ = llp.mlp_forward(p, x)
    z = logits.cpu().numpy()
    pred = np.where((z[:, 0] > 0), 2, np.where(z[:, 1] > 0, 1, 0)) | (np.argmax(z[:, 2:], axis=1) << 8)
    acc = float(np.mean(pred == np.asarray(Y)))
    log(f"training accuracy {acc:.3f} on {len(Y)} rounds")
    return p.cpu().numpy(), acc


def training_graphs(quick=False):
    """(name, EdgeList) of the training set: R-MAT scales 18-22 and a 2048^2 grid
    (seeds 100-107; the evaluation graphs use seed 900)."""
    out = []
    scales = [(14, 100)] if quick else [(18, 100), (18, 101), (19, 102), (19, 103), (20, 104), (20, 105),
                                        (21, 106), (22, 107)]
    for sc, seed in scales:
        out.append((f"rmat{sc}-s{seed}", llpgen.rmat_graph(sc, seed=seed), ("sssp", "bfs")))
    grids = [(64, 100)] if quick else [(2048, 106)]
    for side, seed in grids:
        out.append((f"grid{side}-s{seed}", llpgen.grid_graph(side, side, seed=seed), ("sssp",)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--rows", type=int, default=16, help="rounds labelled per trace")
    ap.add_argument("--grid-rows", type=int, default=12)
    ap.add_argument("--horizon", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--quick", action="store_true", help="tiny graphs (smoke test of the pipeline)")
    ap.add_argument("--save-data", default="", help="also save the labelled rounds (.npz: X, Y)")
    ap.add_argument("--load-data", default="", help="fit on labelled rounds saved earlier instead of labelling")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    X, Y = [], []
    if a.load_data:
        d = np.load(a.load_data)
        X, Y = list(d["X"]), [int(y) for y in d["Y"]]
        log(f"loaded {len(Y)} labelled rounds from {a.load_data}")
    else:
        for name, g, kinds in training_graphs(a.quick):
            rows = a.grid_rows if name.startswith("grid") else a.rows
            reps = a.reps
            x, y = label_graph(name, g, kinds, rows, a.horizon, reps, log, seed=a.seed)
            X += x
            Y += y
    if a.save_data:
        np.savez(a.save_data, X=np.asarray(X, np.float32), Y=np.asarray(Y, np.int32))
    p, acc = fit(X, Y, a.steps, a.lr, a.seed, log)
    np.save(a.out, p.astype(np.float32))
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump({"rows": len(Y), "train_accuracy": acc, "actions": ACTIONS,
                   "labels": {str(k): int(v) for k, v in zip(*np.unique(Y, return_counts=True))}}, f)
    log(f"saved {a.out}")


if __name__ == "__main__":
    main()
