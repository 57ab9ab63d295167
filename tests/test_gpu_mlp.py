"""GPU parity of the learned scheduler's training kernels (forward, loss,
backward, Adam) against the float64 oracle in oracle/mlp.py, and the
consistency between trace features and in-sweep decisions.  Tolerances:
bf16-stored activations within one bf16 unit in the last place; fp32-kept
values within 1e-4 relative (plus a small absolute floor for sums that
cancel)."""
import numpy as np
import pytest

import llpgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")


def rand_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mlp.NPAR).astype(np.float32)


def features(B, seed):
    # the sweep's features lie in [0, 1] apart from two log-ratio terms
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (B, 12)).astype(np.float32)
    x[:, 7] = rng.uniform(-8, 8, B)
    return x


def bf16_close(got, want):
    ulp = np.maximum(np.abs(want), 1e-30) * 2.0 ** -7
    return np.all(np.abs(got - want) <= ulp + 1e-30)


def act_floats(act):
    a = act.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("B,seed", [(1, 1), (63, 2), (1000, 3), (4097, 4)])
def test_forward_layers(B, seed):
    p = rand_params(seed)
    x = features(B, seed)
    pd, xd = torch.tensor(p, device="cuda"), torch.tensor(x, device="cuda")
    logits, act = llp.mlp_forward(pd, xd)
    torch.cuda.synchronize()
    a = act_floats(act)
    h1, h2 = a[:, :64], a[:, 64:]
    assert bf16_close(h1, mlp.layer1(p, x))
    assert bf16_close(h2, mlp.layer2(p, h1))
    want = mlp.layer3(p, h2)
    got = logits.cpu().numpy().astype(np.float64)
    assert np.allclose(got, want, rtol=1e-4, atol=1e-5 * np.abs(want).max())


def test_loss_matches_oracle():
    rng = np.random.default_rng(5)
    B = 777
    z = rng.normal(0, 3, (B, 5)).astype(np.float32)
    labels = (rng.integers(0, 3, B) | (rng.integers(0, 3, B) << 8)).astype(np.int32)
    loss, dl = llp.mlp_loss(torch.tensor(z, device="cuda"), torch.tensor(labels, device="cuda"))
    torch.cuda.synchronize()
    want_l, want_d = mlp.loss(z, labels)
    assert abs(float(loss.item()) - want_l) <= 1e-5 * abs(want_l)
    assert np.allclose(dl.cpu().numpy(), want_d, rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("B,seed", [(1, 6), (300, 7), (5000, 8)])
def test_backward_matches_oracle(B, seed):
    p = rand_params(seed)
    x = features(B, seed)
    rng = np.random.default_rng(seed)
    d = (rng.normal(0, 1, (B, 5)) / B).astype(np.float32)
    pd, xd = torch.tensor(p, device="cuda"), torch.tensor(x, device="cuda")
    _, act = llp.mlp_forward(pd, xd)
    grad = torch.zeros(mlp.NPAR, dtype=torch.float32, device="cuda")
    llp.mlp_backward(pd, xd, act, torch.tensor(d, device="cuda"), grad)
    torch.cuda.synchronize()
    a = act_floats(act)
    want = mlp.backward(p, x, a[:, :64], a[:, 64:], d)
    got = grad.cpu().numpy().astype(np.float64)
    scale = np.abs(want).max()
    assert np.allclose(got, want, rtol=1e-4, atol=1e-6 * scale)
    # accumulation: a second call doubles the gradient
    llp.mlp_backward(pd, xd, act, torch.tensor(d, device="cuda"), grad)
    torch.cuda.synchronize()
    assert np.allclose(grad.cpu().numpy(), 2 * want, rtol=1e-4, atol=2e-6 * scale)


def test_adam_matches_oracle():
    rng = np.random.default_rng(9)
    p = rand_params(9).astype(np.float64)
    m1 = np.zeros(mlp.NPAR)
    m2 = np.zeros(mlp.NPAR)
    pd = torch.tensor(p.astype(np.float32), device="cuda")
    m1d, m2d = torch.zeros_like(pd), torch.zeros_like(pd)
    for step in range(1, 4):
        g = rng.normal(0, 1e-2, mlp.NPAR)
        gd = torch.tensor(g.astype(np.float32), device="cuda")
        llp.mlp_adam(gd, pd, m1d, m2d, step, 1e-3)
        p, m1, m2 = mlp.adam(g.astype(np.float32).astype(np.float64), p, m1, m2, step, 1e-3)
    torch.cuda.synchronize()
    assert np.allclose(pd.cpu().numpy(), p, rtol=1e-5, atol=1e-7)


def test_training_fits_a_separable_rule():
    from paper_2603_13147_amd import train_sched
    rng = np.random.default_rng(10)
    x = features(2000, 10)
    y = np.where(x[:, 0] > 0.5, 2, np.where(x[:, 2] > 0.6, 1, 0)) | (np.where(x[:, 3] > 0.5, 2, 0) << 8)
    p, acc = train_sched.fit(list(x), list(y.astype(np.int32)), 1500, 3e-3, 0, lambda m: None)
    assert acc > 0.95


@pytest.mark.parametrize("which", ["rmat13-sssp", "rmat13-bfs", "grid64-sssp"])
def test_learned_decisions_match_trace_features(which):
    """The decision the sweep takes in round r is the network's output on the
    features llp_trace_features computes from the trace (same function, the
    hybrid's code for the round included: BFS thresholds and the wide
    buckets of a sparse weighted graph), and the learned schedule reaches the
    oracle's fixpoint."""
    g = llpgen.rmat_graph(13, seed=21) if which.startswith("rmat") else llpgen.grid_graph(64, 64, seed=21)
    bfs = which.endswith("bfs")
    s = llpgen.max_outdeg_source(g)
    dg = llp.DeviceGraph(llpgen.CSRGraph(g, weighted=True, out_weights=True))
    p = rand_params(11, scale=0.8)
    llp.set_sched_weights(p)
    trace = llp.trace_buffer(4096)
    st = llp.Stats()
    fn = llp.bfs if bfs else llp.sssp
    d = fn(dg, s, sched=llp.SCHED_LEARNED, flags=llp.TRACE, trace=trace, stats=st)
    torch.cuda.synchronize()
    want = oracle.sssp(g.n, g.src, g.dst, None if bfs else g.w, s, bag=True)
    assert np.array_equal(d.cpu().numpy(), want)
    R = int(st.rounds)
    rec = llp.trace_records(trace, R)
    F = llp.trace_features(trace, R, g.n, g.m, llp.KIND_BFS if bfs else llp.KIND_SSSP)
    # the hybrid's code as a feature: dense above m/3 (SSSP) or m/14 (BFS) out-arcs,
    # wide buckets for the push rounds of the sparse weighted grid
    frac = 1 / 14 if bfs else 1 / 3
    hyb = np.where(rec["in_edges"] > frac * g.m, 1.0, 0.5 if which.startswith("grid") else 0.0)
    assert np.array_equal(F.cpu().numpy()[:, 5], hyb)
    logits, _ = llp.mlp_forward(torch.tensor(p, device="cuda"), F)
    z = logits.cpu().numpy()
    mode = np.where(z[:, 0] > 0, 2, np.where(z[:, 1] > 0, 1, 0))
    dc = np.argmax(z[:, 2:], axis=1)
    # rounds of fewer than m / 256 frontier arcs take the hybrid's code
    gated = rec["in_edges"].astype(np.int64) * 256 < g.m
    hmode = np.where(hyb == 1.0, 1, 2)
    hdc = np.where(hyb == 0.5, llp.DCLASS_WIDE, llp.DCLASS_NONE)
    assert gated.any() and (~gated).any()
    assert np.array_equal(rec["mode"] & 3, np.where(gated, hmode, mode))
    assert np.array_equal((rec["mode"] >> 8) & 3, np.where(gated, hdc, dc))
