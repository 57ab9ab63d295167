"""The Python binding's argument checks: a caller-supplied output or array of
the wrong dtype, shape, device or length is refused with E_ARG before any
kernel runs (the kernels write outputs whole and trust the lengths they are
given), and a correct caller-supplied output is filled in place."""
import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")


def refused(fn, *a, **kw):
    with pytest.raises(llp.LLPError) as e:
        fn(*a, **kw)
    assert e.value.status == llp.E_ARG, str(e.value)


def test_graph_outputs():
    g = llpgen.uniform_graph(300, 2000, seed=3)
    csr = llpgen.CSRGraph(g, weighted=True)
    dg = llp.DeviceGraph(csr)
    for bad in (torch.empty(299, dtype=torch.int32, device="cuda"),        # too short
                torch.empty(300, dtype=torch.int64, device="cuda"),        # wrong dtype
                torch.empty(300, dtype=torch.int32),                       # host memory
                torch.empty(600, dtype=torch.int32, device="cuda")[::2]):  # strided view
        refused(llp.sssp, dg, 0, out=bad)
        refused(llp.bfs, dg, 0, out=bad)
    out = torch.full((300,), -5, dtype=torch.int32, device="cuda")
    got = llp.sssp(dg, 0, out=out)
    torch.cuda.synchronize()
    assert got is out
    assert np.array_equal(out.cpu().numpy(), oracle.sssp(g.n, g.src, g.dst, g.w, 0))


def test_stable_marriage_outputs():
    mp, wr = llpgen.sm_prefs(50, seed=2)
    refused(llp.stable_marriage, mp, wr, wife=torch.empty(49, dtype=torch.int32, device="cuda"))
    refused(llp.stable_marriage, mp, wr, prop=torch.empty(50, dtype=torch.int16, device="cuda"))
    refused(llp.stable_marriage, mp, wr[:, :49])
    wife = torch.empty(50, dtype=torch.int32, device="cuda")
    w, _ = llp.stable_marriage(mp, wr, wife=wife)
    torch.cuda.synchronize()
    assert w is wife
    assert np.array_equal(wife.cpu().numpy(), oracle.stable_marriage(mp, wr)[0])


def test_jobs_lengths():
    pp, pi, du = llpgen.job_dag(200, seed=4)
    sp, si = llpgen.job_succ(pp, pi)
    refused(llp.jobs, pp[:-1], pi, du, sp, si)             # pred_ptr needs n + 1 entries
    refused(llp.jobs, pp, pi, du, sp[:-1], si)
    refused(llp.jobs, pp, pi, du, sp, si[:-1])             # one successor entry per arc
    refused(llp.jobs, pp, pi, du, sp, si, out=torch.empty(200, dtype=torch.int32))


def test_knapsack_tc_reduce():
    refused(llp.knapsack, np.array([1, 2, 3], np.int32), np.array([4, 5], np.int32), 10)
    refused(llp.transitive_closure, 5, np.array([0, 1, 2], np.int32), np.array([1, 2], np.int32))
    refused(llp.reduce_sum, torch.arange(10, dtype=torch.int32, device="cuda"))


def test_mlp_and_trace():
    P = llp.MLP_PARAMS
    p = torch.zeros(P, dtype=torch.float32, device="cuda")
    x = torch.zeros((4, llp.MLP_IN), dtype=torch.float32, device="cuda")
    refused(llp.mlp_forward, p[:-1], x)
    refused(llp.mlp_forward, p, x.double())
    refused(llp.mlp_forward, p, torch.zeros((4, 11), dtype=torch.float32, device="cuda"))
    logits, act = llp.mlp_forward(p, x)
    refused(llp.mlp_loss, logits, torch.zeros(4, dtype=torch.int64, device="cuda"))
    grad = torch.zeros(P, dtype=torch.float32, device="cuda")
    refused(llp.mlp_backward, p, x, act[:3], logits, grad)
    refused(llp.mlp_backward, p, x, act, logits, grad.double())
    refused(llp.mlp_adam, grad, p, grad.clone(), grad[:-1].clone(), 1, 1e-3)
    refused(llp.trace_features, torch.zeros(10, dtype=torch.uint8, device="cuda"), 4, 100, 1000)
    torch.cuda.synchronize()
