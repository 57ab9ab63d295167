"""The status channel's rarer codes on the GPU: the host abort flag
(LLP_E_ABORTED, checked between launch batches) for the graph sweep, the
jobs sweep and stable-marriage rounds, and LLP_E_INFEASIBLE for stable
marriage on malformed lists (a man runs out of women), against the oracle's
status on the same input.  A solve after an abort, with the flag cleared,
reaches the oracle's fixpoint."""
import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")


def flag(v):
    f = torch.full((1,), v, dtype=torch.int32).pin_memory()   # [host, pinned]
    return f


def test_abort_graph_sweep():
    # a bare 3000-vertex cycle under the plain schedule: one vertex per round,
    # far more rounds than the first batch of launches
    g = llpgen.uniform_graph(3000, 0, 1, 100, seed=31)
    dg = llp.DeviceGraph(llpgen.CSRGraph(g, weighted=True, out_weights=True))
    for fn in (llp.sssp, llp.bfs):
        with pytest.raises(llp.LLPError) as e:
            fn(dg, 0, sched=llp.SCHED_PLAIN, abort_host=flag(1))
        torch.cuda.synchronize()
        assert e.value.status == llp.E_ABORTED
    got = llp.sssp(dg, 0, sched=llp.SCHED_PLAIN, abort_host=flag(0))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.sssp(g.n, g.src, g.dst, g.w, 0))


def test_abort_jobs():
    n = 3000
    pp = np.concatenate([[0, 0], np.arange(1, n, dtype=np.int32)]).astype(np.int32)
    pi = np.arange(0, n - 1, dtype=np.int32)
    d = llpgen.uniform_ints(n, 1, 100, seed=5).astype(np.int32)
    sp, si = llpgen.job_succ(pp, pi)
    with pytest.raises(llp.LLPError) as e:
        llp.jobs(pp, pi, d, sp, si, abort_host=flag(1))
    torch.cuda.synchronize()
    assert e.value.status == llp.E_ABORTED
    got = llp.jobs(pp, pi, d, sp, si, abort_host=flag(0))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.jobs(pp, pi, d))


def test_abort_stable_marriage_rounds():
    mpref, wrank = llpgen.sm_prefs(2048, seed=6)
    with pytest.raises(llp.LLPError) as e:
        llp.stable_marriage(mpref, wrank, sched=llp.SCHED_FIXED, flags=llp.DENSE, abort_host=flag(1))
    torch.cuda.synchronize()
    assert e.value.status == llp.E_ABORTED
    w, _ = llp.stable_marriage(mpref, wrank, sched=llp.SCHED_FIXED, flags=llp.DENSE, abort_host=flag(0))
    torch.cuda.synchronize()
    assert np.array_equal(w.cpu().numpy(), oracle.stable_marriage(mpref, wrank)[0])


@pytest.mark.parametrize("kw", [dict(), dict(chunk=1), dict(sched=llp.SCHED_FIXED, flags=llp.DENSE)],
                         ids=["chains", "chunk1", "dense"])
def test_stable_marriage_infeasible_lists(kw):
    # every man lists woman 0 three times: two men run out of women
    n = 3
    mpref = np.zeros((n, n), np.int16)
    wrank = np.tile(np.arange(n, dtype=np.int16), (n, 1))
    st, _ = oracle.stable_marriage(mpref, wrank, check=False)
    assert st == llp.E_INFEASIBLE
    with pytest.raises(llp.LLPError) as e:
        llp.stable_marriage(mpref, wrank, **kw)
    torch.cuda.synchronize()
    assert e.value.status == llp.E_INFEASIBLE
    # validation names the malformed lists instead
    with pytest.raises(llp.LLPError) as e:
        llp.stable_marriage(mpref, wrank, flags=llp.VALIDATE | kw.get("flags", 0),
                            **{k: v for k, v in kw.items() if k != "flags"})
    torch.cuda.synchronize()
    assert e.value.status == llp.E_INPUT
