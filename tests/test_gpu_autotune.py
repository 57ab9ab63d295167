"""The graph sweep's autotuner (llp_autotune_graph) and its records: the
tuned shape is looked up by size class, solves that leave the shape to the
library use it and still reach the oracle's fixpoint, and the records survive
a save, a shutdown and a load."""
import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")


def test_graph_autotune_records_and_reloads(tmp_path):
    g = llpgen.rmat_graph(14, seed=3)
    s = llpgen.max_outdeg_source(g)
    dg = llp.DeviceGraph(llpgen.CSRGraph(g, weighted=True, out_weights=True))
    want_d = oracle.sssp(g.n, g.src, g.dst, g.w, s, bag=True)
    want_b = oracle.bfs(g.n, g.src, g.dst, s, bag=True)
    llp.lib().llp_shutdown()   # no records yet
    with pytest.raises(llp.LLPError):
        llp.autotune_lookup(llp.KIND_SSSP, dg.m)

    rows, out = llp.autotune_graph(dg, s, llp.KIND_SSSP, sched=llp.SCHED_HYBRID)
    torch.cuda.synchronize()
    assert [c for c, _ in rows] == [1, 2, 3, 4] and all(ms > 0 for _, ms in rows)
    assert np.array_equal(out.cpu().numpy(), want_d)
    best = min(rows, key=lambda r: r[1])[0]
    assert llp.autotune_lookup(llp.KIND_SSSP, dg.m) == (0, best)
    assert llp.autotune_get(llp.KIND_SSSP) == (0, best)
    # the nearest size class serves other sizes of the same kind; BFS has no record
    assert llp.autotune_lookup(llp.KIND_SSSP, dg.m * 64) == (0, best)
    assert llp.autotune_lookup(llp.KIND_SSSP, 3) == (0, best)
    with pytest.raises(llp.LLPError):
        llp.autotune_lookup(llp.KIND_BFS, dg.m)

    # solves that leave the shape to the library (chunk 0) take the record, same fixpoint
    for sched in (llp.SCHED_HYBRID, llp.SCHED_PLAIN):
        assert np.array_equal(llp.sssp(dg, s, sched=sched).cpu().numpy(), want_d), sched
    rows_b, out_b = llp.autotune_graph(dg, s, llp.KIND_BFS)
    torch.cuda.synchronize()
    assert np.array_equal(out_b.cpu().numpy(), want_b)
    best_b = min(rows_b, key=lambda r: r[1])[0]
    assert np.array_equal(llp.bfs(dg, s, sched=llp.SCHED_HYBRID).cpu().numpy(), want_b)

    # persisted: save, forget, load
    path = tmp_path / "tune.json"
    llp.autotune_save(path)
    llp.lib().llp_shutdown()
    with pytest.raises(llp.LLPError):
        llp.autotune_lookup(llp.KIND_SSSP, dg.m)
    assert llp.autotune_load(path) == 2
    assert llp.autotune_lookup(llp.KIND_SSSP, dg.m) == (0, best)
    assert llp.autotune_lookup(llp.KIND_BFS, dg.m) == (0, best_b)
    assert np.array_equal(llp.sssp(dg, s).cpu().numpy(), want_d)
    llp.lib().llp_shutdown()


def test_graph_autotune_rejects_other_kinds():
    g = llpgen.uniform_graph(100, 400, seed=2)
    dg = llp.DeviceGraph(llpgen.CSRGraph(g, weighted=True, out_weights=True))
    with pytest.raises(llp.LLPError) as e:
        llp.autotune_graph(dg, 0, llp.KIND_JOBS)
    assert e.value.status == llp.E_ARG
