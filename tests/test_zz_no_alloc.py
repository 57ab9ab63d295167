"""The no-allocation reduction (llp_solve_reduce_noalloc) against the
allocating entry point it mirrors (llp_solve_reduce), through the C ABI, on
two calls in a row, the second with a smaller input (the static scratch
keeps the first call's contents), and against the oracle's sum."""
import ctypes

import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")


def call(name, x):
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    o = llp.make_opts()
    fn = getattr(llp.lib(), name)
    llp._check(fn(x.numel(), llp._ptr(x), llp._ptr(out), ctypes.byref(o)))
    torch.cuda.synchronize()
    return int(out.cpu().numpy().view(np.uint64)[0])


def test_noalloc_reduce_matches_allocating_entry_point():
    for n in (1 << 24, 100003, 1):          # the second and third calls are smaller
        w = llpgen.u64_words(n, seed=11 + n % 7)
        x = torch.from_numpy(w.view(np.int64)).cuda()
        want = call("llp_solve_reduce", x)
        got = call("llp_solve_reduce_noalloc", x)
        assert got == want == oracle.reduce_sum(w), n
    empty = torch.zeros(0, dtype=torch.int64, device="cuda")
    assert call("llp_solve_reduce_noalloc", empty) == call("llp_solve_reduce", empty) == 0


def test_noalloc_reduce_rejects_timing():
    x = torch.ones(8, dtype=torch.int64, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    o = llp.make_opts(flags=llp.TIMING, stats=llp.Stats())
    assert llp.lib().llp_solve_reduce_noalloc(8, llp._ptr(x), llp._ptr(out), ctypes.byref(o)) == llp.E_ARG
