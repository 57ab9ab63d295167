"""Writes gen_checksums.txt: SHA-256 digests of seeded generator outputs, so any
change to the bytes the oracle and the GPU path consume is caught.  Calls only
llpgen (the input generators)."""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import llpgen  # noqa: E402


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(a.tobytes())
    return h.hexdigest()


def cases():
    g = llpgen.uniform_graph(4096, 32768, 1, 100, seed=1)
    yield "uniform_n4096_m32768_seed1", digest(g.src, g.dst, g.w)
    r = llpgen.rmat_graph(14, seed=22)
    yield "rmat_s14_seed22", digest(r.src, r.dst, r.w)
    gr = llpgen.grid_graph(64, 64, 1, 1000, seed=100)
    yield "grid_64x64_seed100", digest(gr.src, gr.dst, gr.w)
    mp, wr = llpgen.sm_prefs(256, seed=3)
    yield "sm_n256_seed3", digest(mp, wr)
    pp, pi, du = llpgen.job_dag(10000, seed=4)
    yield "dag_n10000_seed4", digest(pp, pi, du)
    wt, val, W = llpgen.knapsack(17, seed=5)
    yield "knapsack_inst17_seed5", digest(wt, val) + f":{W}"
    yield "u64_n1000_seed7", digest(llpgen.u64_words(1000, seed=7))


if __name__ == "__main__":
    with open(os.path.join(HERE, "gen_checksums.txt"), "w") as f:
        f.write("# SHA-256 of seeded generator outputs (written by make_gen_checksums.py)\n")
        for name, d in cases():
            f.write(f"{name} {d}\n")
