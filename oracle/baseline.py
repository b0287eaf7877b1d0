"""Timing of the oracle for the benchmark's CPU baseline (test infrastructure:
run only by the CPU-baseline leg of bench.py, as a child process of its own).

One sample = the velocity-pressure and the magnetic solve (seeds 1 and 2) at
N = Nr = n with boxes of `sub` cells, two-level with FGMRES(30) (the large
benchmark's subdomain count at N = Nr = 32 with sub = 8) or one-level with
GMRES(30), to 1e-8 from 0.
With procs = P, P independent processes each set up their own preconditioners,
wait at a barrier, and solve one sample; the wall time from the barrier to
the last process's end gives the throughput of the host's cores.  The oracle
itself is single-threaded and unchanged.

    python -m oracle.baseline --n 32 --sub 8 --levels 2 --procs 16
prints one JSON line: per-process solve times, iterations and the wall time.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time


def _worker(n, sub, levels, barrier, q):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import oracle as O
    from paper_2009_02171_amd import inputs
    cases = []
    for kind, seed in ((0, 1), (1, 2)):
        pb = O.Problem(n, n, kind=kind)
        pc = O.Preconditioner(pb, sub=sub, levels=levels)
        cases.append((kind, pb, pc, inputs.rhs(n, n, seed)))
    barrier.wait()
    out = {}
    t0 = time.perf_counter()
    for kind, pb, pc, b in cases:
        t1 = time.perf_counter()
        _, st, rc = O.gmres(pb, b, pc=pc, flexible=levels == 2, rtol=1e-8, maxit=2000)
        out["VP" if kind == 0 else "BP"] = dict(outer=st["iters"], inner=int(st["inner_iters"]), rc=rc,
                                                 s=time.perf_counter() - t1)
    out["s"] = time.perf_counter() - t0
    out["end"] = time.time()
    q.put(out)


def run(n=32, sub=8, levels=2, procs=1):
    sub = (sub, sub, sub)
    ctx = mp.get_context("fork")  # this process has not touched a GPU
    barrier = ctx.Barrier(procs + 1)
    q = ctx.Queue()
    ps = [ctx.Process(target=_worker, args=(n, sub, levels, barrier, q)) for _ in range(procs)]
    for p in ps:
        p.start()
    barrier.wait()
    t0 = time.time()
    res = [q.get() for _ in ps]
    for p in ps:
        p.join()
    wall = max(r["end"] for r in res) - t0
    return dict(n=n, sub=list(sub), levels=levels, procs=procs, wall_s=wall, per_process=res)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--sub", type=int, default=8)
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--procs", type=int, default=1)
    a = ap.parse_args()
    print(json.dumps(run(a.n, a.sub, a.levels, a.procs)))
