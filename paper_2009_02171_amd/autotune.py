"""Empirical tuning of the launch shapes of one shell's solve: the stencil
kernel's workgroup shape (timed operator applies) and the RAS subdomain size
(timed solves of the shell's own system with the FP32 one-level
preconditioner).  Results are identical for every choice; only the time
differs.  Decisions are cached per (N, Nr, system, coefficients)."""
from __future__ import annotations

import time

import torch

from . import csdyn

TILES = {1: "32x8", 2: "16x16", 3: "64x4", 4: "16x8", 5: "32x4", 6: "16x16 LDS requests"}
SUBDOMAINS = (8, 12, 16, 20, 24)

_cache: dict = {}


def _events_ms(fn, reps):
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def tune_tile(op: csdyn.Operator, reps: int = 10):
    x = torch.randn(op.shape, dtype=torch.float64, device=op.device)
    y = op.empty()
    times = {}
    for t in TILES:
        op.set_tile(t)
        times[t] = _events_ms(lambda: op.apply(x, y), reps)
    best = min(times, key=times.get)
    op.set_tile(best)
    return best, {TILES[k]: round(v * 1e3, 2) for k, v in times.items()}


def candidate_subdomains(n: int, nr: int):
    return [s for s in SUBDOMAINS if n % s == 0 and nr % s == 0]


def tune_subdomain(op: csdyn.Operator, b: torch.Tensor, precision: int = 1, restart: int = 30, rtol: float = 1e-8,
                   log=None):
    """Fastest subdomain edge for this shell: one timed solve per candidate."""
    table = {}
    for s in candidate_subdomains(op.n, op.nr):
        t0 = time.perf_counter()
        pc = csdyn.RAS(op, sub=(s, s, s), levels=1, precision=precision)
        setup = time.perf_counter() - t0
        sol = csdyn.Solver(op, pc, restart=restart, maxit=5000, flexible=True, rtol=rtol)
        x = torch.zeros_like(b)
        sol.solve(b, x.clone())  # warm-up (first launches)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, rc = sol.solve(b, x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        table[s] = dict(solve_ms=round(el * 1e3, 2), iters=st["iters"], setup_s=round(setup, 2), ok=rc == 0)
        if log:
            log(f"  N={op.n} sub {s}^3: {table[s]}")
        del pc, sol
    best = min((s for s in table if table[s]["ok"]), key=lambda s: table[s]["solve_ms"])
    return best, table


def tune_shell(op: csdyn.Operator, b: torch.Tensor, precision: int = 1, log=None):
    key = (op.n, op.nr, op.kind, op.dt, op.ekman, op.pm, precision)
    if key not in _cache:
        tile, tile_table = tune_tile(op)
        sub, sub_table = tune_subdomain(op, b, precision, log=log)
        _cache[key] = dict(tile=tile, sub=sub, tiles_us=tile_table, subdomains=sub_table)
    else:
        op.set_tile(_cache[key]["tile"])
    return _cache[key]
