#!/usr/bin/env python
"""Benchmark: GMRES solves per second to relative residual 1e-8 on one MI355X.

Workload (default, "large"): both systems of the approximate-factorization
step -- velocity-pressure (E = 1e-3, dt = 1e-4) and magnetic / pseudo-
pressure (Pm = 5) -- on the cubed-sphere shell with N = Nr = 96 (5,308,416
cells, 21.2M unknowns per system), preconditioned by the hybrid two-level
RAS (384 subdomains of 24^3 cells, overlap 1, ILU(0); coarse grid 48^3 x 6
solved by GMRES(30) to 0.1 with a one-level RAS of 384 subdomains of 12^3),
flexible GMRES(30) from x0 = 0 to relative residual 1e-8, FP64 throughout.
Right-hand sides: seeded spherical-harmonic x Chebyshev fields plus noise
(seeds 1 and 2), already resident in HBM when timing starts.

One step = one velocity-pressure solve + one magnetic solve.  The timed
region is bracketed by torch.cuda.synchronize(); inside it one launch in
eight of the dominant kernel and of the stencil operator is also timed with
HIP events on its own stream (csdyn_profile_*), which gives their average
durations and achieved algorithmic bandwidth.  Timing every launch costs
about 14% of the step, so the per-kernel breakdown ("kernels") comes from
one extra untimed step in which every launch is timed; the dominant kernel
is the one with the largest total time there.  The event pool is created
before the clock starts and read after it stops.  The forms "*_two_streams"
time the same steps with the two systems (independent of each other) solved
at the same time, each from its own host thread on its own stream.

The default run also carries the other halves of the metric: the small
configuration (N = Nr = 16, one-level RAS, GMRES(30)) and a bounded run of
the learned-guess march (N = Nr = 64, 30 training and 30 evaluation steps by
default) with plain FP64 from the previous solution against the FP32
preconditioner from extrapolation and from the network's guess.  Per-phase
times of one extra step of each form ("phases_ms") come from HIP events
around the outer operator, the fine sweeps (PC-F), the coarse solve (PC-C)
and the transfers (PC-I).

The CPU baseline is the plain C oracle (single-threaded), timed on a bounded
sample: the same two solves with the same solver and subdomain count at
N = Nr = 32, on one thread and as independent solves on all host cores (one
process each), scaled to N = 96 by the cell ratio (27x) times the ratio of
GPU to oracle iterations (outer + inner) per system.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROFILE_EVERY = 8  # in the timed region, one launch in 8 of the timed kernels carries events
METRIC = "GMRES solves/s to rel.res 1e-8 (plain FP64 vs mixed+learned); operator HBM GB/s"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "large": dict(n=96, nr=96, sub=(24, 24, 24), levels=2, flexible=True,
                  desc="VP+BP solves, N=Nr=96 (5.31M cells), two-level RAS 384x24^3 + coarse 48^3x6, FGMRES(30)"),
    "small": dict(n=16, nr=16, sub=(16, 16, 16), levels=1, flexible=False,
                  desc="VP+BP solves, N=Nr=16 (24,576 cells), one-level RAS 6x16^3, GMRES(30)"),
    "batched": dict(n=80, nr=80, ns=(24, 32, 40, 48, 56, 64, 72, 80),
                    desc="8 VP shells, N=Nr in {24,...,80} (9.27M cells), E log-uniform in [1e-4, 1e-3], one-level FP32 "
                         "RAS with autotuned subdomains and stencil tiles, FGMRES(30) to 1e-8, lock-step batch, one "
                         "hipGraph per Arnoldi step"),
    "paper_mesh": dict(n=144, nr=168, sub=(24, 24, 28), levels=2, flexible=True,
                       desc="VP and BP solves on the strong-scaling mesh of the paper, N=144, Nr=168 (20.9M cells, "
                            "83.6M unknowns per system), 1296 subdomains of 24x24x28 (the paper's 1296-core split), "
                            "two- and three-level RAS, FGMRES(30), the paper's tolerance pairs, case P8 "
                            "(E=1e-3, Pm=8) at Delta t=1e-5"),
    "learned": dict(n=64, nr=64, sub=(16, 16, 16), levels=2, flexible=True,
                    desc="200-step VP+BP march, N=Nr=64 (1.57M cells), two-level RAS 384x16^3 + coarse 32^3x6, "
                         "FGMRES(30) to ||r|| <= 1e-8 ||b||; train on steps 1-100, evaluate 101-200"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel_key):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (profiles/traffic.json, calibrated); None when the kernel's
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    h = hashlib.sha1()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["sources_sha1"] else None


def _oracle_run(n, sub, levels, procs):
    """The oracle's timing runner in a child process of its own (no GPU state)."""
    import subprocess
    r = subprocess.run([sys.executable, "-m", "oracle.baseline", "--n", str(n), "--sub", str(sub), "--levels",
                        str(levels), "--procs", str(procs)], cwd=ROOT, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"oracle baseline failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(wl_name: str, gpu_iters: dict):
    """The oracle (plain C, single-threaded) on a bounded sample of the workload:
    the same VP and BP solves with the same solver and subdomain count at
    N = Nr = 32, timed on one thread and as independent solves on all host cores
    (one process per core), scaled to the full size by the cell ratio times the
    ratio of GPU to oracle iterations (outer + inner) per system."""
    wl = WORKLOADS[wl_name]
    n, sub = (32, 8) if wl_name == "large" else (wl["n"], wl["sub"][0])
    cells = (wl["n"] / n) ** 2 * (wl["nr"] / n)
    one = _oracle_run(n, sub, wl["levels"], 1)
    p1 = one["per_process"][0]
    full_s, factors = 0.0, {}
    for name in ("VP", "BP"):
        o = p1[name]
        it = (gpu_iters[name][0] + gpu_iters[name][1]) / (o["outer"] + o["inner"])
        factors[name] = dict(oracle_iters=[o["outer"], o["inner"]], gpu_iters=list(gpu_iters[name]),
                             iteration_factor=round(it, 4), sample_s=round(o["s"], 3))
        full_s += o["s"] * cells * it
    scale = full_s / p1["s"]  # effective sample-to-full-size factor of one VP + BP pair
    procs = max(1, min(16, os.cpu_count() or 1))
    many = _oracle_run(n, sub, wl["levels"], procs)
    rate_all = 2 * procs / many["wall_s"] / scale
    log(f"oracle N={n}: one thread {p1['s']:.2f} s per VP+BP pair; {procs} processes {many['wall_s']:.2f} s; "
        f"scale {scale:.1f} (cells {cells:.0f} x iterations {factors})")
    return {
        "value": rate_all, "unit": "solves/s", "cores": procs, "kind": "oracle",
        "sample": (f"VP+BP solves at N=Nr={n} ({wl['levels']}-level RAS, {sub}^3 boxes, to 1e-8), {procs} independent "
                   f"processes on {procs} host cores ({many['wall_s']:.2f} s wall for {2 * procs} solves), scaled to "
                   f"N=Nr={wl['n']} by the cell ratio {cells:.0f} x the per-system ratio of GPU to oracle "
                   f"iterations (outer + inner): effective factor {scale:.1f}"),
        "single_thread": {"value": 2.0 / full_s, "unit": "solves/s", "cores": 1, "sample_s": round(p1["s"], 3)},
        "scaling": {"cells": cells, "systems": factors, "effective": round(scale, 2)},
        "cpu": _cpu_model(),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical cpus)"
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="large")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-two-streams", action="store_true",
                    help="skip the forms with the two systems on two streams (a profiler's per-kernel averages "
                         "then cover sequential launches only)")
    ap.add_argument("--train-steps", type=int, default=100, help="learned workload: training steps")
    ap.add_argument("--eval-steps", type=int, default=100, help="learned workload: evaluation steps")
    ap.add_argument("--learned-train-steps", type=int, default=30,
                    help="large workload: training steps of the bounded learned-guess leg (0 with "
                         "--learned-eval-steps 0 skips it)")
    ap.add_argument("--learned-eval-steps", type=int, default=30,
                    help="large workload: evaluation steps of the bounded learned-guess leg")
    ap.add_argument("--no-small", action="store_true", help="large workload: skip the small-configuration leg")
    ap.add_argument("--dynamics", choices=("surrogate", "full", "thermal"), default="surrogate",
                    help="learned march: the step without nonlinear terms driven by a drifting forcing, the "
                         "semi-implicit step with nonlinear terms from the benchmark's initial field, or that "
                         "step with the temperature")
    ap.add_argument("--no-three-level", action="store_true", help="large workload: skip the three-level forms")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the solver is single-GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_02171_amd import csdyn, inputs

    wl = WORKLOADS[args.workload]
    n, nr = wl["n"], wl["nr"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "learned":
        return learned(args, wl)
    if args.workload == "paper_mesh":
        return paper_mesh(args, wl)
    if args.workload == "batched":
        return batched(args, wl)
    systems = {"VP": dict(kind=csdyn.VP, seed=1), "BP": dict(kind=csdyn.BP, seed=2)}
    # form -> (precision inside the preconditioner, levels); the three-level forms repeat the hybrid
    # construction on the coarse grid (the paper's extension for larger meshes)
    forms = {"plain_fp64": (0, wl["levels"]), "mixed_fp32_pc": (1, wl["levels"])}
    if args.workload == "large" and not args.no_three_level:
        forms.update({"plain_fp64_3level": (0, 3), "mixed_fp32_3level": (1, 3)})
    state = {f: {} for f in forms}
    setup_s = {f: {} for f in forms}  # preconditioner setup (host build and upload), timed apart from the solves
    for name, s in systems.items():
        t0 = time.perf_counter()
        op = csdyn.Operator(n, nr, kind=s["kind"], dt=1e-4, ekman=1e-3, pm=5.0)
        b = torch.from_numpy(inputs.rhs(n, nr, s["seed"])).to(dev)
        for form, (prec, levels) in forms.items():
            t1 = time.perf_counter()
            pc = csdyn.RAS(op, sub=wl["sub"], levels=levels, coarse_rtol=0.1, coarse_restart=30,
                           coarse_maxit=200, precision=prec)
            torch.cuda.synchronize()
            setup_s[form][name] = round(time.perf_counter() - t1, 2)
            flexible = wl["flexible"] or prec == 1
            sol = csdyn.Solver(op, pc, restart=30, maxit=2000, flexible=flexible, rtol=1e-8)
            state[form][name] = dict(op=op, pc=pc, sol=sol, b=b, x=torch.zeros_like(b), info=pc.info())
        log(f"setup {name}: {time.perf_counter() - t0:.1f} s, info {state['plain_fp64'][name]['info']}")
    torch.cuda.synchronize()

    iters = {f: {} for f in forms}

    def step(form):
        for name, s in state[form].items():
            s["x"].zero_()
            _, st, rc = s["sol"].solve(s["b"], s["x"])
            if rc != 0 or not st["relres_true"] <= 1.0001e-8:
                raise RuntimeError(f"{form} {name} solve did not converge: rc={rc} {st}")
            iters[form][name] = [st["iters"], st["inner_iters"], st["relres_true"], st["inner2_iters"]]

    streams = {name: torch.cuda.Stream() for name in systems}  # default priority

    def solve_on_stream(form, name, failures):
        s = state[form][name]
        try:
            with torch.cuda.stream(streams[name]):
                s["x"].zero_()
                _, st, rc = s["sol"].solve(s["b"], s["x"], stream=streams[name])
            if rc != 0 or not st["relres_true"] <= 1.0001e-8:
                raise RuntimeError(f"{form} {name} solve did not converge: rc={rc} {st}")
            iters[form][name] = [st["iters"], st["inner_iters"], st["relres_true"], st["inner2_iters"]]
        except Exception as e:  # reported by the caller
            failures.append(e)

    def step_two_streams(form):
        failures = []
        threads = [threading.Thread(target=solve_on_stream, args=(form, name, failures)) for name in state[form]]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if failures:
            raise failures[0]

    for form in forms:
        for w in range(args.warmup):
            t0 = time.perf_counter()
            step(form)
            torch.cuda.synchronize()
            log(f"warmup {form} step {w}: {time.perf_counter() - t0:.3f} s, iters {iters[form]}")

    # per-phase times of one untimed step of each form (HIP events around the outer operator, the fine
    # sweeps, the coarse solve, the transfers and the Gram-Schmidt; the rest of the span is "other")
    phases = {f: {} for f in forms}
    for form in forms:
        for name, s in state[form].items():
            s["sol"].opts.timing = 1
            s["x"].zero_()
            _, st, rc = s["sol"].solve(s["b"], s["x"])
            s["sol"].opts.timing = 0
            phases[form][name] = {k: round(v, 3) for k, v in st["t_ms"].items()}
            phases[form][name]["span_ms"] = round(st["t_span_ms"], 3)
    log(f"phases (ms): {phases}")

    # per-kernel breakdown: one untimed plain FP64 step with every launch timed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with csdyn.Profile() as prof_all:
        step("plain_fp64")
        torch.cuda.synchronize()
    elapsed_all = time.perf_counter() - t0
    dom_kernel = max(prof_all.result.items(), key=lambda kv: kv[1]["ms"])[0][0]
    log(f"profiled plain_fp64 step: {elapsed_all:.3f} s, dominant kernel {dom_kernel}")
    # the headline form: plain FP64; the dominant kernel and the operator timed with HIP events.  The
    # event pool is created before the clock starts and read after it stops (creating and destroying
    # the events is host work that is not part of a step).
    prof = csdyn.Profile(max_launches=16384, select=[dom_kernel, "op_main"], every=PROFILE_EVERY)
    prof.__enter__()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step("plain_fp64")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof.__exit__(None, None, None)
    log(f"timed plain_fp64: {args.steps} steps in {elapsed:.3f} s, iters {iters['plain_fp64']}")
    # the other forms: FP32 inside the preconditioner (FP64 FGMRES), and the three-level hybrids
    elapsed_form = {}
    for form in forms:
        if form == "plain_fp64":
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(form)
        torch.cuda.synchronize()
        elapsed_form[form] = time.perf_counter() - t0
        log(f"timed {form}: {args.steps} steps in {elapsed_form[form]:.3f} s, iters {iters[form]}")
    elapsed_mixed = elapsed_form["mixed_fp32_pc"]
    # the two-level forms again with the two systems of a step solved at the same time, each from its own
    # host thread on its own stream (the systems are independent; results are identical)
    elapsed_two = {}
    for form in ([] if args.no_two_streams else ("plain_fp64", "mixed_fp32_pc")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step_two_streams(form)
        torch.cuda.synchronize()
        elapsed_two[form] = time.perf_counter() - t0
        log(f"timed {form} on two streams: {args.steps} steps in {elapsed_two[form]:.3f} s, iters {iters[form]}")
    err = {f: {} for f in forms if f != "plain_fp64"}
    for f in err:
        for name in systems:
            xp, xm = state["plain_fp64"][name]["x"], state[f][name]["x"]
            err[f][name] = float(torch.linalg.norm(xm - xp) / torch.linalg.norm(xp))
    iters_plain = iters["plain_fp64"]

    kernels = {}
    for (name, size), e in sorted(prof_all.result.items(), key=lambda kv: -kv[1]["ms"]):
        avg_ms = e["ms"] / max(e["count"], 1)
        gbs = e["bytes"] / (e["ms"] * 1e-3) / 1e9 if e["ms"] > 0 else 0.0
        kernels[f"{name}@{size}"] = dict(launches=e["count"], total_ms=round(e["ms"], 3), avg_us=round(avg_ms * 1e3, 2),
                                         alg_GBs=round(gbs, 1), share=round(e["ms"] / (elapsed_all * 1e3), 4))
    dom_name, dom = max(prof.result.items(), key=lambda kv: kv[1]["ms"])
    dom_gbs = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    op_key = [k for k in prof.result if k[0] == "op_main" and k[1] == 6 * n * n * nr]
    operator = None
    if op_key:
        e = prof.result[op_key[0]]
        g = e["bytes"] / (e["ms"] * 1e-3) / 1e9
        operator = dict(kernel="op_main", cells=6 * n * n * nr, avg_us=round(e["ms"] / e["count"] * 1e3, 2),
                        achieved=round(g, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(g / HBM_PEAK_GBS, 4),
                        bytes_per_cell=64)

    out = {
        "metric": METRIC,
        "value": round(2 * args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "nr": nr, "systems": ["VP", "BP"], "subdomain": list(wl["sub"]),
                   "levels": wl["levels"], "krylov": "FGMRES(30)" if wl["flexible"] else "GMRES(30)",
                   "rtol": 1e-8, "form": "plain FP64"},
        "iters": {k: {"outer": v[0], "inner": v[1], "relres": v[2]} for k, v in iters_plain.items()},
        "forms": {
            "plain_fp64": {"solves_per_s": round(2 * args.steps / elapsed, 4),
                           "ms_per_step": round(elapsed / args.steps * 1e3, 3)},
            **{f: {"solves_per_s": round(2 * args.steps / el, 4), "ms_per_step": round(el / args.steps * 1e3, 3),
                   "precision": "fp32 preconditioner" if forms[f][0] else "fp64", "levels": forms[f][1],
                   "iters": {k: {"outer": v[0], "inner": v[1], "coarsest": v[3], "relres": v[2]}
                             for k, v in iters[f].items()},
                   "rel_err_vs_plain_fp64_solution": err[f]}
               for f, el in elapsed_form.items()},
            **{f"{form}_two_streams": {"solves_per_s": round(2 * args.steps / el, 4),
                                       "ms_per_step": round(el / args.steps * 1e3, 3)}
               for form, el in elapsed_two.items()},
        },
        "roofline": {"kernel": f"{dom_name[0]}@{dom_name[1]}", "bound": "hbm", "achieved": round(dom_gbs, 1),
                     "timed_launches": dom["count"], "timed_every": PROFILE_EVERY,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(f"{dom_name[0]}@{dom_name[1]}"),
                     "avg_us": round(dom["ms"] / dom["count"] * 1e3, 2),
                     "alg_bytes_per_launch": round(dom["bytes"] / dom["count"])},
        "operator": operator,
        "phases_ms": phases,
        "setup_s": setup_s,
        "setup_note": ("RAS setup per form and system: assembly, ILU(0) factorization, level schedules and packing "
                       "on the host cores, then the upload; a form with the FP32 preconditioner reuses the host "
                       "build of the FP64 form with the same levels"),
        "kernels": kernels,
        "kernels_from": "one untimed plain FP64 step with every launch timed (share = of that step)",
    }
    outer = sum(v[0] for v in iters_plain.values())
    out["us_per_outer_iteration"] = round(elapsed / args.steps / outer * 1e6, 2)
    if args.workload == "large":
        out["operator_n128"] = operator_rate(128, 128)
        out["hbm_copy"] = copy_rate()
    if args.workload == "large" and not args.no_small:
        out["small_config"] = small_leg(args)
    if args.workload == "large" and args.learned_train_steps + args.learned_eval_steps > 0:
        out["learned"] = learned_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, {k: v[:2] for k, v in iters_plain.items()})
    print(json.dumps(out))


# The paper's numbers on this mesh (Table strong, 1296 to 10368 cores, Sunway TaihuLight): context only.
PAPER_DT = 1e-5  # Table strong's time step (viscous time units)
PAPER_STRONG = {"cores": [1296, 2592, 5184, 10368],
                "VTBE": {"iters": [3.0, 3.0, 3.0, 3.0], "time_s": [6.65, 3.41, 1.77, 0.92]},
                "PPBE_1level": {"iters": [144.9, 154.0, 158.0, 151.1], "time_s": [29.69, 16.90, 9.60, 5.24]},
                "PPBE_2level": {"iters": [22.0, 22.2, 22.1, 22.4], "inner": [13.4, 16.0, 14.0, 16.1],
                                "time_s": [15.80, 10.18, 5.72, 4.20]}}


def paper_mesh(args, wl):
    """Solves on the paper's strong-scaling mesh with its subdomain split, for
    context next to its Table strong.  The paper's systems (VTBE with u, Theta, B;
    PPBE with P, P_b) are not this build's (VP and BP, each one block-triangular
    4-unknown system), so both of ours are solved with both of the paper's
    tolerance pairs: (rtol 1e-8, atol 1e-10) as for its VTBE, (rtol 1e-6,
    atol 1e-8) as for its PPBE.  One preconditioner at a time (device memory)."""
    import torch
    from paper_2009_02171_amd import csdyn, inputs
    n, nr, sub = wl["n"], wl["nr"], wl["sub"]
    tols = {"vtbe_tol": (1e-8, 1e-10), "ppbe_tol": (1e-6, 1e-8)}
    forms = {"plain_fp64_2level": (0, 2), "plain_fp64_3level": (0, 3), "mixed_fp32_3level": (1, 3)}
    res = {}
    for name, kind, seed in (("VP", csdyn.VP, 1), ("BP", csdyn.BP, 2)):
        # case P8 (E = 1e-3, Pm = 8) at the table's time step Delta t = 1e-5, i.e. dt = Delta t / (2 E)
        op = csdyn.Operator(n, nr, kind=kind, dt=PAPER_DT / (2 * 1e-3), ekman=1e-3, pm=8.0)
        b = torch.from_numpy(inputs.rhs(n, nr, seed)).cuda()
        x = torch.zeros_like(b)
        sol = None
        for form, (prec, levels) in forms.items():
            t0 = time.perf_counter()
            pc = csdyn.RAS(op, sub=sub, levels=levels, coarse_rtol=0.1, coarse_restart=30, coarse_maxit=200,
                           precision=prec)
            setup_s = time.perf_counter() - t0
            log(f"{name} {form}: setup {setup_s:.1f} s, info {pc.info()}")
            for tname, (rtol, atol) in tols.items():
                sol = csdyn.Solver(op, pc, restart=30, maxit=2000, flexible=True, rtol=rtol, atol=atol)
                times, st = [], None
                for rep in range(1 + max(1, args.steps)):
                    x.zero_()
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    _, st, rc = sol.solve(b, x)
                    torch.cuda.synchronize()
                    if rc != 0:
                        raise RuntimeError(f"{name} {form} {tname}: {st}")
                    if rep > 0:
                        times.append(time.perf_counter() - t1)
                med = sorted(times)[len(times) // 2]
                res.setdefault(form, {}).setdefault(name, {})[tname] = dict(
                    seconds=round(med, 4), iters=st["iters"], inner=st["inner_iters"], coarsest=st["inner2_iters"],
                    relres=st["relres_true"], setup_s=round(setup_s, 1))
                log(f"{name} {form} {tname}: {med:.3f} s, {st['iters']} iterations ({st['inner_iters']} inner, "
                    f"{st['inner2_iters']} coarsest)")
                del sol
            del pc
            torch.cuda.synchronize()
    print(json.dumps({
        "metric": METRIC, "workload": wl["desc"], "n": n, "nr": nr, "subdomain": list(sub), "subdomains": 1296,
        "n_gpus": 1, "dtype": "f64 solve", "data": "synthetic", "solves": res,
        "paper_table_strong_context": PAPER_STRONG,
        "note": ("context only: the paper's VTBE/PPBE systems, its machine (Sunway TaihuLight) and precision differ; "
                 "seconds are one solve each, median of the timed repetitions, preconditioner setup excluded"),
    }))


SMALL_DEVICE_STEPS = (0, 4, 8)  # 0: one host round trip per Arnoldi step; k: one per k steps


def small_leg(args, steps=20):
    """The small configuration (N = Nr = 16, one-level RAS with one subdomain per
    panel, GMRES(30), FP64): VP + BP solves, mean over `steps` steps, with the
    host forming each step's rotation (device_steps 0) and with device-resident
    steps read back once per 4 or 8 steps."""
    import torch
    from paper_2009_02171_amd import csdyn, inputs
    wl = WORKLOADS["small"]
    n = wl["n"]
    systems = []
    for kind, seed in ((csdyn.VP, 0), (csdyn.BP, 0)):
        op = csdyn.Operator(n, n, kind=kind, dt=1e-4, ekman=1e-3, pm=5.0)
        pc = csdyn.RAS(op, sub=wl["sub"], levels=1)
        b = torch.from_numpy(inputs.rhs(n, n, seed)).cuda()
        systems.append((op, pc, b, torch.zeros_like(b)))
    forms = {}
    for ds in SMALL_DEVICE_STEPS:
        sols = [(csdyn.Solver(op, pc, restart=30, maxit=2000, rtol=1e-8, device_steps=ds), b, x)
                for op, pc, b, x in systems]
        iters = {}

        def step():
            for (sol, b, x), name in zip(sols, ("VP", "BP")):
                x.zero_()
                _, st, rc = sol.solve(b, x)
                if rc != 0:
                    raise RuntimeError(f"small {name} did not converge: {st}")
                iters[name] = st["iters"]

        for _ in range(3):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        forms[f"device_steps_{ds}"] = {"solves_per_s": round(2 * steps / el, 3),
                                       "ms_per_step": round(el / steps * 1e3, 3), "iters": dict(iters)}
        log(f"small, device_steps {ds}: {forms[f'device_steps_{ds}']}")
    best = max(forms, key=lambda f: forms[f]["solves_per_s"])
    return {"workload": wl["desc"], "solves_per_s": forms[best]["solves_per_s"],
            "ms_per_step": forms[best]["ms_per_step"], "form": best, "iters": forms[best]["iters"],
            "steps": steps, "forms": forms}


def learned_leg(args):
    """A bounded run of the learned-guess march (N = Nr = 64, two-level RAS on
    16^3 boxes): train_steps steps with online training, then eval_steps steps
    solved from every guess; solves/s per form (guess time included, training
    time separate), iterations, and how often and how much the network's
    correction is used."""
    import torch
    from paper_2009_02171_amd import march
    wl = WORKLOADS["learned"]
    t0 = time.perf_counter()
    res = march.run(n=wl["n"], nr=wl["nr"], sub=wl["sub"], levels=wl["levels"], train_steps=args.learned_train_steps,
                    eval_steps=args.learned_eval_steps, log=log, dynamics=args.dynamics)
    torch.cuda.synchronize()
    sp = res["solves_per_s"]
    sysd = {}
    for name, r in res["systems"].items():
        sysd[name] = {v: {"iters": round(r[v]["iters_mean"], 2), "inner": round(r[v]["inner_mean"], 1),
                          "solves_per_s": round(r[v]["solves_per_s"], 3),
                          "res0_rel_median": r[v]["res0_rel_median"]}
                      for v in ("plain_a", "mixed_a", "mixed_b", "mixed_c", "mixed_d", "mixed_e")}
        sysd[name]["net_chosen"] = f"{r['net_chosen']}/{r['mixed_c']['solves']}"
        sysd[name]["guess_quality_median"] = r["guess_quality_median"]
    return {
        "workload": (f"VP+BP march N=Nr={wl['n']}, two-level RAS 384x16^3, FGMRES(30) to ||r|| <= 1e-8 ||b||; "
                     f"{args.learned_train_steps} training steps, {args.learned_eval_steps} evaluation steps; "
                     f"{args.dynamics} dynamics"),
        "forms": {"plain_a (FP64 PC, previous solution)": round(sp["plain_a"], 3),
                  "mixed_a (FP32 PC, previous solution)": round(sp["mixed_a"], 3),
                  "mixed_b (FP32 PC, extrapolation)": round(sp["mixed_b"], 3),
                  "mixed_c (FP32 PC, network with residual fallback)": round(sp["mixed_c"], 3),
                  "mixed_d (FP32 PC, minimal-residual step along the network's correction)": round(sp["mixed_d"], 3),
                  "mixed_e (FP32 PC, the network's guess as it is)": round(sp["mixed_e"], 3)},
        "speedup_mixed_c_vs_plain_a": round(res["speedup_mixed_c_vs_plain_a"], 3),
        "speedup_mixed_d_vs_plain_a": round(res["speedup_mixed_d_vs_plain_a"], 3),
        "speedup_mixed_b_vs_plain_a": round(sp["mixed_b"] / sp["plain_a"], 3),
        "speedup_mixed_e_vs_plain_a": round(sp["mixed_e"] / sp["plain_a"], 3),
        "systems": sysd, "train_s": round(res["train_s"], 2), "wall_s": round(time.perf_counter() - t0, 1),
    }


def operator_rate(n, nr, reps=20):
    """The stencil operator alone at a size no cache holds (N = Nr = 128:
    805 MB per apply), each launch timed with HIP events."""
    import torch
    from paper_2009_02171_amd import csdyn, inputs
    op = csdyn.Operator(n, nr, kind=csdyn.VP, dt=1e-4, ekman=1e-3)
    x = torch.from_numpy(inputs.random_field(op.shape, 7)).cuda()
    y = op.empty()
    for _ in range(3):
        op.apply(x, y)
    prof = csdyn.Profile(max_launches=256, select=["op_main"], every=1)
    prof.__enter__()
    for _ in range(reps):
        op.apply(x, y)
    torch.cuda.synchronize()
    prof.__exit__(None, None, None)
    e = prof.result[("op_main", 6 * n * n * nr)]
    g = e["bytes"] / (e["ms"] * 1e-3) / 1e9
    return dict(kernel="op_main", n=n, nr=nr, cells=6 * n * n * nr, avg_us=round(e["ms"] / e["count"] * 1e3, 2),
                achieved=round(g, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(g / HBM_PEAK_GBS, 4))


def copy_rate(nbytes=1 << 30, reps=20):
    """Achievable HBM bandwidth for reference: a device-to-device copy of
    1 GiB (read + write counted), timed with events on the current stream."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    g = 2 * nbytes / (ms * 1e-3) / 1e9
    return dict(bytes_per_copy=2 * nbytes, avg_us=round(ms * 1e3, 1), achieved=round(g, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(g / HBM_PEAK_GBS, 4), kernel="torch device copy")


def batched(args, wl):
    """Eight uneven shells solved as one batch (hipGraph per Arnoldi step)
    against the same eight solves one after another."""
    import torch
    from paper_2009_02171_amd import autotune, csdyn, inputs
    ops, pcs, bs, tuned = [], [], [], {}
    t0 = time.perf_counter()
    for s, n in enumerate(wl["ns"]):
        ek, b = inputs.shell_case(s, n, n)
        op = csdyn.Operator(n, n, kind=csdyn.VP, dt=1e-4, ekman=ek, pm=5.0)
        bt = torch.from_numpy(b).cuda()
        tn = autotune.tune_shell(op, bt, precision=1, log=log)
        ops.append(op)
        bs.append(bt)
        pcs.append(csdyn.RAS(op, sub=(tn["sub"],) * 3, levels=1, precision=1))
        tuned[f"N={n}"] = dict(ekman=round(ek, 7), tile=autotune.TILES[tn["tile"]], sub=tn["sub"],
                               tiles_us=tn["tiles_us"], subdomains=tn["subdomains"])
        log(f"shell {s}: N={n} E={ek:.3e} tile {autotune.TILES[tn['tile']]} sub {tn['sub']}")
    tune_s = time.perf_counter() - t0
    solvers = [csdyn.Solver(op, pc, restart=30, maxit=5000, flexible=True, rtol=1e-8) for op, pc in zip(ops, pcs)]
    batch = csdyn.Batch(ops, pcs, restart=30, maxit=5000, rtol=1e-8)
    iters = {}

    def sequential():
        for i, (sol, b) in enumerate(zip(solvers, bs)):
            _, st, rc = sol.solve(b, torch.zeros_like(b))
            if rc != 0:
                raise RuntimeError(f"shell {i} did not converge: {st}")

    def run_batch(mode):
        xs = [torch.zeros_like(b) for b in bs]
        stats, rc = batch.solve(bs, xs, use_graph=mode)
        if rc != 0 or any(not st["res_true"] <= 1.0001e-8 * st["res0"] for st in stats):
            raise RuntimeError(f"batch did not converge: {stats}")
        iters[("eager", "graph", "phases", "persistent")[mode]] = [st["iters"] for st in stats]

    forms = {"sequential": sequential, "batched_eager": lambda: run_batch(csdyn.Batch.EAGER),
             "batched_graph": lambda: run_batch(csdyn.Batch.GRAPH)}
    if batch.available(csdyn.Batch.PHASES):
        forms["batched_phases"] = lambda: run_batch(csdyn.Batch.PHASES)
    if batch.persistent_available:
        forms["batched_persistent"] = lambda: run_batch(csdyn.Batch.PERSISTENT)
    timing = {}
    for name, fn in forms.items():
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        timing[name] = (time.perf_counter() - t1) / args.steps
        log(f"{name}: {timing[name] * 1e3:.1f} ms per batch of 8 solves")
    with csdyn.Profile() as prof:
        run_batch(csdyn.Batch.EAGER)
        torch.cuda.synchronize()
    dom_name, dom = max(prof.result.items(), key=lambda kv: kv[1]["ms"])
    phases = None
    if "batched_phases" in forms:
        with csdyn.Profile() as pprof:
            run_batch(csdyn.Batch.PHASES)
            torch.cuda.synchronize()
        phases = {}
        for kname in ("batch_ras_f32", "batch_op_edges", "batch_op_main", "batch_orth"):
            e = [v for k, v in pprof.result.items() if k[0] == kname]
            ms, by, cnt = sum(v["ms"] for v in e), sum(v["bytes"] for v in e), sum(v["count"] for v in e)
            phases[kname] = dict(launches=cnt, total_ms=round(ms, 2), avg_us=round(ms / max(cnt, 1) * 1e3, 2),
                                 alg_GBs=round(by / (ms * 1e-3) / 1e9, 1) if ms and by else None)
    dom_gbs = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    kernels = {f"{k[0]}@{k[1]}": dict(launches=v["count"], total_ms=round(v["ms"], 3),
                                      avg_us=round(v["ms"] / v["count"] * 1e3, 2),
                                      alg_GBs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] else None)
               for k, v in sorted(prof.result.items(), key=lambda kv: -kv[1]["ms"])[:16]}
    best = max((f for f in timing if f.startswith("batched")), key=lambda f: -timing[f])
    tg = timing[best]
    out = {
        "metric": METRIC, "value": round(8 / tg, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tg * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 solve, f32 preconditioner", "data": "synthetic",
        "config": {"workload": wl["desc"], "shells": list(wl["ns"]), "krylov": "FGMRES(30)", "rtol": 1e-8},
        "forms": {k: {"solves_per_s": round(8 / v, 4), "ms_per_batch": round(v * 1e3, 2)} for k, v in timing.items()},
        "form": best,
        "speedup_vs_sequential": round(timing["sequential"] / tg, 4),
        "speedup_graph_vs_sequential": round(timing["sequential"] / timing["batched_graph"], 4),
        "iters": {f"N={n}": it for n, it in zip(wl["ns"], iters["graph"])},
        "phase_launches": phases,
        "autotune": tuned, "autotune_s": round(tune_s, 1),
        "roofline": {"kernel": f"{dom_name[0]}@{dom_name[1]}", "bound": "hbm", "achieved": round(dom_gbs, 1),
                     "timed_launches": dom["count"], "timed_every": 1, "timed_in": "one extra eager batch",
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "kernels": kernels,
    }
    print(json.dumps(out))


def learned(args, wl):
    """The learned-guess comparison: plain FP64 solves from the previous
    solution against FP32-preconditioned solves from the network's guess."""
    import torch
    from paper_2009_02171_amd import csdyn, inputs, march
    t0 = time.perf_counter()
    res = march.run(n=wl["n"], nr=wl["nr"], sub=wl["sub"], levels=wl["levels"], train_steps=args.train_steps,
                    eval_steps=args.eval_steps, log=log, dynamics=args.dynamics)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the network's kernels, each launch timed with HIP events: 3 inferences and 3 training steps
    n, nr = wl["n"], wl["nr"]
    net = csdyn.Net(n, nr, torch.from_numpy(inputs.net_params(5)).cuda())
    xs = [torch.from_numpy(inputs.rhs(n, nr, seed)).cuda() for seed in (41, 42, 43)]
    net.predict(xs[1], xs[0])
    net.train_step(*xs, lr=1e-4)
    torch.cuda.synchronize()
    with csdyn.Profile() as prof:
        for _ in range(3):
            net.predict(xs[1], xs[0])
        for _ in range(3):
            net.train_step(*xs, lr=1e-4, want_loss=False)
        torch.cuda.synchronize()
    conv = {k: v for k, v in prof.result.items() if k[0].startswith("conv_")}
    fl = sum(v["flops"] for v in conv.values())
    ms = sum(v["ms"] for v in conv.values())
    dom_name, dom = max(conv.items(), key=lambda kv: kv[1]["ms"]) if conv else (("none", 0), None)
    kernels = {f"{k[0]}@{k[1]}": dict(launches=v["count"], total_ms=round(v["ms"], 3),
                                      avg_us=round(v["ms"] / v["count"] * 1e3, 2),
                                      TFLOPs=round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] else None)
               for k, v in sorted(conv.items(), key=lambda kv: -kv[1]["ms"])}
    sp = res["solves_per_s"]
    out = {
        "metric": METRIC,
        "value": round(sp["mixed_c"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.eval_steps,
        "warmup": args.train_steps,
        "ms_per_step": round(2e3 / sp["mixed_c"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 solve, f32 preconditioner, bf16 network",
        "data": "synthetic",
        "config": {"workload": f"{wl['desc']} ({args.train_steps} training + {args.eval_steps} evaluation steps here)",
                   "n": wl["n"], "nr": wl["nr"], "subdomain": list(wl["sub"]),
                   "levels": wl["levels"], "drift_rad_per_step": res["drift_rad_per_step"],
                   "network_params": res["param_count"], "dynamics": res["dynamics"]},
        "forms": {v: round(x, 4) for v, x in sp.items()},
        "speedup_mixed_learned_vs_plain": round(res["speedup_mixed_c_vs_plain_a"], 4),
        "systems": res["systems"],
        "train_s": round(res["train_s"], 2),
        "wall_s": round(elapsed, 1),
        "roofline": {"kernel": f"{dom_name[0]}@{dom_name[1]}", "bound": "mfma",
                     "achieved": round(dom["flops"] / (dom["ms"] * 1e-3) / 1e12, 2) if dom else None,
                     "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(dom["flops"] / (dom["ms"] * 1e-3) / 1e12 / 2500.0, 4) if dom else None,
                     "traffic": None, "all_conv_TFLOPs": round(fl / (ms * 1e-3) / 1e12, 2) if ms else None},
        "kernels": kernels,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
