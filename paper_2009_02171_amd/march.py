"""Time march that feeds the learned initial guess.  With dynamics = "full"
the step is the paper's semi-implicit step (Sec. 3.1, Steps 1-3, step.py:
nonlinear terms, Adams-Bashforth, Crank-Nicolson right-hand sides) from the
benchmark's initial field; with the default "surrogate" it is the step
without its nonlinear terms, driven by a drifting forcing, as follows.

Per step n and per system (VP: velocity / pressure, BP: magnetic field /
pseudo-pressure), with a longitudinally drifting forcing
f^n = F(r, theta, phi - n * drift):

    b^n = (v^{n-1} + dt f^n, 0)          v = u (VP) or B (BP), projected
    A x^n = b^n                          FGMRES(30) + two-level RAS, to
                                         ||b - A x|| <= 1e-8 ||b||
    v^n = Step 3 of x^n                  csdyn_project

The solve's initial guess is one of
    (a) x^{n-1}                          (the paper's choice, Sec. 3.3)
    (b) 2 x^{n-1} - x^{n-2}              (linear extrapolation)
    (c) the network's guess, or (b) when (b) has the smaller ||b - A x0||
    (d) (b) + alpha (network's guess - (b)), alpha minimising ||b - A x0||
    (e) the network's guess as it is (its error, not its residual, decides
        what the solve has left to do)
Steps 1..train_steps advance with guess (b) and train one network per
system online (Adam on a replay buffer of the latest samples); the network
is then frozen and steps train_steps+1.. are solved from the same state with
every guess, the FP64 preconditioner for (a) ("plain") and the FP32 one for
(a) .. (e); the plain solution advances the state.  Every solve must reach
the tolerance whatever its guess.  Right-hand sides, guesses and the Step-3
state come from the library (csdyn_march_rhs, csdyn_guess, csdyn_project);
the forcing is generated on the host with the other synthetic inputs.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import csdyn, inputs

DRIFT = 0.02  # rad per step, fixed before training (about one cell per step at N = 64)


def _sync():
    torch.cuda.synchronize()


class _System:
    def __init__(self, kind, n, nr, sub, levels, dt, ekman, pm, net_seed, widths, dev, op=None):
        self.kind = kind
        self.op = op if op is not None else csdyn.Operator(n, nr, kind=kind, dt=dt, ekman=ekman, pm=pm, device=dev)
        self.pc = {p: csdyn.RAS(self.op, sub=sub, levels=levels, coarse_rtol=0.1, coarse_restart=30,
                                coarse_maxit=200, precision=p) for p in (0, 1)}
        self.sol = {p: csdyn.Solver(self.op, self.pc[p], restart=30, maxit=3000, flexible=True, rtol=1e-8,
                                    rhs_relative=True) for p in (0, 1)}
        self.guess = csdyn.Guess(self.op)
        self.net = csdyn.Net(n, nr, torch.from_numpy(inputs.net_params(net_seed, widths)).to(dev), widths=widths)
        self.state = self.op.empty().zero_()
        self.hist = []  # latest solutions, newest last

    def rhs(self, f, dt):
        return csdyn.march_rhs(self.op, self.state, f, dt)


def run(n=64, nr=64, sub=(16, 16, 16), levels=2, train_steps=100, eval_steps=100, train_iters=8, replay=16,
        lr=5e-4, dt=1e-4, ekman=1e-3, pm=5.0, forcing_seed=4, widths=inputs.NET_WIDTHS, log=print,
        dev="cuda", dynamics="surrogate", force_amp=0.0, ra=100.0, pr=1.0):
    """dynamics = "surrogate": b^n = (v^{n-1} + dt f^n, 0) with the drifting
    forcing (the systems decoupled); "full": the semi-implicit step of Sec. 3.1
    (step.SemiImplicit: nonlinear terms, Adams-Bashforth, Crank-Nicolson
    right-hand sides) from the benchmark's initial magnetic field and u = 0,
    with the drifting field times force_amp as a body force on the velocity;
    "thermal": the same step with the temperature (the VT solve first, from
    the previous solution with the FP64 preconditioner, then the pressure from
    the VP system) from the benchmark's initial Theta and B.  The learned and
    classical guesses are compared on the VP and BP solves."""
    dev = torch.device(dev)
    rng = np.random.default_rng(forcing_seed + 1000)
    sim = None
    if dynamics in ("full", "thermal"):
        from . import step as step_mod
        thermal = dynamics == "thermal"
        sim = step_mod.SemiImplicit(n, nr, dt=dt, ekman=ekman, pm=pm, solvers=False, temperature=thermal, ra=ra,
                                    pr=pr, b0=torch.from_numpy(inputs.benchmark_b0(n, nr)).to(dev),
                                    theta0=(torch.from_numpy(inputs.benchmark_theta0(n, nr)).to(dev)
                                            if thermal else None), device=dev)
        if thermal:
            vt_pc = csdyn.RAS(sim.vt, sub=sub, levels=1)
            vt_sol = csdyn.Solver(sim.vt, vt_pc, restart=30, maxit=3000, flexible=False, rtol=1e-8,
                                  rhs_relative=True)
    elif dynamics != "surrogate":
        raise ValueError(f"dynamics must be 'surrogate', 'full' or 'thermal', not {dynamics!r}")
    systems = {"VP": _System(csdyn.VP, n, nr, sub, levels, dt, ekman, pm, 5, widths, dev,
                             op=sim.vp if sim else None),
               "BP": _System(csdyn.BP, n, nr, sub, levels, dt, ekman, pm, 6, widths, dev,
                             op=sim.bp if sim else None)}
    forcing = inputs.DriftingField(n, nr, forcing_seed)

    def force(step):  # synthetic input, generated on the host
        return torch.from_numpy(forcing.field(DRIFT * step)).to(dev)

    variants = ("plain_a", "mixed_a", "mixed_b", "mixed_c", "mixed_d", "mixed_e")
    acc = {name: {v: dict(iters=0, inner=0, solve_s=0.0, guess_s=0.0, res0_rel=[], solves=0, relres=[])
                  for v in variants} for name in systems}
    chosen_net = {name: 0 for name in systems}
    netd = {name: {k: [] for k in ("err_net", "err_extrap", "err_prev", "res_net", "res_extrap", "res_minres",
                                   "alpha")} for name in systems}
    div = {name: [] for name in systems}
    train_s, losses = 0.0, {name: [] for name in systems}

    def solve(s, b, x0, prec):
        x = x0.clone()
        _sync()
        t0 = time.perf_counter()
        _, st, rc = s.sol[prec].solve(b, x)
        _sync()
        el = time.perf_counter() - t0
        if rc != 0 or not st["res_true"] <= 1.0001e-8 * st["bnorm"]:
            raise RuntimeError(f"solve did not reach 1e-8: rc={rc} {st}")
        return x, st, el

    pending = {}
    vt_iters = []

    def advance(s, x, name, bnorm):
        out = s.op.project(x)
        if sim is None:
            s.state.copy_(out)
        else:
            pending[name] = x
        div[name].append(float(torch.linalg.norm(out[..., 3])) / bnorm)
        s.hist.append(x)
        del s.hist[:-(replay + 2)]

    total = train_steps + eval_steps
    for step in range(1, total + 1):
        f = force(step) if sim is None or force_amp else None
        if sim is not None:
            sim.force, sim.force_scale = (f, force_amp) if force_amp else (None, 1.0)
            bs, fterms = sim.rhs()
            if sim.temperature:  # Step 1's VT solve, then Step 2's right-hand side
                xvt = sim.x["VT"].clone()
                _, st_vt, rc = vt_sol.solve(bs["VT"], xvt)
                if rc != 0:
                    raise RuntimeError(f"VT solve did not converge: {st_vt}")
                vt_iters.append(st_vt["iters"])
                pending["VT"] = xvt
                bs["VP"] = sim.pressure_rhs(xvt)
        for name, s in systems.items():
            b = s.rhs(f, dt) if sim is None else bs[name]
            h = s.hist
            if step <= train_steps:
                x0 = s.guess(h[-1], h[-2])[0] if len(h) >= 2 else (h[-1].clone() if h else torch.zeros_like(b))
                x, st, _ = solve(s, b, x0, 1)
                advance(s, x, name, st["bnorm"])
                if len(s.hist) >= 3:
                    _sync()
                    t0 = time.perf_counter()
                    nsamp = len(s.hist) - 2
                    for _ in range(train_iters):
                        i = int(rng.integers(0, nsamp))
                        s.net.train_step(s.hist[i], s.hist[i + 1], s.hist[i + 2], lr=lr, want_loss=False)
                    losses[name].append(s.net.train_step(s.hist[-3], s.hist[-2], s.hist[-1], lr=lr))
                    _sync()
                    train_s += time.perf_counter() - t0
                continue
            # evaluation: the same b^n from every guess
            A = acc[name]
            bn = None
            for v in variants:
                _sync()
                t0 = time.perf_counter()
                if v in ("plain_a", "mixed_a"):
                    x0 = h[-1].clone()
                elif v == "mixed_b":
                    x0, _ = s.guess(h[-1], h[-2], csdyn.GUESS_EXTRAPOLATE)
                elif v == "mixed_c":
                    x0, gi = s.guess(h[-1], h[-2], csdyn.GUESS_FALLBACK, net=s.net, b=b)
                    chosen_net[name] += int(gi["alpha"] == 1.0)
                    netd[name]["res_net"].append(gi["res_net"])
                    netd[name]["res_extrap"].append(gi["res_extrap"])
                elif v == "mixed_d":
                    x0, gi = s.guess(h[-1], h[-2], csdyn.GUESS_MINRES, net=s.net, b=b)
                    netd[name]["res_minres"].append(gi["res_guess"])
                    netd[name]["alpha"].append(gi["alpha"])
                else:  # the network's guess as it is, whatever its residual
                    x0 = s.net.predict(h[-1], h[-2])
                _sync()
                tg = time.perf_counter() - t0
                x, st, el = solve(s, b, x0, 0 if v == "plain_a" else 1)
                A[v]["iters"] += st["iters"]
                A[v]["inner"] += st["inner_iters"]
                A[v]["solve_s"] += el
                A[v]["guess_s"] += tg
                A[v]["solves"] += 1
                A[v]["res0_rel"].append(st["res0"] / st["bnorm"])
                A[v]["relres"].append(st["res_true"] / st["bnorm"])
                if v == "plain_a":
                    bn = x
            # measurement only: the network's own guess and extrapolation against the
            # solution (error norms) and their residuals, relative to ||b||
            nrm = float(torch.linalg.norm(bn))
            xe, _ = s.guess(h[-1], h[-2])
            xg = s.net.predict(h[-1], h[-2])
            netd[name]["err_net"].append(float(torch.linalg.norm(xg - bn)) / nrm)
            netd[name]["err_extrap"].append(float(torch.linalg.norm(xe - bn)) / nrm)
            netd[name]["err_prev"].append(float(torch.linalg.norm(h[-1] - bn)) / nrm)
            for k in ("res_net", "res_extrap", "res_minres"):
                netd[name][k][-1] /= st["bnorm"]
            advance(s, bn, name, st["bnorm"])
        if sim is not None:
            sim.advance(pending, fterms)
        if step % 10 == 0 or step == total:
            log(f"step {step}/{total} done")

    out = {"n": n, "nr": nr, "dynamics": dynamics, "force_amp": force_amp if sim is not None else None,
           "vt_iters_mean": float(np.mean(vt_iters)) if vt_iters else None,
           "state_absmax": ({name: float(sim.state[name][..., :3].abs().max()) for name in systems}
                            if sim is not None else None),
           "train_steps": train_steps, "eval_steps": eval_steps, "drift_rad_per_step": DRIFT,
           "train_s": train_s, "param_count": systems["VP"].net.nparam, "systems": {}}
    for name in systems:
        r = {}
        for v in variants:
            a = acc[name][v]
            t = a["solve_s"] + a["guess_s"]
            r[v] = dict(solves=a["solves"], iters_mean=a["iters"] / max(a["solves"], 1),
                        inner_mean=a["inner"] / max(a["solves"], 1), solves_per_s=a["solves"] / t if t else None,
                        solve_s=a["solve_s"], guess_s=a["guess_s"],
                        res0_rel_median=float(np.median(a["res0_rel"])) if a["res0_rel"] else None,
                        relres_max=float(max(a["relres"])) if a["relres"] else None)
        r["net_chosen"] = chosen_net[name]
        r["guess_quality_median"] = {k: float(np.median(v)) for k, v in netd[name].items() if v}
        r["loss_first"] = losses[name][0] if losses[name] else None
        r["loss_last"] = losses[name][-1] if losses[name] else None
        r["face_div_rel_max"] = max(div[name]) if div[name] else None
        out["systems"][name] = r
    tot = {}
    for v in variants:
        s_ = sum(out["systems"][k][v]["solves"] for k in systems)
        t_ = sum(out["systems"][k][v]["solve_s"] + out["systems"][k][v]["guess_s"] for k in systems)
        tot[v] = s_ / t_ if t_ else None
    out["solves_per_s"] = tot
    out["speedup_mixed_c_vs_plain_a"] = tot["mixed_c"] / tot["plain_a"] if tot["plain_a"] else None
    out["speedup_mixed_d_vs_plain_a"] = tot["mixed_d"] / tot["plain_a"] if tot["plain_a"] else None
    return out
