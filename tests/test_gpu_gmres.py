"""GPU solve parity: csdyn_gmres_solve against the oracle's GMRES (Sec. 3.3).

Every solve reaches the relative residual 1e-8; the iteration count is
within +-1 of the oracle's and the solution within 1e-7 of the oracle's
(relative 2-norm; for the velocity-pressure system both sides return the
pressure with zero volume-weighted mean)."""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs

pytestmark = pytest.mark.gpu


def _gpu_solve(n, nr, kind, b, sub=None, levels=1, flexible=False, restart=30, maxit=2000, rtol=1e-8, orth=0,
               precision=0, **opkw):
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(n, nr, kind=kind, **opkw)
    pc = csdyn.RAS(op, sub=sub, levels=levels, precision=precision) if sub else None
    sol = csdyn.Solver(op, pc, restart=restart, maxit=maxit, flexible=flexible, rtol=rtol, orth=orth)
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    x, st, rc = sol.solve(bt)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st, rc


CASES = [
    # n, nr, kind, sub, levels, flexible, orth
    (16, 16, 0, (16, 16, 16), 1, False, 0),   # the small configuration: one subdomain per panel
    (16, 16, 0, (16, 16, 16), 1, False, 1),
    (16, 16, 1, (16, 16, 16), 1, False, 0),
    (16, 16, 0, (8, 8, 8), 2, True, 0),       # two-level hybrid, flexible GMRES
    (16, 16, 1, (8, 8, 8), 2, True, 1),
    (8, 8, 1, None, 1, False, 0),             # unpreconditioned
]


@pytest.mark.parametrize("n,nr,kind,sub,levels,flexible,orth", CASES)
def test_solve_matches_oracle(n, nr, kind, sub, levels, flexible, orth):
    print(f"[gmres parity] n={n} kind={kind} sub={sub} levels={levels} orth={orth}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    b = inputs.rhs(n, nr, seed=0)
    pc = O.Preconditioner(pb, sub=sub, levels=levels) if sub else None
    x_ref, st_ref, rc_ref = O.gmres(pb, b, pc=pc, flexible=flexible, maxit=2000)
    assert rc_ref == 0
    x, st, rc = _gpu_solve(n, nr, kind, b, sub=sub, levels=levels, flexible=flexible, orth=orth)
    assert rc == 0, st
    assert st["relres_true"] <= 1.0001e-8
    assert abs(st["iters"] - st_ref["iters"]) <= 1, (st, st_ref)
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert err <= 1e-7, err
    bb = O.project_pressure(pb, b) if kind == 0 else b
    r = bb - O.apply(pb, x)
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(bb)


def test_solve_status_codes():
    import torch
    from paper_2009_02171_amd import csdyn
    b = inputs.rhs(8, 4, seed=1)
    x, st, rc = _gpu_solve(8, 4, 1, b, maxit=1)
    assert rc == csdyn.ENOTCONV and st["iters"] == 1
    bn = b.copy()
    bn[0, 0, 0, 0, 0] = np.nan
    with pytest.raises(csdyn.CsdynError) as e:
        _gpu_solve(8, 4, 1, bn)
    assert e.value.status == csdyn.EBREAKDOWN


@pytest.mark.parametrize("kind,levels", [(0, 1), (0, 2), (1, 2)])
def test_mixed_precision_solve(kind, levels):
    """FP32 preconditioner inside FP64 FGMRES(30): still reaches 1e-8; iterations
    within one of the oracle's mixed solve; solution within 1e-7 of the FP64 oracle."""
    n, nr, sub = 16, 16, (8, 8, 8)
    print(f"[mixed solve] kind={kind} levels={levels}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    b = inputs.rhs(n, nr, seed=0)
    x64, _, _ = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=sub, levels=levels), flexible=True)
    xm, stm, _ = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=sub, levels=levels, precision=1), flexible=True)
    x, st, rc = _gpu_solve(n, nr, kind, b, sub=sub, levels=levels, flexible=True, precision=1)
    assert rc == 0 and st["relres_true"] <= 1.0001e-8
    assert abs(st["iters"] - stm["iters"]) <= 1, (st, stm)
    err = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    print(f"  iterations {st['iters']} (oracle mixed {stm['iters']}), error vs FP64 oracle {err:.2e}")
    assert err <= 1e-7


@pytest.mark.parametrize("kind", [0, 1])
def test_residual_norm_of_a_guess(kind):
    """||P b - A x|| of a candidate guess (P: the solve's VP pressure
    projection) on a grid whose reduction uses fewer than the maximum blocks."""
    import torch
    from paper_2009_02171_amd import csdyn
    n, nr = 16, 16
    pb = O.Problem(n, nr, kind=kind)
    b = inputs.rhs(n, nr, seed=51)
    x = inputs.random_field(pb.shape(), seed=52)
    bb = O.project_pressure(pb, b) if kind == 0 else b
    ref = np.linalg.norm(bb - O.apply(pb, x))
    op = csdyn.Operator(n, nr, kind=kind)
    got = csdyn.Residual(op)(torch.from_numpy(b).cuda(), torch.from_numpy(x).cuda())
    assert abs(got - ref) <= 1e-12 * ref


def test_two_systems_on_two_streams_match_sequential():
    """The two systems of a step solved at the same time from two host threads
    on two streams (as bench.py's *_two_streams forms do) give bit-identical
    solutions and iteration counts to the same solves one after the other."""
    import threading

    import torch
    from paper_2009_02171_amd import csdyn
    n, nr, sub = 16, 16, (8, 8, 8)
    print(f"[two streams] n={n} sub={sub} two-level, FP64 and FP32 preconditioners", flush=True)
    for prec in (0, 1):
        sys_ = {}
        for kind, seed in ((csdyn.VP, 1), (csdyn.BP, 2)):
            op = csdyn.Operator(n, nr, kind=kind)
            pc = csdyn.RAS(op, sub=sub, levels=2, precision=prec)
            sol = csdyn.Solver(op, pc, restart=30, maxit=2000, flexible=True, rtol=1e-8)
            b = torch.from_numpy(inputs.rhs(n, nr, seed)).cuda()
            sys_[kind] = (op, pc, sol, b, torch.cuda.Stream())
        seq = {}
        for kind, (_, _, sol, b, _) in sys_.items():
            x, st, rc = sol.solve(b, torch.zeros_like(b))
            torch.cuda.synchronize()
            assert rc == 0
            seq[kind] = (x.clone(), st["iters"], st["inner_iters"])
        par, errors = {}, []

        def run(kind):
            try:
                _, _, sol, b, s = sys_[kind]
                with torch.cuda.stream(s):
                    x = torch.zeros_like(b)
                    x, st, rc = sol.solve(b, x, stream=s)
                s.synchronize()
                par[kind] = (x, st["iters"], st["inner_iters"], rc)
            except Exception as e:  # reported below
                errors.append(e)

        threads = [threading.Thread(target=run, args=(k,)) for k in sys_]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        assert not errors, errors
        for kind in sys_:
            x, it, inner, rc = par[kind]
            assert rc == 0
            assert (it, inner) == seq[kind][1:], (kind, prec, it, inner, seq[kind][1:])
            assert torch.equal(x, seq[kind][0]), (kind, prec)


@pytest.mark.parametrize("precision", [0, 1])
def test_phase_times(precision):
    """opts.timing: the phase times cover the solve's span, the span is the solve's
    wall time within 5%, the coarse solve (PC-C) is the largest phase of the
    two-level preconditioner, and timing changes nothing in the result."""
    import time

    import torch
    from paper_2009_02171_amd import csdyn
    n, sub = 32, (8, 8, 8)
    op = csdyn.Operator(n, n, kind=0)
    pc = csdyn.RAS(op, sub=sub, levels=2, precision=precision)
    b = torch.from_numpy(inputs.rhs(n, n, seed=1)).cuda()
    plain = csdyn.Solver(op, pc, flexible=True)
    timed = csdyn.Solver(op, pc, flexible=True, timing=True)
    x0, st0, _ = plain.solve(b)
    timed.solve(b)  # first timed solve on this thread creates the events
    torch.cuda.synchronize()
    t = time.perf_counter()
    x1, st1, rc = timed.solve(b)
    wall = (time.perf_counter() - t) * 1e3
    ph = st1["t_ms"]
    print(f"[phase times] precision={precision} wall {wall:.2f} ms span {st1['t_span_ms']:.2f} ms {ph}", flush=True)
    assert rc == 0 and st1["iters"] == st0["iters"] and torch.equal(x0, x1)
    assert all(v >= -1e-3 for v in ph.values())
    assert abs(sum(ph.values()) - st1["t_span_ms"]) <= 1e-6 * st1["t_span_ms"] + 1e-6
    assert abs(st1["t_span_ms"] - wall) <= 0.05 * wall
    assert ph["pc_coarse"] == max(ph.values())
    assert ph["pc_fine"] > 0 and ph["pc_interp"] > 0 and ph["op"] > 0 and ph["orth"] > 0
    assert "t_ms" not in st0


@pytest.mark.parametrize("kind", [0, 1])
def test_three_level_solve_matches_oracle(kind):
    """FGMRES with the three-level hybrid at N = Nr = 32 (coarse 16, coarsest 8):
    iterations within one of the oracle's, solution within 1e-7, and fewer coarse
    iterations than with two levels."""
    n, sub = 32, (8, 8, 8)
    print(f"[three-level solve] kind={kind}", flush=True)
    pb = O.Problem(n, n, kind=kind)
    b = inputs.rhs(n, n, seed=0)
    x_ref, st_ref, rc_ref = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=sub, levels=3), flexible=True)
    assert rc_ref == 0
    x, st, rc = _gpu_solve(n, n, kind, b, sub=sub, levels=3, flexible=True)
    _, st2, _ = _gpu_solve(n, n, kind, b, sub=sub, levels=2, flexible=True)
    print(f"[three-level solve] gpu {st} oracle {st_ref} two-level inner {st2['inner_iters']}", flush=True)
    assert rc == 0 and st["relres_true"] <= 1.0001e-8
    assert abs(st["iters"] - st_ref["iters"]) <= 1, (st, st_ref)
    assert np.linalg.norm(x - x_ref) <= 1e-7 * np.linalg.norm(x_ref)
    assert 0 < st["inner_iters"] < st2["inner_iters"] and st["inner2_iters"] > 0


@pytest.mark.parametrize("n,nr,kind,sub,levels,flexible,orth,steps", [
    (16, 16, 0, (16, 16, 16), 1, False, 0, 4),   # the small configuration
    (16, 16, 1, (16, 16, 16), 1, False, 1, 7),
    (16, 16, 0, (8, 8, 8), 2, True, 0, 1),
    (8, 8, 1, None, 1, False, 0, 32),
])
def test_device_steps_match_oracle_and_host_path(n, nr, kind, sub, levels, flexible, orth, steps):
    """Device-resident Arnoldi steps (Hessenberg column and Givens rotation on
    the device, the convergence state read once per group of steps): the stop
    point is the oracle's within one step and the host path's exactly, and the
    solution matches both."""
    import torch
    from paper_2009_02171_amd import csdyn
    print(f"[device steps] n={n} kind={kind} sub={sub} levels={levels} steps={steps}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    b = inputs.rhs(n, nr, seed=3)
    pc_ref = O.Preconditioner(pb, sub=sub, levels=levels) if sub else None
    x_ref, st_ref, rc_ref = O.gmres(pb, b, pc=pc_ref, flexible=flexible, maxit=2000)
    assert rc_ref == 0
    op = csdyn.Operator(n, nr, kind=kind)
    pc = csdyn.RAS(op, sub=sub, levels=levels) if sub else None
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    out = {}
    for ds in (0, steps):
        sol = csdyn.Solver(op, pc, restart=30, maxit=2000, flexible=flexible, rtol=1e-8, orth=orth, device_steps=ds)
        x, st, rc = sol.solve(bt)
        torch.cuda.synchronize()
        assert rc == 0, st
        out[ds] = (x.cpu().numpy(), st)
    (xh, sth), (xd, std) = out[0], out[steps]
    assert std["iters"] == sth["iters"] and std["restarts"] == sth["restarts"], (std, sth)
    assert abs(std["iters"] - st_ref["iters"]) <= 1, (std, st_ref)
    assert std["relres_true"] <= 1.0001e-8
    assert abs(std["relres_est"] - sth["relres_est"]) <= 1e-6 * sth["relres_est"]
    assert np.linalg.norm(xd - xh) <= 1e-12 * np.linalg.norm(xh)
    assert np.linalg.norm(xd - x_ref) <= 1e-7 * np.linalg.norm(x_ref)


def test_device_steps_limits():
    """maxit inside a group stops at maxit exactly; out-of-range values are rejected."""
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(8, 4, kind=1)
    bt = torch.from_numpy(inputs.rhs(8, 4, seed=1)).cuda()
    sol = csdyn.Solver(op, None, restart=30, maxit=5, rtol=1e-12, device_steps=4)
    _, st, rc = sol.solve(bt)
    assert rc == csdyn.ENOTCONV and st["iters"] == 5
    sol = csdyn.Solver(op, None, restart=3, maxit=7, rtol=1e-12, device_steps=2)
    _, st, rc = sol.solve(bt)
    assert rc == csdyn.ENOTCONV and st["iters"] == 7 and st["restarts"] == 3
    with pytest.raises(csdyn.CsdynError) as e:
        csdyn.Solver(op, None, device_steps=33).solve(bt)
    assert e.value.status == csdyn.EINVAL
