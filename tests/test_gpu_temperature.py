"""GPU parity of the velocity-temperature system (the VTBE's u and Theta block,
Sec. 3.1 eq. tsvelocity, tstemperature) against the oracle: the operator, the
one- and two-level RAS, the solve, the temperature's nonlinear term, the
Crank-Nicolson right-hand side, Step 2's right-hand side, and three whole
steps with the temperature from the benchmark's initial state (Sec. 4.2)."""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs

pytestmark = pytest.mark.gpu

KW = dict(dt=2e-3, ekman=1e-3, ra=100.0, pr=0.8)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ops(n, nr):
    from paper_2009_02171_amd import csdyn
    return O.Problem(n, nr, kind=2, **KW), csdyn.Operator(n, nr, kind=csdyn.VT, **KW)


@pytest.mark.parametrize("n,nr", [(4, 4), (12, 5), (16, 16), (24, 7)])
def test_vt_operator_matches_oracle(n, nr):
    print(f"[vt operator] n={n} nr={nr}", flush=True)
    pb, op = _ops(n, nr)
    x = inputs.random_field(pb.shape(), 81)
    want = O.apply(pb, x)
    got = op.apply(_t(x)).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_vt_operator_large_shell_uses_the_register_kernel():
    """At N = Nr = 96 the FP64 default is the LDS-request kernel for VP / BP;
    VT goes to the register kernel: sampled rows against the oracle."""
    n = 96
    pb, op = _ops(n, n)
    x = inputs.random_field(pb.shape(), 82)
    got = op.apply(_t(x)).cpu().numpy().reshape(-1)
    rows = np.random.default_rng(83).integers(0, got.size, 4000)
    want = O.apply_rows(pb, x, rows)
    assert np.abs(got[rows] - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("levels,precision,tol", [(1, 0, 1e-12), (2, 0, 1e-9), (1, 1, 1e-5)])
def test_vt_ras_matches_oracle(levels, precision, tol):
    from paper_2009_02171_amd import csdyn
    n, nr, sub = 16, 8, (8, 8, 4)
    print(f"[vt ras] levels={levels} precision={precision}", flush=True)
    pb, op = _ops(n, nr)
    x = inputs.random_field(pb.shape(), 84)
    want = O.Preconditioner(pb, sub=sub, levels=levels, precision=precision).apply(x)
    got = csdyn.RAS(op, sub=sub, levels=levels, precision=precision).apply(_t(x)).cpu().numpy()
    assert np.abs(got - want).max() <= tol * np.abs(want).max()


def test_vt_solve_matches_oracle():
    from paper_2009_02171_amd import csdyn
    n, nr, sub = 16, 16, (8, 8, 8)
    pb, op = _ops(n, nr)
    b = inputs.rhs(n, nr, seed=85)
    x_ref, st_ref, rc_ref = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=sub, levels=1))
    assert rc_ref == 0
    x, st, rc = csdyn.Solver(op, csdyn.RAS(op, sub=sub, levels=1), rtol=1e-8).solve(_t(b))
    x = x.cpu().numpy()
    assert rc == 0 and st["relres_true"] <= 1.0001e-8
    assert abs(st["iters"] - st_ref["iters"]) <= 1, (st, st_ref)
    assert np.linalg.norm(x - x_ref) <= 1e-7 * np.linalg.norm(x_ref)


def test_temperature_nonlinear_cn_rhs_and_vector_rows():
    import torch
    from paper_2009_02171_amd import csdyn
    n, nr = 12, 6
    pb, op = _ops(n, nr)
    u = inputs.random_field(pb.shape(), 86)
    B = inputs.random_field(pb.shape(), 87)
    T = inputs.random_field(pb.shape(), 88)
    f1r, f3r = O.nonlinear(n, nr, u, B, 20.0, T=T)
    vp = csdyn.Operator(n, nr, kind=csdyn.VP, **KW)
    bp = csdyn.Operator(n, nr, kind=csdyn.BP, **KW)
    f1, f3 = csdyn.Nonlinear(vp, bp)(_t(u), _t(B), 20.0, T=_t(T))
    torch.cuda.synchronize()
    for got, want in ((f1, f1r), (f3, f3r)):
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()
    fm = inputs.random_field(pb.shape(), 89)
    want = O.cn_rhs(pb, T, f1r, 0.3, fm=fm, c2=-0.1)
    got = csdyn.cn_rhs(op, _t(T), _t(f1r), 0.3, fm=_t(fm), c2=-0.1).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(got[..., 3]).max() > 0                       # the Theta row is kept
    pv = O.Problem(n, nr, kind=0, **KW)
    want = O.vector_rows(pv, T)
    got = csdyn.vector_rows(vp, _t(T)).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    with pytest.raises(csdyn.CsdynError):
        csdyn.vector_rows(op, _t(T))
    with pytest.raises(csdyn.CsdynError):
        op.project(_t(T))


def _oracle_steps_with_temperature(n, nr, nsteps, dt, ekman, pm, ra, pr, sub, rtol):
    kw = dict(dt=dt, ekman=ekman, pm=pm, ra=ra, pr=pr)
    pv, pbm, pt = (O.Problem(n, nr, kind=k, **kw) for k in (0, 1, 2))
    pcs = {k: O.Preconditioner(p, sub=sub, levels=1) for k, p in ((0, pv), (1, pbm), (2, pt))}
    Dt, cB = 2 * ekman * dt, 1.0 / (ekman * pm)
    z = np.zeros((6, nr, n, n, 4))
    state = {0: z.copy(), 1: inputs.benchmark_b0(n, nr), 2: inputs.benchmark_theta0(n, nr)}
    xs = {0: z.copy(), 1: z.copy(), 2: z.copy()}
    fprev, iters = None, []
    for _ in range(nsteps):
        f1, f3 = O.nonlinear(n, nr, state[0], state[1], cB, T=state[2])
        first = fprev is None
        c1, c2 = (Dt, 0.0) if first else (1.5 * Dt, -0.5 * Dt)
        uhat = state[0] if first else O.project(pv, state[0])
        xhat = uhat.copy()
        xhat[..., 3] = state[2][..., 3]
        it = {}
        b = O.cn_rhs(pt, xhat, f1, c1, fm=None if first else fprev[2], c2=c2)
        xs[2], st, rc = O.gmres(pt, b, x0=xs[2], pc=pcs[2], rtol=rtol, maxit=2000)
        assert rc == 0
        it[2] = st["iters"]
        x0 = xs[0].copy()
        x0[..., :3] = xs[2][..., :3]
        xs[0], st, rc = O.gmres(pv, O.vector_rows(pv, xs[2]), x0=x0, pc=pcs[0], rtol=rtol, maxit=2000)
        assert rc == 0
        it[0] = st["iters"]
        bhat = state[1] if first else O.project(pbm, state[1])
        b = O.cn_rhs(pbm, bhat, f3, c1, fm=None if first else fprev[1], c2=c2)
        xs[1], st, rc = O.gmres(pbm, b, x0=xs[1], pc=pcs[1], rtol=rtol, maxit=2000)
        assert rc == 0
        it[1] = st["iters"]
        state = {0: O.step3_state(pv, xs[0]), 1: O.step3_state(pbm, xs[1]), 2: xs[2]}
        fprev = {2: f1, 1: f3}
        iters.append(it)
    return state, iters


def test_three_steps_with_temperature_match_oracle():
    import torch
    from paper_2009_02171_amd import step
    n, nr, sub = 8, 8, (8, 8, 8)
    dt, ekman, pm, ra, pr, rtol = 2e-2, 1e-2, 5.0, 100.0, 1.0, 1e-10
    print("[full steps with temperature]", flush=True)
    want, want_it = _oracle_steps_with_temperature(n, nr, 3, dt, ekman, pm, ra, pr, sub, rtol)
    s = step.SemiImplicit(n, nr, dt=dt, ekman=ekman, pm=pm, sub=sub, levels=1, rtol=rtol, temperature=True, ra=ra,
                          pr=pr, b0=_t(inputs.benchmark_b0(n, nr)), theta0=_t(inputs.benchmark_theta0(n, nr)))
    for k in range(3):
        st = s.step()
        for kind, name in ((2, "VT"), (0, "VP"), (1, "BP")):
            assert abs(st[name]["iters"] - want_it[k][kind]) <= 1, (k, name, st[name], want_it[k])
    torch.cuda.synchronize()
    for kind, name, sl in ((0, "VP", slice(0, 3)), (1, "BP", slice(0, 3)), (2, "VT", slice(3, 4))):
        got = s.state[name].cpu().numpy()[..., sl]
        ref = want[kind][..., sl]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"[full steps with temperature] {name} rel err {err:.2e}", flush=True)
        assert err <= 1e-7
