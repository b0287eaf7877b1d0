"""Batched lock-step FGMRES over shells of different sizes, eager and
hipGraph-captured, against one solve per shell (itself pinned to the oracle),
and the operator's workgroup shapes against each other."""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs

pytestmark = pytest.mark.gpu

SHELLS = [(8, 0.0008), (16, 0.0003), (24, 0.0001), (16, 0.001)]  # (N = Nr, Ekman number)


def _setup(kind=0):
    import torch
    from paper_2009_02171_amd import csdyn
    ops, pcs, bs = [], [], []
    for s, (n, ek) in enumerate(SHELLS):
        op = csdyn.Operator(n, n, kind=kind, dt=1e-4, ekman=ek, pm=5.0)
        ops.append(op)
        pcs.append(csdyn.RAS(op, sub=(8, 8, 8), levels=1, precision=1))
        bs.append(torch.from_numpy(inputs.rhs(n, n, seed=100 + s)).cuda())
    return ops, pcs, bs


@pytest.mark.parametrize("kind", [0, 1])
def test_batched_matches_single_solves(kind):
    import torch
    from paper_2009_02171_amd import csdyn
    ops, pcs, bs = _setup(kind)
    ref = []
    for op, pc, b in zip(ops, pcs, bs):
        x, st, rc = csdyn.Solver(op, pc, restart=30, maxit=2000, flexible=True, rtol=1e-8).solve(b)
        assert rc == 0
        ref.append((x.clone(), st))
    batch = csdyn.Batch(ops, pcs, restart=30, maxit=2000, rtol=1e-8)
    results = {}
    for mode in ("eager", "graph", "graph_again"):
        xs = [torch.zeros_like(b) for b in bs]
        stats, rc = batch.solve(bs, xs, use_graph=mode != "eager")
        assert rc == 0
        results[mode] = xs
        for (xr, sr), x, st in zip(ref, xs, stats):
            assert abs(st["iters"] - sr["iters"]) <= 1, (mode, st, sr)
            assert st["res_true"] <= 1.0001e-8 * st["res0"]
            assert float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr)) <= 1e-9
        torch.cuda.synchronize()
    # a replay of the cached graphs reproduces the first graph solve exactly
    for a, b in zip(results["graph"], results["graph_again"]):
        assert torch.equal(a, b)


def test_batched_small_shell_matches_oracle():
    import torch
    from paper_2009_02171_amd import csdyn
    ops, pcs, bs = _setup(0)
    xs = [torch.zeros_like(b) for b in bs]
    stats, rc = csdyn.Batch(ops, pcs, restart=30, maxit=2000, rtol=1e-8).solve(bs, xs)
    n, ek = SHELLS[0]
    pb = O.Problem(n, n, kind=0, dt=1e-4, ekman=ek, pm=5.0)
    xo, so, rco = O.gmres(pb, bs[0].cpu().numpy(), pc=O.Preconditioner(pb, sub=(8, 8, 8), levels=1, precision=1),
                          flexible=True, rtol=1e-8)
    assert rco == 0 and abs(so["iters"] - stats[0]["iters"]) <= 1
    x = xs[0].cpu().numpy()
    assert np.linalg.norm(x - xo) <= 1e-7 * np.linalg.norm(xo)


def test_batched_rejects_two_level():
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(16, 16)
    pc = csdyn.RAS(op, sub=(8, 8, 8), levels=2)
    with pytest.raises(csdyn.CsdynError):
        csdyn.Batch([op], [pc])


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("kind", [0, 1])
def test_operator_tiles_agree(tile, kind):
    # tiles that hold one, two or four panel edges, odd layer counts; tile 6
    # (its own kernel) equal up to rounding
    import torch
    from paper_2009_02171_amd import csdyn
    for n, nr in ((40, 6), (24, 5), (17, 3), (5, 3), (8, 9)):
        op = csdyn.Operator(n, nr, kind=kind, dt=1e-2)
        x = torch.from_numpy(inputs.random_field((6, nr, n, n, 4), seed=n)).cuda()
        y0 = op.apply(x).clone()
        op.set_tile(tile)
        y = op.apply(x)
        if tile == 6:
            assert float((y - y0).abs().max()) <= 1e-13 * float(y0.abs().max())
        else:
            assert torch.equal(y, y0)


PSHELLS = [(16, 0.0003), (24, 0.0001), (32, 0.0005)]  # (N = Nr, Ekman number), all N >= 16


PERSISTENT_OFF = ("the persistent step is switched off: its first solve did not finish within 180 s on the GPU "
                  "(twice, the second time with relaxed polls); the cause is not shown")


@pytest.mark.parametrize("kind", [0, 1])
def test_phase_batched_step_matches_eager(kind):
    """One launch per phase for all shells (every shell's subdomain solves in one
    launch, then the edge fills, stencil tiles and Gram-Schmidt blocks) gives the
    eager batch's iterations and solutions bit for bit, on two solves in a row
    (the second replays the captured step graphs)."""
    import torch
    from paper_2009_02171_amd import csdyn
    ops, pcs, bs = [], [], []
    for s, (n, ek) in enumerate(PSHELLS):
        op = csdyn.Operator(n, n, kind=kind, dt=1e-4, ekman=ek, pm=5.0)
        ops.append(op)
        pcs.append(csdyn.RAS(op, sub=(8, 8, 8), levels=1, precision=1))
        bs.append(torch.from_numpy(inputs.rhs(n, n, seed=200 + s)).cuda())
    batch = csdyn.Batch(ops, pcs, restart=30, maxit=2000, rtol=1e-8)
    assert batch.available(csdyn.Batch.PHASES)
    xe = [torch.zeros_like(b) for b in bs]
    se, rc = batch.solve(bs, xe, use_graph=csdyn.Batch.EAGER)
    assert rc == 0
    for rep in range(2):
        print(f"[phase-batched] kind={kind} solve {rep}", flush=True)
        xp = [torch.zeros_like(b) for b in bs]
        sp, rc = batch.solve(bs, xp, use_graph=csdyn.Batch.PHASES)
        assert rc == 0
        for a, b, sa, sb in zip(xe, xp, se, sp):
            assert sa["iters"] == sb["iters"], (sa, sb)
            assert torch.equal(a, b), float((a - b).abs().max())


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("kind", [0, 1])
def test_persistent_step_matches_eager(kind):
    """One persistent launch per Arnoldi step (work-list of every shell's subdomain
    solves, edge fills, stencil tiles and Gram-Schmidt blocks) gives the eager
    batch's iterations and solutions bit for bit, on two solves in a row (the
    second reuses the captured step graphs)."""
    import torch
    from paper_2009_02171_amd import csdyn
    ops, pcs, bs = [], [], []
    for s, (n, ek) in enumerate(PSHELLS):
        op = csdyn.Operator(n, n, kind=kind, dt=1e-4, ekman=ek, pm=5.0)
        ops.append(op)
        pcs.append(csdyn.RAS(op, sub=(8, 8, 8), levels=1, precision=1))
        bs.append(torch.from_numpy(inputs.rhs(n, n, seed=200 + s)).cuda())
    batch = csdyn.Batch(ops, pcs, restart=30, maxit=2000, rtol=1e-8)
    assert batch.persistent_available
    xe = [torch.zeros_like(b) for b in bs]
    se, rc = batch.solve(bs, xe, use_graph=csdyn.Batch.EAGER)
    assert rc == 0
    for rep in range(2):
        print(f"[persistent] kind={kind} solve {rep}", flush=True)
        xp = [torch.zeros_like(b) for b in bs]
        sp, rc = batch.solve(bs, xp, use_graph=csdyn.Batch.PERSISTENT)
        assert rc == 0
        for a, b, sa, sb in zip(xe, xp, se, sp):
            assert sa["iters"] == sb["iters"], (sa, sb)
            assert torch.equal(a, b), float((a - b).abs().max())
            assert sb["res_true"] <= 1.0001e-8 * sb["res0"]


def test_persistent_step_is_switched_off():
    """While it is off, no handle offers the persistent step and asking for it is an error."""
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(16, 16)
    pc = csdyn.RAS(op, sub=(8, 8, 8), levels=1, precision=1)
    b = csdyn.Batch([op], [pc])
    assert not b.persistent_available and b.available(csdyn.Batch.PHASES)
    with pytest.raises(csdyn.CsdynError):
        b.solve([op.empty().zero_()], [op.empty().zero_()], use_graph=csdyn.Batch.PERSISTENT)
    op64 = csdyn.Operator(16, 16)
    b64 = csdyn.Batch([op64], [csdyn.RAS(op64, sub=(8, 8, 8), levels=1, precision=0)])
    assert not b64.available(csdyn.Batch.PHASES)   # FP64 preconditioner: modes 0 and 1 only
    with pytest.raises(csdyn.CsdynError):
        b64.solve([op64.empty().zero_()], [op64.empty().zero_()], use_graph=csdyn.Batch.PHASES)


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_step_needs_fp32_one_level():
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(16, 16)
    pc64 = csdyn.RAS(op, sub=(8, 8, 8), levels=1, precision=0)
    b = csdyn.Batch([op], [pc64])
    assert not b.persistent_available
    import torch
    x = [op.empty().zero_()]
    with pytest.raises(csdyn.CsdynError):
        b.solve([op.empty().zero_()], x, use_graph=csdyn.Batch.PERSISTENT)


def test_batched_uneven_shells_match_oracle():
    """The two smallest shells of the eight-shell batch (N = Nr = 24 and 32, their
    own Ekman numbers and right-hand sides), solved as one batch with the FP32
    one-level preconditioner on 8^3 boxes (graph of per-shell branches, and one
    launch per phase for both shells, which must agree bit for bit), against the
    oracle's FGMRES with its FP32 preconditioner emulation."""
    import torch
    from paper_2009_02171_amd import csdyn
    ops, pcs, bs, cases = [], [], [], []
    for s, n in enumerate((24, 32)):
        ek, b = inputs.shell_case(s, n, n)
        cases.append((n, ek, b))
        op = csdyn.Operator(n, n, kind=0, dt=1e-4, ekman=ek, pm=5.0)
        ops.append(op)
        pcs.append(csdyn.RAS(op, sub=(8, 8, 8), levels=1, precision=1))
        bs.append(torch.from_numpy(b).cuda())
    xs = [torch.zeros_like(b) for b in bs]
    batch = csdyn.Batch(ops, pcs, restart=30, maxit=3000, rtol=1e-8)
    stats, rc = batch.solve(bs, xs, use_graph=True)
    assert rc == 0
    xp = [torch.zeros_like(b) for b in bs]
    sp, rc = batch.solve(bs, xp, use_graph=csdyn.Batch.PHASES)
    assert rc == 0
    assert all(torch.equal(a, b) for a, b in zip(xs, xp)) and [s["iters"] for s in sp] == [s["iters"] for s in stats]
    for (n, ek, b), x, st in zip(cases, xs, stats):
        pb = O.Problem(n, n, kind=0, dt=1e-4, ekman=ek, pm=5.0)
        xo, so, rco = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=(8, 8, 8), levels=1, precision=1), flexible=True,
                              rtol=1e-8, maxit=3000)
        rel = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        print(f"[batched vs oracle] N={n} iters {st['iters']} / {so['iters']} rel {rel:.2e}", flush=True)
        assert rco == 0 and abs(so["iters"] - st["iters"]) <= 1
        assert rel <= 1e-7
