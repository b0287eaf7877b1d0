"""GPU operator parity: csdyn_operator_apply against the oracle's row-by-row
operator (Sec. 3.2), element by element, relative max-norm error <= 1e-12."""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _gpu_apply(n, nr, kind, x, tile=0, **kw):
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(n, nr, kind=kind, **kw)
    op.set_tile(tile)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = op.apply(xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("n,nr", [(4, 4), (5, 3), (16, 16), (24, 7), (40, 6), (33, 4)])
@pytest.mark.parametrize("kind", [0, 1])
def test_operator_matches_oracle(n, nr, kind):
    print(f"[operator parity] n={n} nr={nr} kind={kind}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=100 + n + kind)
    y_ref = O.apply(pb, x)
    y = _gpu_apply(n, nr, kind, x)
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    assert err <= TOL, err


@pytest.mark.parametrize("n,nr", [(17, 9), (40, 13), (33, 4), (64, 96)])
@pytest.mark.parametrize("kind", [0, 1])
def test_operator_lds_request_kernel_matches_oracle(n, nr, kind):
    """The FP64 kernel that requests its layers straight into LDS (tile 6):
    tiles on one and on two panel edges, layer chunks that end inside the
    six-step loop (9 = 6 + 3 and 13 = 6 + 6 + 1 layers) and chunks of two
    whole trips (N = 64, Nr = 96: 12 layers)."""
    print(f"[operator parity, tile 6] n={n} nr={nr} kind={kind}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=200 + n + kind)
    y_ref = O.apply(pb, x)
    y = _gpu_apply(n, nr, kind, x, tile=6)
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    assert err <= TOL, err


def test_operator_lds_request_kernel_graph_replays():
    """The FP64 layers-into-LDS stencil (tile 6) captured in a HIP graph: every
    replay, with eager work and synchronisations between the replays, equals
    the eager apply bit for bit."""
    import torch
    from paper_2009_02171_amd import csdyn
    n = nr = 48
    print(f"[operator graph replays] n={n}", flush=True)
    op = csdyn.Operator(n, nr, kind=0)
    op.set_tile(6)
    x = torch.from_numpy(inputs.random_field(op.shape, seed=5)).cuda()
    y_eager = op.apply(x).clone()
    y = op.empty()
    side = torch.cuda.Stream()  # default priority
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        op.apply(x, y)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        op.apply(x, y)
    for r in range(3):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), r
        assert float((x * 2).abs().sum()) > 0  # eager work between the replays


@pytest.mark.parametrize("kind", [0, 1])
def test_operator_stiff_parameters(kind):
    """dt*E = 1: the Laplacian dominates every row."""
    n, nr = 12, 8
    pb = O.Problem(n, nr, kind=kind, dt=1.0, ekman=1.0, pm=1.0)
    x = inputs.rhs(n, nr, seed=3)
    y_ref = O.apply(pb, x)
    y = _gpu_apply(n, nr, kind, x, dt=1.0, ekman=1.0, pm=1.0)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= TOL


@pytest.mark.parametrize("kind", [0, 1])
def test_operator_full_size_sampled(kind):
    """N = Nr = 96 (the large configuration): all rows next to the panel edges
    and walls of one k-plane pair, plus random rows, computed one by one."""
    n = nr = 96
    print(f"[operator parity, sampled] n={n} kind={kind}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=7 + kind)
    y = _gpu_apply(n, nr, kind, x)
    rng = np.random.default_rng(11)
    rows = set(rng.integers(0, pb.nunk, 20000).tolist())
    for p in range(6):
        for k in (0, 1, nr // 2, nr - 1):
            for t in range(n):
                for (i, j) in ((0, t), (n - 1, t), (t, 0), (t, n - 1)):
                    cell = ((p * nr + k) * n + j) * n + i
                    rows.update(4 * cell + c for c in range(4))
    rows = np.array(sorted(rows), dtype=np.int64)
    y_ref = O.apply_rows(pb, x, rows)
    yf = y.reshape(-1)[rows]
    assert np.abs(yf - y_ref).max() / np.abs(y_ref).max() <= TOL


def test_operator_rejects_aliasing():
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(8, 4)
    x = torch.zeros(op.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(csdyn.CsdynError):
        op.apply(x, x)


@pytest.mark.parametrize("kind", [0, 1])
def test_project_matches_oracle(kind):
    """Step 3 (Sec. 3.1): u~ - dt grad_h P and the corrected face divergence."""
    import torch
    from paper_2009_02171_amd import csdyn
    n, nr = 16, 8
    pb = O.Problem(n, nr, kind=kind, dt=1e-2)
    x = inputs.random_field(pb.shape(), seed=70 + kind)
    ref = O.project(pb, x)
    op = csdyn.Operator(n, nr, kind=kind, dt=1e-2)
    out = op.project(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.abs(out - ref).max() / np.abs(ref).max() <= 1e-12


def test_profile_select_times_only_the_named_kernels():
    """csdyn_profile_select: only the listed kernels are timed; the default times every launch."""
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(16, 8)
    x = torch.zeros(op.shape, dtype=torch.float64, device="cuda")
    with csdyn.Profile(select=["op_main"]) as p:
        op.apply(x)
        op.apply(x)
        torch.cuda.synchronize()
    assert {k[0] for k in p.result} == {"op_main"}
    assert sum(e["count"] for e in p.result.values()) == 2
    with csdyn.Profile() as q:
        op.apply(x)
        torch.cuda.synchronize()
    assert "op_main" in {k[0] for k in q.result} and len(q.result) >= 2
    with csdyn.Profile(select=["op_main"], every=3) as r:
        for _ in range(7):
            op.apply(x)
        torch.cuda.synchronize()
    assert sum(e["count"] for e in r.result.values()) == 3  # launches 0, 3 and 6
