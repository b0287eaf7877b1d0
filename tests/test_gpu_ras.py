"""GPU preconditioner parity: csdyn_ras_apply against the oracle's RAS
(eq. onelevel) and two-level hybrid (eq. twolevel), element by element."""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs

pytestmark = pytest.mark.gpu


def _setup(n, nr, kind, sub, levels=1, **kw):
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(n, nr, kind=kind)
    pc = csdyn.RAS(op, sub=sub, levels=levels, **kw)
    return op, pc


def _apply(pc, x):
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = pc.apply(xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


# storage 1: ring of recent levels; 2: whole subdomain vector in LDS (too large
# for the 16^3 boxes in FP64)
ONE_LEVEL_CASES = [(8, 4, 0, (4, 4, 2), 1), (8, 4, 1, (4, 4, 2), 1), (16, 16, 0, (16, 16, 16), 1),
                   (16, 16, 1, (16, 16, 16), 1), (12, 6, 1, (6, 4, 3), 1), (24, 8, 0, (8, 8, 4), 1),
                   (8, 4, 0, (4, 4, 2), 2), (8, 4, 1, (4, 4, 2), 2), (12, 6, 1, (6, 4, 3), 2), (24, 8, 0, (8, 8, 4), 2)]


@pytest.mark.parametrize("n,nr,kind,sub,storage", ONE_LEVEL_CASES)
def test_one_level_matches_oracle(n, nr, kind, sub, storage):
    print(f"[ras parity] n={n} nr={nr} kind={kind} sub={sub} storage={storage}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=21 + n)
    y_ref = O.Preconditioner(pb, sub=sub, levels=1).apply(x)
    _, pc = _setup(n, nr, kind, sub, storage=storage)
    assert pc.info()["box_in_lds_fine"] == storage
    y = _apply(pc, x)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= 1e-12


@pytest.mark.parametrize("kind", [0, 1])
def test_one_level_full_size_sampled(kind):
    """N = Nr = 96 with 384 subdomains of 24^3: sampled subdomains (corner,
    edge, interior, both walls) checked one by one against the oracle."""
    n, nr, sub = 96, 96, (24, 24, 24)
    print(f"[ras parity, sampled] n={n} kind={kind}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=5 + kind)
    _, pc = _setup(n, nr, kind, sub)
    y = _apply(pc, x)
    for s in (0, 5, 21, 63, 64 + 42, 383):
        ys = O.subdomain_solve(pb, sub, s, x)
        m = ~np.isnan(ys)
        assert m.sum() == 4 * 24 ** 3
        assert np.abs(y[m] - ys[m]).max() / np.abs(ys[m]).max() <= 1e-12, s


@pytest.mark.parametrize("kind,storage", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_two_level_matches_oracle(kind, storage):
    """Hybrid two-level apply; the inner coarse GMRES runs to rtol 0.1 on both
    sides, so the Krylov paths agree to rounding."""
    n, nr, sub = 16, 8, (8, 8, 4)
    print(f"[two-level parity] kind={kind} storage={storage}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=31 + kind)
    y_ref = O.Preconditioner(pb, sub=sub, levels=2).apply(x)
    _, pc = _setup(n, nr, kind, sub, levels=2, storage=storage)
    y = _apply(pc, x)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= 1e-9


def test_two_level_near_exact_coarse():
    n, nr, sub = 8, 4, (4, 4, 2)
    pb = O.Problem(n, nr, kind=1)
    x = inputs.random_field(pb.shape(), seed=41)
    kw = dict(coarse_rtol=1e-12, coarse_restart=30, coarse_maxit=600)
    y_ref = O.Preconditioner(pb, sub=sub, levels=2, **kw).apply(x)
    _, pc = _setup(n, nr, 1, sub, levels=2, **kw)
    y = _apply(pc, x)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= 1e-9


def test_ras_rejects_bad_options():
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(12, 6)
    with pytest.raises(csdyn.CsdynError):
        csdyn.RAS(op, sub=(5, 4, 3))
    with pytest.raises(csdyn.CsdynError):
        csdyn.RAS(op, sub=(6, 6, 3), levels=2)   # odd subdomain size for two levels
    with pytest.raises(csdyn.CsdynError):
        csdyn.RAS(op, sub=(6, 6, 3), storage=4)
    big = csdyn.Operator(16, 20)
    with pytest.raises(csdyn.CsdynError):       # a 16^2 x 20 box's FP64 vector does not fit in LDS, even folded
        csdyn.RAS(big, sub=(16, 16, 20), storage=2)
    with pytest.raises(csdyn.CsdynError):       # no such value layout
        csdyn.RAS(op, sub=(6, 6, 3), values=3)
    with pytest.raises(csdyn.CsdynError):       # the packed value layout is for FP64 factors only
        csdyn.RAS(op, sub=(6, 6, 3), precision=1, values=1)


@pytest.mark.parametrize("n,nr,kind,sub,storage,levels", [
    (16, 16, 0, (8, 8, 8), 0, 1),      # box vector
    (16, 16, 1, (8, 8, 8), 1, 1),      # ring
    (24, 24, 0, (12, 12, 12), 0, 1),   # the coarse 12^3 shape: folded box vector
    (16, 16, 0, (16, 16, 16), 1, 1),   # one ring box per panel
    (32, 32, 1, (8, 8, 8), 0, 2)])     # two levels: both levels' sweeps
def test_packed_values_equal_padded(n, nr, kind, sub, storage, levels):
    """The packed value layout (odd widths' last entries unpadded) and padded pairs give the same bits."""
    print(f"[ras value layouts] n={n} nr={nr} kind={kind} sub={sub} storage={storage} levels={levels}", flush=True)
    x = inputs.random_field((6, nr, n, n, 4), seed=61 + n)
    ys = []
    for values in (1, 2):
        _, pc = _setup(n, nr, kind, sub, levels=levels, storage=storage, values=values)
        info = pc.info()
        assert info["packed_fine"] == (values == 1)
        if levels == 2:
            assert info["packed_coarse"] == (values == 1)
        ys.append(_apply(pc, x))
    assert np.array_equal(ys[0], ys[1])


@pytest.mark.parametrize("n,nr,kind,sub,storage", [(8, 4, 0, (4, 4, 2), 1), (16, 16, 1, (16, 16, 16), 1),
                                                   (24, 8, 0, (8, 8, 4), 1), (8, 4, 0, (4, 4, 2), 2),
                                                   (24, 8, 0, (8, 8, 4), 2)])
def test_one_level_fp32_matches_oracle_emulation(n, nr, kind, sub, storage):
    """FP32 factors and sweeps: GPU against the oracle's FP32 emulation."""
    print(f"[ras fp32 parity] n={n} nr={nr} kind={kind} storage={storage}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=51 + n)
    y_ref = O.Preconditioner(pb, sub=sub, levels=1, precision=1).apply(x)
    _, pc = _setup(n, nr, kind, sub, precision=1, storage=storage)
    y = _apply(pc, x)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= 1e-5


@pytest.mark.parametrize("kind", [0, 1])
def test_two_level_fp32_matches_oracle_emulation(kind):
    n, nr, sub = 16, 8, (8, 8, 4)
    print(f"[two-level fp32 parity] kind={kind}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=61 + kind)
    y_ref = O.Preconditioner(pb, sub=sub, levels=2, precision=1).apply(x)
    _, pc = _setup(n, nr, kind, sub, levels=2, precision=1)
    y = _apply(pc, x)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= 1e-4


def _sampled_parity(n, nr, kind, sub, precision, subdomains, tol, seed):
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=seed)
    _, pc = _setup(n, nr, kind, sub, precision=precision)
    info = pc.info()
    y = _apply(pc, x)
    worst = 0.0
    for s in subdomains:
        ys = O.subdomain_solve(pb, sub, s, x, precision=precision)
        m = ~np.isnan(ys)
        assert m.sum() == 4 * sub[0] * sub[1] * sub[2]
        worst = max(worst, np.abs(y[m] - ys[m]).max() / np.abs(ys[m]).max())
    print(f"[ras parity, sampled] n={n} sub={sub} precision={precision} info={info} worst {worst:.2e}", flush=True)
    assert worst <= tol
    return info


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_coarse_level_shape_sampled(precision, tol):
    """The coarse level of the N = Nr = 96 two-level preconditioner: N = Nr = 48
    with 384 boxes of 12^3 (sweep with the whole box vector in LDS), sampled
    subdomains (panel corners and edges, both walls, interior) against the
    oracle's single-subdomain solve in the same precision."""
    info = _sampled_parity(48, 48, 0, (12, 12, 12), precision, (0, 3, 17, 21, 42, 63, 64 + 21, 383), tol,
                           seed=81 + precision)
    # FP64: the vector folded so that two workgroups share a compute unit
    assert info["box_in_lds_fine"] == (3 if precision == 0 else 2) and info["threads_fine"] == 512
    assert info["blocks_per_cu_fine"] >= 2


@pytest.mark.parametrize("kind,precision,tol", [(0, 0, 1e-12), (1, 0, 1e-12), (0, 1, 1e-5), (1, 1, 1e-5)])
def test_coarse_box_shape_full(kind, precision, tol):
    """Every subdomain of N = Nr = 24 with 12^3 boxes (the coarse level's box
    shape and kernel instance) against the oracle's full one-level apply."""
    n, nr, sub = 24, 24, (12, 12, 12)
    print(f"[ras parity] n={n} sub={sub} kind={kind} precision={precision}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=91 + kind)
    y_ref = O.Preconditioner(pb, sub=sub, levels=1, precision=precision).apply(x)
    _, pc = _setup(n, nr, kind, sub, precision=precision)
    info = pc.info()
    assert info["box_in_lds_fine"] == (3 if precision == 0 else 2) and info["threads_fine"] == 512, info
    y = _apply(pc, x)
    assert np.abs(y - y_ref).max() / np.abs(y_ref).max() <= tol


@pytest.mark.parametrize("n,nr,sub,kind", [(24, 24, (12, 12, 12), 0), (24, 24, (12, 12, 12), 1),
                                            (24, 24, (12, 12, 12), 2), (48, 48, (12, 12, 12), 0),
                                            (48, 48, (12, 12, 12), 1), (24, 33, (12, 12, 11), 0),
                                            (24, 33, (12, 12, 11), 1)])
def test_folded_box_vector_equals_unfolded(n, nr, sub, kind):
    """The folded FP64 box vector (late rows in the slots of the early rows,
    the early rows' L results back from a per-subdomain buffer) gives the
    unfolded sweep's results bit for bit, on every subdomain of the 12^3-box
    shape, and on a grid where only the boxes away from the walls are folded
    (Nr = 33 with 12 x 12 x 11 boxes: the wall boxes fit unfolded); the folded
    sweep fits two workgroups per compute unit, the unfolded one."""
    print(f"[ras fold] n={n} nr={nr} sub={sub} kind={kind}", flush=True)
    x = inputs.random_field((6, nr, n, n, 4), seed=121 + n + kind)
    _, pf = _setup(n, nr, kind, sub, storage=2)
    _, pu = _setup(n, nr, kind, sub, storage=3)
    fi, ui = pf.info(), pu.info()
    assert fi["box_in_lds_fine"] == 3 and ui["box_in_lds_fine"] == 2, (fi, ui)
    assert fi["lds_fine"] <= 80 * 1024 - 512 < ui["lds_fine"]
    assert fi["blocks_per_cu_fine"] == 2 and ui["blocks_per_cu_fine"] == 1, (fi, ui)
    yf, yu = _apply(pf, x), _apply(pu, x)
    assert np.array_equal(yf, yu)
    if (n, nr, kind) in ((24, 24, 2), (24, 33, 0)):  # and the oracle: the temperature system, the mixed grid
        pb = O.Problem(n, nr, kind=kind)
        y_ref = O.Preconditioner(pb, sub=sub, levels=1).apply(x)
        assert np.abs(yf - y_ref).max() / np.abs(y_ref).max() <= 1e-12


@pytest.mark.parametrize("n,sub,kind", [(16, (16, 16, 16), 0), (16, (16, 16, 16), 1), (32, (16, 16, 16), 0)])
def test_large_box_vector_folded_into_one_workgroup(n, sub, kind):
    """A subdomain vector above the automatic bound (the small configuration's
    one box per panel, 20480 rows = 160 KiB in FP64) folded into one
    workgroup's LDS: the oracle's result to 1e-12, and the ring sweep's result
    bit for bit (the same slices in the same order, only the storage differs)."""
    print(f"[ras fold, one workgroup] n={n} sub={sub} kind={kind}", flush=True)
    x = inputs.random_field((6, n, n, n, 4), seed=131 + n + kind)
    _, pf = _setup(n, n, kind, sub)
    _, pr = _setup(n, n, kind, sub, storage=1)
    fi, ri = pf.info(), pr.info()
    assert fi["box_in_lds_fine"] == 3 and ri["box_in_lds_fine"] in (0, 1), (fi, ri)
    assert 80 * 1024 < fi["lds_fine"] <= 160 * 1024 - 512 and fi["blocks_per_cu_fine"] == 1, fi
    yf, yr = _apply(pf, x), _apply(pr, x)
    assert np.array_equal(yf, yr)
    if n == 16:
        pb = O.Problem(n, n, kind=kind)
        y_ref = O.Preconditioner(pb, sub=sub, levels=1).apply(x)
        assert np.abs(yf - y_ref).max() / np.abs(y_ref).max() <= 1e-12


@pytest.mark.parametrize("kind,precision,tol", [(0, 0, 1e-9), (1, 0, 1e-9), (0, 1, 1e-4)])
def test_two_level_n32_matches_oracle(kind, precision, tol):
    """Two-level apply at N = Nr = 32 with 8^3 fine boxes (coarse N = 16, 4^3 boxes)."""
    n, nr, sub = 32, 32, (8, 8, 8)
    print(f"[two-level parity] n={n} kind={kind} precision={precision}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=101 + kind)
    y_ref = O.Preconditioner(pb, sub=sub, levels=2, precision=precision).apply(x)
    _, pc = _setup(n, nr, kind, sub, levels=2, precision=precision)
    y = _apply(pc, x)
    rel = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    print(f"[two-level parity] rel {rel:.2e}", flush=True)
    assert rel <= tol


@pytest.mark.parametrize("n,nr,sub,kind,precision,tol", [(16, 8, (8, 8, 4), 0, 0, 1e-9), (16, 8, (8, 8, 4), 1, 0, 1e-9),
                                                         (32, 32, (8, 8, 8), 0, 0, 1e-9), (16, 8, (8, 8, 4), 0, 1, 1e-4),
                                                         (32, 32, (8, 8, 8), 1, 1, 1e-4)])
def test_three_level_matches_oracle(n, nr, sub, kind, precision, tol):
    """Three-level hybrid (the two-level construction repeated on the coarse grid:
    FGMRES coarse solve preconditioned by the coarse grid's own hybrid) against
    the oracle, FP64 and FP32 (the oracle's FP32 emulation of the same structure)."""
    print(f"[three-level parity] n={n} nr={nr} kind={kind} precision={precision}", flush=True)
    pb = O.Problem(n, nr, kind=kind)
    x = inputs.random_field(pb.shape(), seed=111 + n + kind)
    y_ref = O.Preconditioner(pb, sub=sub, levels=3, precision=precision).apply(x)
    _, pc = _setup(n, nr, kind, sub, levels=3, precision=precision)
    info = pc.info()
    assert info["nsd_coarse"] == info["nsd_fine"]
    y = _apply(pc, x)
    rel = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    print(f"[three-level parity] rel {rel:.2e}", flush=True)
    assert rel <= tol


def test_three_level_rejects_bad_sizes():
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(16, 8)
    with pytest.raises(csdyn.CsdynError):
        csdyn.RAS(op, sub=(8, 8, 2), levels=3)      # 2 is not divisible by 4
    with pytest.raises(csdyn.CsdynError):
        csdyn.RAS(csdyn.Operator(12, 12), sub=(4, 4, 4), levels=3)   # N/4 = 3 < 4
