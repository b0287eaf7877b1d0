"""Oracle operator pins (finite-volume operators of Sec. 3.2 and the two
systems of Sec. 3.1).

* constants: the Neumann Laplacian annihilates 1 exactly;
* conservation (Gauss' theorem, eq. divdiscretization): the volume-weighted
  sum of the Neumann Laplacian and of D(u) for a no-slip field vanishes;
* the cube's rotation group maps the grid to itself, so the discrete
  operators commute with it (all 24 rotations for the Laplacian and the
  magnetic system, the 4 about z for the Coriolis system) -- this exercises
  every panel edge and cube corner;
* manufactured solutions converge at second order (Sec. 4.1 reports second
  order in space), L2 norm of the paper's error definition;
* the assembled matrix equals the row-by-row operator.
"""
import itertools

import numpy as np
import pytest

import oracle as O
import mms


def rotations():
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3))
            for a in range(3):
                m[a, perm[a]] = signs[a]
            if np.linalg.det(m) > 0:
                out.append(m)
    assert len(out) == 24
    return out


def cell_perm(xyz, R):
    """perm[a] = b such that centre_b = R centre_a."""
    flat = xyz.reshape(-1, 3)
    key = lambda v: tuple(np.round(v * 1e9).astype(np.int64))
    index = {key(v): b for b, v in enumerate(flat)}
    return np.array([index[key(R @ v)] for v in flat])


def rotate_field(x, perm, R, vector=True):
    flat = x.reshape(-1, 4)
    out = np.empty_like(flat)
    out[perm] = flat
    if vector:
        out[perm, :3] = flat[:, :3] @ R.T
    return out.reshape(x.shape)


def test_laplacian_of_constant_is_zero():
    pb = O.Problem(8, 6, kind=0)
    x = np.zeros(pb.shape())
    x[..., 3] = 1.7
    assert np.abs(O.apply(pb, x)).max() < 1e-13


@pytest.mark.parametrize("n,nr", [(4, 4), (8, 5)])
def test_conservation(n, nr):
    pb = O.Problem(n, nr, kind=0)
    _, vol = O.cell_geometry(pb)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(pb.shape())
    xp = x.copy(); xp[..., :3] = 0
    y = O.apply(pb, xp)[..., 3]
    assert abs((vol * y).sum()) <= 1e-13 * (vol * np.abs(y)).sum()
    xu = x.copy(); xu[..., 3] = 0
    y = O.apply(pb, xu)[..., 3]
    assert abs((vol * y).sum()) <= 1e-13 * (vol * np.abs(y)).sum()


@pytest.mark.parametrize("kind", [0, 1])
def test_assembled_equals_rowwise(kind):
    pb = O.Problem(8, 4, kind=kind)
    A = O.assemble(pb)
    x = np.random.default_rng(5).standard_normal(pb.nunk)
    y = O.apply(pb, x).ravel()
    assert np.abs(A @ x - y).max() <= 1e-13 * np.abs(y).max()
    rows = np.array([0, 7, 1234, pb.nunk - 1])
    np.testing.assert_allclose(O.apply_rows(pb, x, rows), y[rows], rtol=0, atol=1e-13 * np.abs(y).max())


def test_rotation_invariance_all_24():
    pb = O.Problem(6, 3, kind=1, dt=0.01, ekman=1.0, pm=1.0)
    xyz, _ = O.cell_geometry(pb)
    x = np.random.default_rng(7).standard_normal(pb.shape())
    y = O.apply(pb, x)
    scale = np.abs(y).max()
    for R in rotations():
        perm = cell_perm(xyz, R)
        xr = rotate_field(x, perm, R)
        np.testing.assert_allclose(O.apply(pb, xr), rotate_field(y, perm, R), rtol=0, atol=1e-12 * scale)
    # Neumann scalar Laplacian (VP pressure rows with u = 0)
    pv = O.Problem(6, 3, kind=0, dt=0.01, ekman=1.0)
    xs = x.copy(); xs[..., :3] = 0
    ys = O.apply(pv, xs)
    for R in rotations():
        perm = cell_perm(xyz, R)
        np.testing.assert_allclose(O.apply(pv, rotate_field(xs, perm, R)), rotate_field(ys, perm, R), rtol=0,
                                   atol=1e-12 * np.abs(ys).max())


def test_rotation_invariance_about_z_with_coriolis():
    pb = O.Problem(6, 3, kind=0, dt=0.05, ekman=0.5)
    xyz, _ = O.cell_geometry(pb)
    x = np.random.default_rng(8).standard_normal(pb.shape())
    y = O.apply(pb, x)
    for q in range(4):
        c, s = np.round(np.cos(q * np.pi / 2)), np.round(np.sin(q * np.pi / 2))
        R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
        perm = cell_perm(xyz, R)
        np.testing.assert_allclose(O.apply(pb, rotate_field(x, perm, R)), rotate_field(y, perm, R), rtol=0,
                                   atol=1e-12 * np.abs(y).max())
    # a rotation about x does not commute with the Coriolis term
    R = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], float)
    perm = cell_perm(xyz, R)
    assert np.abs(O.apply(pb, rotate_field(x, perm, R)) - rotate_field(y, perm, R)).max() > 1e-3


def _mms_error(kind, n):
    pb = O.Problem(n, n, kind=kind, dt=1.0, ekman=1.0, pm=1.0)
    ex, bx = mms.rhs_exprs(kind, O.RI, O.RO, 1.0, 1.0, 1.0)
    xyz, vol = O.cell_geometry(pb)
    xs = mms.evaluate(ex, xyz)
    b = mms.evaluate(bx, xyz)
    pc = O.Preconditioner(pb, sub=(n // 2, n // 2, n // 2), levels=1)
    x, st, rc = O.gmres(pb, b, pc=pc, restart=60, maxit=3000, rtol=1e-12)
    assert rc == 0, st
    if kind == 0:
        xs[..., 3] -= (vol * xs[..., 3]).sum() / vol.sum()
    # L2 error of Sec. 4.1: sqrt(sum (v - v_ref)^2 V)
    return np.sqrt(((x - xs) ** 2 * vol[..., None]).sum(axis=(0, 1, 2, 3)))


@pytest.mark.parametrize("kind", [0, 1])
def test_mms_second_order(kind):
    ns = (8, 12, 16)
    errs = np.array([_mms_error(kind, n) for n in ns])
    rates = np.log(errs[:-1] / errs[1:]) / np.log(np.array(ns[1:]) / np.array(ns[:-1]))[:, None]
    assert (rates > 1.85).all(), (errs, rates)
    assert (rates[-1] > 1.9).all(), (errs, rates)


@pytest.mark.parametrize("kind", [0, 1])
def test_dense_lu_tiny_grid(kind):
    """GMRES on N=4, Nr=4 (1,536 unknowns) reaches the LAPACK solution."""
    from paper_2009_02171_amd import inputs
    pb = O.Problem(4, 4, kind=kind)
    b = inputs.rhs(4, 4, seed=0)
    A = O.assemble(pb).toarray()
    _, vol = O.cell_geometry(pb)
    if kind == 0:
        # bordered system [[A, n], [w^T, 0]] with n = (0, 1_P), w = (0, V)
        nvec = np.zeros(pb.shape()); nvec[..., 3] = 1
        wvec = np.zeros(pb.shape()); wvec[..., 3] = vol
        bb = O.project_pressure(pb, b).ravel()
        M = np.block([[A, nvec.reshape(-1, 1)], [wvec.reshape(1, -1), np.zeros((1, 1))]])
        xd = np.linalg.solve(M, np.concatenate([bb, [0.0]]))
        assert abs(xd[-1]) < 1e-10
        xd = xd[:-1]
    else:
        bb = b.ravel()
        xd = np.linalg.solve(A, bb)
    for pc in (None, O.Preconditioner(pb, sub=(2, 2, 2), levels=1)):
        x, st, rc = O.gmres(pb, b, pc=pc, restart=40, maxit=2000, rtol=1e-13)
        assert rc == 0
        assert np.linalg.norm(x.ravel() - xd) <= 1e-9 * np.linalg.norm(xd)


def test_step3_gradient_second_order_and_divergence_identity():
    """Step 3 (Sec. 3.1): the cell-centred gradient converges at second order
    away from the walls; the divergence of the corrected face fluxes is the
    pressure row of A x; the projection reduces the cell divergence of a
    solved velocity and that divergence decreases under refinement."""
    import sympy as sp
    from paper_2009_02171_amd import inputs
    Pexpr = sp.sin(mms.X) * mms.Y + mms.Z**2 * mms.X + sp.cos(mms.Y * mms.Z)
    grad = [sp.diff(Pexpr, v) for v in (mms.X, mms.Y, mms.Z)]
    errs = []
    for n in (8, 16, 32):
        pb = O.Problem(n, n, kind=0, dt=1.0)
        xyz, vol = O.cell_geometry(pb)
        x = np.zeros(pb.shape())
        x[..., 3] = mms.evaluate([Pexpr], xyz)[..., 0]
        out = O.project(pb, x)
        k = slice(1, n - 1)
        e = -out[:, k, ..., :3] - mms.evaluate(grad, xyz)[:, k]
        errs.append(np.sqrt((e**2 * vol[:, k, ..., None]).sum()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 1.8, (errs, rates)
    divs = []
    for n in (8, 16):
        pb = O.Problem(n, n, kind=0, dt=1e-2, ekman=1.0)
        b = inputs.rhs(n, n, seed=3, noise=0.0)
        b[..., 3] = 0
        xs, st, rc = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=(n // 2,) * 3, levels=1), rtol=1e-12, maxit=3000)
        assert rc == 0
        out = O.project(pb, xs)
        np.testing.assert_array_equal(out[..., 3], O.apply(pb, xs)[..., 3])
        _, vol = O.cell_geometry(pb)
        D = lambda v: O.apply(O.Problem(n, n, kind=0, dt=0.0), v)[..., 3]
        un, ut = out.copy(), xs.copy()
        un[..., 3] = 0
        ut[..., 3] = 0
        dn, dt_ = np.sqrt((D(un) ** 2 * vol).sum()), np.sqrt((D(ut) ** 2 * vol).sum())
        assert dn < 0.5 * dt_
        divs.append(dn)
    assert divs[1] < 0.6 * divs[0]
