"""Oracle solver pins (Sec. 3.3).

* ILU(0): (LU)_ij = a_ij on the pattern; on a dense pattern it is Gaussian
  elimination without pivoting (checked against LAPACK's LU with identity
  permutation on a strictly diagonally dominant matrix).
* Subdomain matrices are R_i A R_i^T of the globally assembled matrix
  (eq. onelevel), re-extracted here independently.
* One-level RAS equals the sum of restricted triangular solves done with
  scipy's sparse triangular solver.
* The two-level hybrid equals w + M_one (x - A_f w), w = P A_c^{-1} R x
  (eq. coarsesolve, finesolve), with A_c^{-1} from LAPACK.
* Status codes of the solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle as O
from paper_2009_02171_amd import inputs


def test_ilu0_dense_pattern_is_lu_without_pivoting():
    rng = np.random.default_rng(0)
    n = 12
    a = rng.standard_normal((n, n))
    a += np.diag(np.abs(a).sum(1) + 1.0)
    rc, f = O.ilu0(sp.csr_matrix(a))
    assert rc == 0
    f = f.toarray()
    P, L, U = sla.lu(a)
    assert np.allclose(P, np.eye(n))
    np.testing.assert_allclose(np.tril(f, -1) + np.eye(n), L, atol=1e-13)
    np.testing.assert_allclose(np.triu(f), U, atol=1e-12)


def test_ilu0_zero_pivot_is_reported():
    a = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 1.0]]))
    rc, _ = O.ilu0(a)
    assert rc == O.EZEROPIVOT


def _split(f):
    L = sp.tril(f, -1).tocsr() + sp.identity(f.shape[0], format="csr")
    U = sp.triu(f).tocsr()
    return L, U


@pytest.mark.parametrize("kind", [0, 1])
def test_subdomain_matrix_and_ilu_property(kind):
    pb = O.Problem(8, 4, kind=kind)
    A = O.assemble(pb)
    pc = O.Preconditioner(pb, sub=(4, 4, 2), levels=1)
    assert pc.count() == 6 * 2 * 2 * 2
    for s in (0, 5, 17, 47):
        gcell, owned, f = pc.subdomain(s)
        idx = (4 * gcell[:, None] + np.arange(4)[None, :]).ravel()
        Ai = A[idx][:, idx].tocsr()
        Ai.sort_indices()
        # pattern = structural pattern of A restricted to the box
        assert (Ai.indptr == f.indptr).all() and (Ai.indices == f.indices).all()
        L, U = _split(f)
        LU = (L @ U).tocsr()
        # defining property of ILU(0): (LU)_ij = a_ij on the pattern
        rows = np.repeat(np.arange(Ai.shape[0]), np.diff(Ai.indptr))
        got = np.asarray(LU[rows, Ai.indices]).ravel()
        assert np.abs(got - Ai.data).max() <= 1e-12 * np.abs(Ai.data).max()
        assert owned.sum() == 4 * 4 * 2


def test_subdomain_boxes_cover_each_cell_once():
    pb = O.Problem(8, 4, kind=1)
    pc = O.Preconditioner(pb, sub=(4, 4, 4), levels=1)
    count = np.zeros(pb.ncell, int)
    for s in range(pc.count()):
        gcell, owned, _ = pc.subdomain(s)
        count[gcell[owned]] += 1
        # overlap 1: box = owned (4x4x4) + one layer on the 4 lateral sides;
        # walls clip it radially, and with 2x2 subdomains per panel every
        # box has exactly one cube-corner position, which does not exist
        assert len(gcell) == 4 * (6 * 6 - 1)
    assert (count == 1).all()


@pytest.mark.parametrize("kind", [0, 1])
def test_ras_apply_matches_triangular_solves(kind):
    pb = O.Problem(8, 4, kind=kind)
    pc = O.Preconditioner(pb, sub=(4, 8, 2), levels=1)
    x = np.random.default_rng(1).standard_normal(pb.nunk)
    y = np.zeros(pb.nunk)
    for s in range(pc.count()):
        gcell, owned, f = pc.subdomain(s)
        idx = (4 * gcell[:, None] + np.arange(4)[None, :]).ravel()
        L, U = _split(f)
        z = spl.spsolve_triangular(L, x[idx], lower=True)
        z = spl.spsolve_triangular(U, z, lower=False)
        own = np.repeat(owned, 4)
        y[idx[own]] = z[own]
    np.testing.assert_allclose(pc.apply(x).ravel(), y, rtol=0, atol=1e-12 * np.abs(y).max())


def test_two_level_matches_dense_composition():
    pb = O.Problem(8, 4, kind=1)
    pc2 = O.Preconditioner(pb, sub=(4, 4, 2), levels=2, coarse_rtol=1e-14, coarse_restart=200, coarse_maxit=2000)
    pc1 = O.Preconditioner(pb, sub=(4, 4, 2), levels=1)
    pcb = O.Problem(4, 2, kind=1)
    Ac = O.assemble(pcb).toarray()
    Af = O.assemble(pb)
    x = np.random.default_rng(2).standard_normal(pb.shape())
    # restriction: mean of the 8 children; prolongation: copy to children
    xc = x.reshape(6, 2, 2, 4, 2, 4, 2, 4).mean(axis=(2, 4, 6))
    ec = np.linalg.solve(Ac, xc.ravel()).reshape(xc.shape)
    w = np.repeat(np.repeat(np.repeat(ec, 2, axis=1), 2, axis=2), 2, axis=3)
    y = w + pc1.apply(x.ravel() - Af @ w.ravel())
    got = pc2.apply(x)
    assert np.abs(got - y).max() <= 1e-9 * np.abs(y).max()


def test_one_subdomain_exact_when_pattern_is_complete():
    """RAS with the whole grid as one subdomain and a complete factorization
    is A^{-1}; with ILU(0) it is not, but GMRES still reaches the LU solution."""
    pb = O.Problem(4, 2, kind=1)
    A = O.assemble(pb).toarray()
    b = inputs.rhs(4, 2, seed=3)
    pc = O.Preconditioner(pb, sub=(4, 4, 2), levels=1)
    x, st, rc = O.gmres(pb, b, pc=pc, restart=30, maxit=500, rtol=1e-13)
    xd = np.linalg.solve(A, b.ravel())
    assert rc == 0 and np.linalg.norm(x.ravel() - xd) <= 1e-10 * np.linalg.norm(xd)


def test_gmres_status_codes():
    pb = O.Problem(8, 4, kind=1)
    b = inputs.rhs(8, 4, seed=1)
    x, st, rc = O.gmres(pb, b, maxit=1)
    assert rc == O.ENOTCONV and st["iters"] == 1
    bn = b.copy(); bn[0, 0, 0, 0, 0] = np.nan
    _, _, rc = O.gmres(pb, bn)
    assert rc == O.EBREAKDOWN
    with pytest.raises(RuntimeError):
        O.Preconditioner(O.Problem(6, 4, kind=1), sub=(3, 3, 2), levels=2)
    # dt = 0: the VP pressure rows have no diagonal -> zero pivot
    with pytest.raises(RuntimeError):
        O.Preconditioner(O.Problem(8, 4, kind=0, dt=0.0), sub=(4, 4, 4), levels=1)


def test_fgmres_two_level_reaches_tolerance():
    pb = O.Problem(8, 8, kind=0)
    b = inputs.rhs(8, 8, seed=0)
    pc = O.Preconditioner(pb, sub=(4, 4, 4), levels=2)
    x, st, rc = O.gmres(pb, b, pc=pc, flexible=True, rtol=1e-8)
    assert rc == 0 and st["relres_true"] <= 1.01e-8 and st["inner_iters"] > 0
    bb = O.project_pressure(pb, b)
    r = bb - O.apply(pb, x)
    assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(bb)


def test_fp32_preconditioner_emulation():
    """FP32 inside M^{-1}: the one-level apply stays within FP32 rounding of the
    FP64 apply, and the flexible solve still reaches 1e-8 at the FP64 solution."""
    pb = O.Problem(8, 8, kind=0)
    x = inputs.random_field(pb.shape(), seed=4)
    y64 = O.Preconditioner(pb, sub=(4, 4, 4), levels=1).apply(x)
    y32 = O.Preconditioner(pb, sub=(4, 4, 4), levels=1, precision=1).apply(x)
    rel = np.abs(y32 - y64).max() / np.abs(y64).max()
    assert 1e-9 < rel < 1e-4
    b = inputs.rhs(8, 8, seed=0)
    x64, s64, _ = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=(4, 4, 4), levels=2), flexible=True)
    x32, s32, rc = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=(4, 4, 4), levels=2, precision=1), flexible=True)
    assert rc == 0 and s32["relres_true"] <= 1.0001e-8
    assert abs(s32["iters"] - s64["iters"]) <= 1
    assert np.linalg.norm(x32 - x64) <= 1e-7 * np.linalg.norm(x64)
