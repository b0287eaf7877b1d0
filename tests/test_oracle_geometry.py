"""Oracle geometry pins (grid and metric of Sec. 3.2).

sqrt(g) is checked against the paper's printed closed form, the covariant
basis against finite differences of the embedding, the dual basis against
g^m . g_n = delta, the total volume against the exact shell volume, and the
panel-edge tables against the 3-D positions they claim to match.
"""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs

PANELS = inputs._PANELS


def embed(p, xi, eta, r):
    loc = np.array([1.0, np.tan(xi), np.tan(eta)])
    return r * PANELS[p] @ (loc / np.linalg.norm(loc))


@pytest.mark.parametrize("p", range(6))
def test_sqrtg_matches_paper_formula(p):
    rng = np.random.default_rng(p)
    for _ in range(20):
        xi, eta = rng.uniform(-np.pi / 4, np.pi / 4, 2)
        r = rng.uniform(O.RI, O.RO)
        sg, gcov, gcon = O.metric(p, xi, eta, r)
        # Sec. 3.2: sqrt(g) = r^2 sec^2(xi) sec^2(eta) / (1 + tan^2 xi + tan^2 eta)^(3/2)
        paper = r**2 / np.cos(xi) ** 2 / np.cos(eta) ** 2 / (1 + np.tan(xi) ** 2 + np.tan(eta) ** 2) ** 1.5
        assert sg == pytest.approx(paper, rel=1e-13)


@pytest.mark.parametrize("p", range(6))
def test_covariant_basis_is_embedding_derivative(p):
    rng = np.random.default_rng(10 + p)
    h = 1e-6
    for _ in range(10):
        xi, eta = rng.uniform(-np.pi / 4, np.pi / 4, 2)
        r = rng.uniform(O.RI, O.RO)
        _, gcov, gcon = O.metric(p, xi, eta, r)
        d1 = (embed(p, xi + h, eta, r) - embed(p, xi - h, eta, r)) / (2 * h)
        d2 = (embed(p, xi, eta + h, r) - embed(p, xi, eta - h, r)) / (2 * h)
        d3 = (embed(p, xi, eta, r + h) - embed(p, xi, eta, r - h)) / (2 * h)
        np.testing.assert_allclose(gcov[0], d1, atol=1e-8)
        np.testing.assert_allclose(gcov[1], d2, atol=1e-8)
        np.testing.assert_allclose(gcov[2], d3, atol=1e-8)
        np.testing.assert_allclose(gcon @ gcov.T, np.eye(3), atol=1e-13)
        # g_13 = g_23 = 0, g_33 = 1 (radial coordinate is orthogonal and unit)
        assert abs(gcov[0] @ gcov[2]) < 1e-13 and abs(gcov[1] @ gcov[2]) < 1e-13
        assert gcov[2] @ gcov[2] == pytest.approx(1.0, rel=1e-14)


def test_panels_tile_the_sphere_right_handed():
    for p in range(6):
        m = PANELS[p]
        assert np.linalg.det(m) == pytest.approx(1.0)
        # xi increases eastward for equatorial panels: d/dxi along +phi
    c = PANELS[:, :, 0]
    assert {tuple(v) for v in c} == {(1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)}


def test_total_volume_second_order():
    exact = 4 * np.pi / 3 * (O.RO**3 - O.RI**3)
    errs = []
    for n in (8, 16, 32):
        _, vol = O.cell_geometry(O.Problem(n, n))
        errs.append(abs(vol.sum() - exact) / exact)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > 1.9).all(), (errs, rates)


def test_cell_centres_match_shared_generator():
    pb = O.Problem(6, 3)
    xyz, _ = O.cell_geometry(pb)
    d = inputs.cell_directions(6)
    r = O.RI + (np.arange(3) + 0.5) * (O.RO - O.RI) / 3
    np.testing.assert_allclose(xyz, r[None, :, None, None, None] * d[:, None], atol=1e-14)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_seam_ghosts_lie_on_neighbour_first_layer(n):
    """A ghost at extended index -1 (or N) lies exactly on the neighbour's
    first-layer normal coordinate; cubic weights reproduce its tangential
    coordinate, and its 3-D position is the point on the neighbour's line."""
    pb = O.Problem(n, 2)
    st = O.seam_tables(pb)
    h = np.pi / (2 * n)
    a = lambda i: -np.pi / 4 + (i + 0.5) * h
    for p in range(6):
        for e in range(4):
            for t in range(n):
                if e == 0:
                    xi, eta = a(-1), a(t)
                elif e == 1:
                    xi, eta = a(n), a(t)
                elif e == 2:
                    xi, eta = a(t), a(-1)
                else:
                    xi, eta = a(t), a(n)
                target = embed(p, xi, eta, 1.0)
                q, fix, idx, m0, w = st["q"][p, e, t], st["fix_i"][p, e, t], st["idx"][p, e, t], st["m0"][p, e, t], \
                    st["w"][p, e, t]
                assert q != p and idx in (0, n - 1) and 0 <= m0 <= n - 4
                assert w.sum() == pytest.approx(1.0, abs=1e-14)
                # tangential angle reproduced exactly by the cubic weights
                ang = sum(w[m] * a(m0 + m) for m in range(4))
                if fix:
                    pt = embed(q, a(idx), ang, 1.0)
                else:
                    pt = embed(q, ang, a(idx), 1.0)
                np.testing.assert_allclose(pt, target, atol=1e-13)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_seam_faces_conform_and_pair_up(n):
    pb = O.Problem(n, 2)
    st = O.seam_tables(pb)
    h = np.pi / (2 * n)
    a = lambda i: -np.pi / 4 + (i + 0.5) * h
    fpt = {0: lambda t: (-np.pi / 4, a(t)), 1: lambda t: (np.pi / 4, a(t)),
           2: lambda t: (a(t), -np.pi / 4), 3: lambda t: (a(t), np.pi / 4)}
    pairs = set()
    for p in range(6):
        for e in range(4):
            for t in range(n):
                q, eq, tq = st["face_q"][p, e, t], st["face_e"][p, e, t], st["face_t"][p, e, t]
                np.testing.assert_allclose(embed(p, *fpt[e](t), 1.0), embed(q, *fpt[eq](tq), 1.0), atol=1e-13)
                # the neighbour maps back
                assert (st["face_q"][q, eq, tq], st["face_e"][q, eq, tq], st["face_t"][q, eq, tq]) == (p, e, t)
                pairs.add(frozenset([(p, e, t), (q, eq, tq)]))
    assert len(pairs) == 12 * n   # 12 cube edges, n faces each


def test_drifting_field_is_the_rhs_field_rotated():
    """The march's forcing: at alpha = 0 it is rhs() without noise, and a drift
    by alpha equals the field sampled at the cell centres rotated by -alpha
    about z (checked where a quarter turn maps cells onto cells)."""
    from paper_2009_02171_amd import inputs
    n, nr = 8, 4
    F = inputs.DriftingField(n, nr, seed=4)
    np.testing.assert_allclose(F.field(0.0), inputs.rhs(n, nr, 4, noise=0.0), rtol=0, atol=1e-12)
    # panel 0 (+x) drifted by pi/2 equals panel 3 (-y): F(phi - pi/2) at +x is F at -y
    f = F.field(np.pi / 2)
    f0 = F.field(0.0)
    np.testing.assert_allclose(f[0], f0[3], rtol=0, atol=1e-10)
