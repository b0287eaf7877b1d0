"""Oracle pins of the nonlinear terms and the explicit parts of the time step
(Sec. 3.1, eq. nonlinearoperator, tsvelocity, tsmag; Sec. 3.2, eq.
nonlinearint).

* (a.grad)b in the conservative form is exactly conservative: the
  volume-weighted sum over the shell of each component is the wall flux, which
  vanishes for a no-slip a (interior faces cancel, panel-edge faces by the mean
  of the two one-sided fluxes).
* Second-order consistency with closed forms: a solid-body rotation advecting
  a quadratic field (walls included: the rotation has no normal component),
  the position field x advecting it away from the walls (div x = 3 enters the
  conservative form), and a no-slip swirl advecting itself (convergent at the
  cube corners too).
* f1, f3 are the stated combinations of the four advections; bilinearity.
* The Crank-Nicolson right-hand side is (I + (Delta t/2) L) xhat plus the
  explicit terms, with L read off the operator at two time steps.
"""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs


def _fields(n, nr):
    xyz, vol = O.cell_geometry(O.Problem(n, nr))
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    rot = np.zeros((6, nr, n, n, 4))
    rot[..., 0], rot[..., 1] = -y, x
    pos = np.zeros((6, nr, n, n, 4))
    pos[..., :3] = xyz
    b = np.zeros((6, nr, n, n, 4))
    b[..., 0], b[..., 1], b[..., 2] = x * y, y * z, z * x
    return xyz, vol, rot, pos, b


@pytest.mark.parametrize("kind_a,kind_b", [(0, 0), (0, 1)])
def test_advection_is_conservative_for_a_no_slip_carrier(kind_a, kind_b):
    n, nr = 8, 4
    _, vol = O.cell_geometry(O.Problem(n, nr))
    a = inputs.random_field((6, nr, n, n, 4), 1)
    b = inputs.random_field((6, nr, n, n, 4), 2)
    f = O.advect(n, nr, kind_a, a, kind_b, b)
    scale = np.abs(f).max() * vol.sum()
    for c in range(3):
        assert abs((vol * f[..., c]).sum()) <= 1e-14 * scale
    assert (f[..., 3] == 0).all()


def test_advection_conserves_up_to_the_wall_flux():
    """A pseudo-vacuum carrier crosses the walls: the shell sum equals the sum of
    the wall fluxes (a_f . sqrt(g) g^3) b_f h^2, computed here from the ghost
    rules written out (no-slip b: b_f = 0 at the walls, so the sum is 0; with a
    pseudo-vacuum b it is not)."""
    n, nr = 8, 4
    xyz, vol, _, _, _ = _fields(n, nr)
    a = inputs.random_field((6, nr, n, n, 4), 3)
    b = inputs.random_field((6, nr, n, n, 4), 4)
    f0 = O.advect(n, nr, 1, a, 0, b)
    scale = np.abs(f0).max() * vol.sum()
    assert max(abs((vol * f0[..., c]).sum()) for c in range(3)) <= 1e-14 * scale
    f1 = O.advect(n, nr, 1, a, 1, b)
    # wall fluxes with the pseudo-vacuum ghost g = -v + (1 + q)(n.v) n, q = (r_in / r_g)^2
    h, hr = np.pi / 2 / n, (O.RO - O.RI) / nr
    total = np.zeros(3)
    for kin, kg, sgn in ((0, -1, -1.0), (nr - 1, nr, 1.0)):
        r_in, r_g = O.RI + (kin + 0.5) * hr, O.RI + (kg + 0.5) * hr
        r_f = O.RI if kin == 0 else O.RO
        q = (r_in / r_g) ** 2
        nrm = xyz[:, kin] / np.linalg.norm(xyz[:, kin], axis=-1, keepdims=True)

        def face(v):
            vin = v[:, kin, ..., :3]
            vn = (vin * nrm).sum(-1, keepdims=True)
            return 0.5 * (vin + (-vin + (1 + q) * vn * nrm))

        # sqrt(g) at the wall = r_f^2 * (sqrt(g)/r^2), the latter = V / (r_in^2 h^2 hr) of the wall cell
        sg = r_f ** 2 * vol[:, kin] / (r_in ** 2 * h * h * hr)
        flux = sgn * sg * (face(a) * nrm).sum(-1) * h * h
        total += (flux[..., None] * face(b)).sum(axis=(0, 1, 2))
    got = np.array([(vol * f1[..., c]).sum() for c in range(3)])
    np.testing.assert_allclose(got, total, rtol=1e-10, atol=1e-14 * np.abs(f1).max() * vol.sum())
    assert np.abs(total).max() > 1e-6 * np.abs(f1).max() * vol.sum()


def test_advection_second_order_closed_forms():
    errs = {"rot": [], "pos": [], "swirl": []}
    for n in (8, 16):
        nr = n // 2
        xyz, vol, rot, pos, b = _fields(n, nr)
        x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
        # (zhat x x).grad of (xy, yz, zx) = (x^2 - y^2, xz, -yz); no normal component at the walls
        ex = np.stack([x * x - y * y, x * z, -y * z], -1)
        f = O.advect(n, nr, 0, rot, 0, b)[..., :3]
        errs["rot"].append(np.abs(f - ex).max() / np.abs(ex).max())
        # div(x b_c) = (x.grad) b_c + 3 b_c = 5 b_c for b of degree 2 (away from the walls, whose
        # pseudo-vacuum ghost is not that of the position field)
        ex = 5 * b[..., :3]
        f = O.advect(n, nr, 1, pos, 0, b)[..., :3]
        errs["pos"].append(np.abs(f[:, 1:-1] - ex[:, 1:-1]).max() / np.abs(ex).max())
        # u = s(r) zhat x x with s = (r - ri)(ro - r): no-slip, tangential; (u.grad)u = s zhat x u
        r = np.linalg.norm(xyz, axis=-1)
        s = (r - O.RI) * (O.RO - r)
        u = np.zeros_like(rot)
        u[..., 0], u[..., 1] = -y * s, x * s
        ex = np.stack([-s * u[..., 1], s * u[..., 0], 0 * s], -1)
        f = O.advect(n, nr, 0, u, 0, u)[..., :3]
        errs["swirl"].append(np.abs(f - ex).max() / np.abs(ex).max())
    print(errs)
    assert errs["rot"][1] < 0.01 and errs["rot"][0] / errs["rot"][1] > 3.5
    assert errs["pos"][1] < 0.006 and errs["pos"][0] / errs["pos"][1] > 3.5
    # the cube corners' one-sided interpolation limits the swirl's order there
    assert errs["swirl"][1] < 0.012 and errs["swirl"][0] / errs["swirl"][1] > 2.4


def test_nonlinear_terms_are_their_combinations_and_bilinear():
    n, nr = 8, 4
    u = inputs.random_field((6, nr, n, n, 4), 5)
    B = inputs.random_field((6, nr, n, n, 4), 6)
    cB = 0.37
    f1, f3 = O.nonlinear(n, nr, u, B, cB)
    want1 = -O.advect(n, nr, 0, u, 0, u) + cB * O.advect(n, nr, 1, B, 1, B)
    want3 = O.advect(n, nr, 1, B, 0, u) - O.advect(n, nr, 0, u, 1, B)
    np.testing.assert_array_equal(f1, want1)
    np.testing.assert_array_equal(f3, want3)
    # bilinear: (2u) advecting B is twice u advecting B; the pressure slot is never read
    u2 = u.copy()
    u2[..., 3] = 7.0
    a1 = O.advect(n, nr, 0, 2 * u, 1, B)
    a2 = O.advect(n, nr, 0, u2, 1, B)
    np.testing.assert_allclose(a1, 2 * a2, rtol=1e-13, atol=1e-13 * np.abs(a1).max())


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_cn_rhs_is_i_plus_half_dt_l(kind):
    """2 xhat - A_dt xhat = xhat + (Delta t/2) L xhat: with L read off the
    operator's rows at another dt (A_dt = I - dt M, M independent of dt in this
    scaling), 2x - A_dt x = x + dt M x; VP and BP on the vector rows (their
    scalar rows are the divergence rows, set to 0), VT on every row (its Theta
    row is a time-stepped equation, eq. tstemperature)."""
    n, nr = 8, 4
    x = inputs.random_field((6, nr, n, n, 4), 7)
    fn = inputs.random_field((6, nr, n, n, 4), 8)
    fm = inputs.random_field((6, nr, n, n, 4), 9)
    dt = 2e-3
    pb = O.Problem(n, nr, kind=kind, dt=dt)
    pb1 = O.Problem(n, nr, kind=kind, dt=1.0)
    xv = x.copy()
    if kind != 2:
        xv[..., 3] = 0.0
    Mx = xv - O.apply(pb1, xv)                 # dt = 1: A = I - M
    got = O.cn_rhs(pb, x, fn, 0.3, fm=fm, c2=-0.1)
    want = xv + dt * Mx + 0.3 * fn - 0.1 * fm
    if kind != 2:
        want[..., 3] = 0.0
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
