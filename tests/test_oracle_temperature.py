"""Oracle pins of the velocity-temperature system (the VTBE's u and Theta
block, Sec. 3.1 eq. tsvelocity, tstemperature; operators of eq.
linearoperator) and of the temperature's nonlinear term f2 = -(u.grad)Theta.

* Its velocity rows with Theta = 0 are the VP system's velocity rows.
* Its Theta row with u = 0 is Theta - dt (E/Pr) lap_D Theta, with the
  Dirichlet Laplacian read off the BP system's scalar row at dt = 1 (the
  isothermal wall takes the same ghost rule as P_b).
* The couplings are the closed forms -(Delta t/2) R1(Theta) = -dt Ra/r_o Theta x
  and -(Delta t/2) R2(u) = -dt E r_i r_o / r^3 (x . u) at the cell centres.
* f2 is conservative and converges on a closed form (about second order,
  1.6 in the maximum norm at the cube corners).
* GMRES with one-level RAS solves the system.
"""
import numpy as np
import pytest

import oracle as O
from paper_2009_02171_amd import inputs


def _vt(n, nr, **kw):
    return O.Problem(n, nr, kind=2, **kw)


def test_velocity_rows_are_the_vp_rows():
    n, nr = 8, 4
    x = inputs.random_field((6, nr, n, n, 4), 1)
    xt = x.copy()
    xt[..., 3] = 0.0
    a = O.apply(_vt(n, nr, dt=1e-3), xt)[..., :3]
    b = O.apply(O.Problem(n, nr, kind=0, dt=1e-3), x)[..., :3]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(b).max())


def test_theta_row_is_identity_minus_dirichlet_laplacian():
    n, nr, dt, E, Pr = 8, 4, 2e-3, 1e-3, 0.7
    th = inputs.random_field((6, nr, n, n, 4), 2)
    th[..., :3] = 0.0
    got = O.apply(_vt(n, nr, dt=dt, ekman=E, pr=Pr), th)[..., 3]
    lapD = -O.apply(O.Problem(n, nr, kind=1, dt=1.0), th)[..., 3]     # D(0) - 1 * lap_D Theta
    want = th[..., 3] - dt * E / Pr * lapD
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_couplings_are_the_closed_forms():
    n, nr, dt, E, Ra = 8, 4, 1e-3, 1e-3, 100.0
    xyz, _ = O.cell_geometry(O.Problem(n, nr))
    r = np.linalg.norm(xyz, axis=-1)
    pb = _vt(n, nr, dt=dt, ekman=E, ra=Ra)
    th = inputs.random_field((6, nr, n, n, 4), 3)
    th[..., :3] = 0.0
    got = O.apply(pb, th)[..., :3]                    # velocity rows of (0, Theta): the buoyancy coupling
    want = -dt * Ra / O.RO * th[..., 3:4] * xyz
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())
    u = inputs.random_field((6, nr, n, n, 4), 4)
    u[..., 3] = 0.0
    got = O.apply(pb, u)[..., 3]                      # Theta row of (u, 0): the R2 coupling
    want = -dt * E * O.RI * O.RO / r**3 * (xyz * u[..., :3]).sum(-1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_temperature_advection_conservative_and_second_order():
    n, nr = 8, 4
    _, vol = O.cell_geometry(O.Problem(n, nr))
    u = inputs.random_field((6, nr, n, n, 4), 5)
    T = inputs.random_field((6, nr, n, n, 4), 6)
    f = O.advect(n, nr, 0, u, 2, T, scalar=True)
    assert (f[..., :3] == 0).all()
    assert abs((vol * f[..., 3]).sum()) <= 1e-14 * np.abs(f).max() * vol.sum()
    errs = []
    for n in (8, 16):
        nr = n // 2
        xyz, _ = O.cell_geometry(O.Problem(n, nr))
        x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
        u = np.zeros((6, nr, n, n, 4))
        u[..., 0], u[..., 1] = -y, x                  # rotation about z: tangential, divergence-free
        T = np.zeros_like(u)
        T[..., 3] = z * x                              # (u.grad)(zx) = -y z
        f = O.advect(n, nr, 0, u, 2, T, scalar=True)[..., 3]
        ex = -y * z
        errs.append(np.abs(f - ex).max() / np.abs(ex).max())
    # the cube corners' one-sided ghost interpolation keeps the maximum-norm order near 1.6 there
    assert errs[1] < 0.015 and errs[0] / errs[1] > 2.8, errs


def test_nonlinear_with_temperature_fills_the_scalar_slot():
    n, nr = 8, 4
    u = inputs.random_field((6, nr, n, n, 4), 7)
    B = inputs.random_field((6, nr, n, n, 4), 8)
    T = inputs.random_field((6, nr, n, n, 4), 9)
    f1, f3 = O.nonlinear(n, nr, u, B, 2.0)
    g1, g3 = O.nonlinear(n, nr, u, B, 2.0, T=T)
    np.testing.assert_array_equal(g1[..., :3], f1[..., :3])
    np.testing.assert_array_equal(g3, f3)
    np.testing.assert_array_equal(g1[..., 3], -O.advect(n, nr, 0, u, 2, T, scalar=True)[..., 3])


def test_vt_solve_converges():
    n, nr = 8, 8
    pb = _vt(n, nr, dt=5e-3)
    b = inputs.rhs(n, nr, seed=10)
    x, st, rc = O.gmres(pb, b, pc=O.Preconditioner(pb, sub=(8, 8, 8), levels=1), rtol=1e-10)
    assert rc == 0 and st["relres_true"] <= 1.0001e-10
    r = b - O.apply(pb, x)
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)


def test_project_rejects_vt():
    pb = _vt(8, 4)
    with pytest.raises(RuntimeError):
        O.project(pb, np.zeros(pb.shape()))
