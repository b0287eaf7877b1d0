"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds none of the solver's arithmetic: it only samples a smooth
random field on the cubed-sphere cell centres.  Right-hand side recipe per
component c: a sum of real orthonormal spherical harmonics Y_lm (l <= 8) times
Chebyshev polynomials T_q (q <= 4) of the normalised radius, with N(0,1)
coefficients, plus U(-1e-3, 1e-3) noise per unknown.  All coefficients are
drawn first, then the noise, from numpy's PCG64 ``default_rng(seed)``.

Cell centres follow the grid of Sec. 3.2 (xi_i = -pi/4 + (i+1/2) h_s,
r_k = r_i + (k+1/2) h_r) with panels 0-3 equatorial (+x, +y, -x, -y),
4 = +z and 5 = -z.
"""
from __future__ import annotations

import numpy as np

LMAX, QMAX = 8, 4
RI, RO = 7.0 / 13.0, 20.0 / 13.0

# global = M[p] @ (1, tan xi, tan eta)
_PANELS = np.array([
    [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
    [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
    [[-1, 0, 0], [0, -1, 0], [0, 0, 1]],
    [[0, 1, 0], [-1, 0, 0], [0, 0, 1]],
    [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
    [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
], dtype=np.float64)


def cell_directions(n: int) -> np.ndarray:
    """Unit vectors to the (xi, eta) cell centres, [6, N, N, 3] indexed [p, j, i]."""
    h = np.pi / (2 * n)
    a = -np.pi / 4 + (np.arange(n) + 0.5) * h
    X = np.tan(a)[None, :]
    Y = np.tan(a)[:, None]
    loc = np.stack([np.ones((n, n)), np.broadcast_to(X, (n, n)), np.broadcast_to(Y, (n, n))], -1)
    loc /= np.linalg.norm(loc, axis=-1, keepdims=True)
    return np.einsum("pab,jib->pjia", _PANELS, loc)


def _real_sph(lmax: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    from scipy.special import sph_harm_y
    cols = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                cols.append(np.sqrt(2.0) * (-1) ** m * y.real)
            elif m < 0:
                cols.append(np.sqrt(2.0) * (-1) ** m * y.imag)
            else:
                cols.append(y.real)
    return np.stack(cols, -1)


def rhs(n: int, nr: int, seed: int, ri: float = RI, ro: float = RO, noise: float = 1e-3) -> np.ndarray:
    """Seeded right-hand side, float64 [6, Nr, N, N, 4] (panel, k, j, i, component)."""
    return _rhs(n, nr, np.random.default_rng(seed), ri, ro, noise)


def shell_case(s: int, n: int, nr: int, ri: float = RI, ro: float = RO):
    """Shell s of the uneven-size batch: (Ekman number, right-hand side), both
    from the stream default_rng(100 + s), the Ekman number drawn first,
    log-uniform in [1e-4, 1e-3]."""
    rng = np.random.default_rng(100 + s)
    ekman = 10.0 ** rng.uniform(-4.0, -3.0)
    return ekman, _rhs(n, nr, rng, ri, ro, 1e-3)


def _rhs(n, nr, rng, ri, ro, noise):
    nlm = (LMAX + 1) ** 2
    coef = rng.standard_normal((4, nlm, QMAX + 1))
    d = cell_directions(n)
    theta = np.arccos(np.clip(d[..., 2], -1.0, 1.0))
    phi = np.arctan2(d[..., 1], d[..., 0])
    Y = _real_sph(LMAX, theta, phi)                       # [6, N, N, nlm]
    r = ri + (np.arange(nr) + 0.5) * (ro - ri) / nr
    s = 2.0 * (r - ri) / (ro - ri) - 1.0
    T = np.polynomial.chebyshev.chebvander(s, QMAX)       # [Nr, 5]
    b = np.einsum("pjil,kq,clq->pkjic", Y, T, coef, optimize=True)
    b += rng.uniform(-noise, noise, size=b.shape)
    return np.ascontiguousarray(b)


def random_field(shape, seed: int) -> np.ndarray:
    """Plain seeded N(0,1) array (operator and preconditioner probes)."""
    return np.random.default_rng(seed).standard_normal(shape)


NET_WIDTHS = (32, 48, 64, 128)


def net_layer_shapes(widths=NET_WIDTHS, cin=8, cout=4):
    """(cout, cin) of the eight 3x3x3 convolutions of the learned-guess network."""
    c0, c1, c2, c3 = widths
    return [(c0, cin), (c1, c0), (c2, c1), (c3, c2), (c2, c3), (c1, c2), (c0, c1), (cout, c0)]


def net_params(seed, widths=NET_WIDTHS):
    """Initial network parameters, flat FP32, layer by layer w[cout][27][cin]
    then bias[cout]: He-uniform weights (bound sqrt(6 / (27 cin))), the last
    layer scaled by 0.1 so the initial correction is small, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    shapes = net_layer_shapes(widths)
    for li, (co, ci) in enumerate(shapes):
        bound = np.sqrt(6.0 / (27 * ci))
        w = rng.uniform(-bound, bound, (co, 27, ci))
        if li == len(shapes) - 1:
            w *= 0.1
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


class DriftingField:
    """The smooth part of ``rhs(n, nr, seed)`` (no noise) drifted in longitude:
    F_alpha(r, theta, phi) = F(r, theta, phi - alpha), each component treated
    as a scalar field.  ``angular(alpha)`` gives A[p, j, i, c, q] and
    ``radial`` T[k, q] with F_alpha[p, k, j, i, c] = sum_q A[p, j, i, c, q] T[k, q]."""

    def __init__(self, n: int, nr: int, seed: int, ri: float = RI, ro: float = RO):
        rng = np.random.default_rng(seed)
        self.coef = rng.standard_normal((4, (LMAX + 1) ** 2, QMAX + 1))
        d = cell_directions(n)
        self.theta = np.arccos(np.clip(d[..., 2], -1.0, 1.0))
        self.phi = np.arctan2(d[..., 1], d[..., 0])
        r = ri + (np.arange(nr) + 0.5) * (ro - ri) / nr
        self.radial = np.polynomial.chebyshev.chebvander(2.0 * (r - ri) / (ro - ri) - 1.0, QMAX)

    def angular(self, alpha: float) -> np.ndarray:
        Y = _real_sph(LMAX, self.theta, self.phi - alpha)
        return np.einsum("pjil,clq->pjicq", Y, self.coef, optimize=True)

    def field(self, alpha: float) -> np.ndarray:
        return np.ascontiguousarray(np.einsum("pjicq,kq->pkjic", self.angular(alpha), self.radial, optimize=True))


def benchmark_b0(n: int, nr: int, ri: float = RI, ro: float = RO) -> np.ndarray:
    """The benchmark's initial magnetic field (Sec. 4.2, eq. initial) at the
    cell centres in Cartesian components, float64 [6, Nr, N, N, 4] with the
    scalar slot 0 (theta colatitude from +z, phi longitude):
        B_r     = 5/8 (9 r^3 - 4 (4 + 3 (ri + ro)) r^2 + 6 (4 ro + ri (4 + 3 ro)) r - 48 ri ro) / r cos(theta)
        B_theta = -15/4 (r - ri)(r - ro)(3 r - 4) / r sin(theta)
        B_phi   = 15/8 sin(pi (r - ri)) sin(2 theta)."""
    d = cell_directions(n)                                   # [6, N, N, 3]
    th = np.arccos(np.clip(d[..., 2], -1.0, 1.0))[:, None]   # [6, 1, N, N]
    ph = np.arctan2(d[..., 1], d[..., 0])[:, None]
    r = (ri + (np.arange(nr) + 0.5) * (ro - ri) / nr)[None, :, None, None]
    br = 5.0 / 8.0 * (9 * r**3 - 4 * (4 + 3 * (ri + ro)) * r**2 + 6 * (4 * ro + ri * (4 + 3 * ro)) * r
                      - 48 * ri * ro) / r * np.cos(th)
    bt = -15.0 / 4.0 * (r - ri) * (r - ro) * (3 * r - 4) / r * np.sin(th)
    bp = 15.0 / 8.0 * np.sin(np.pi * (r - ri)) * np.sin(2 * th)
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    out = np.zeros((6, nr, n, n, 4))
    out[..., 0] = br * st * cp + bt * ct * cp - bp * sp
    out[..., 1] = br * st * sp + bt * ct * sp + bp * cp
    out[..., 2] = br * ct - bt * st
    return out


def benchmark_theta0(n: int, nr: int, ri: float = RI, ro: float = RO) -> np.ndarray:
    """The benchmark's initial temperature perturbation (Sec. 4.2, eq. initial)
    in the scalar slot of a velocity-temperature vector, float64
    [6, Nr, N, N, 4] (vector slots 0):
        Theta = 21 / sqrt(17920 pi) (1 - 3 x^2 + 3 x^4 - x^6) sin^4(theta) cos(4 phi),
        x = 2 r - ri - ro."""
    d = cell_directions(n)
    th = np.arccos(np.clip(d[..., 2], -1.0, 1.0))[:, None]
    ph = np.arctan2(d[..., 1], d[..., 0])[:, None]
    r = (ri + (np.arange(nr) + 0.5) * (ro - ri) / nr)[None, :, None, None]
    x = 2 * r - ri - ro
    out = np.zeros((6, nr, n, n, 4))
    out[..., 3] = 21.0 / np.sqrt(17920.0 * np.pi) * (1 - 3 * x**2 + 3 * x**4 - x**6) * np.sin(th)**4 * np.cos(4 * ph)
    return out
