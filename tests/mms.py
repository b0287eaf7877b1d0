"""Manufactured solutions for the operator-order pins (test helper).

The exact fields satisfy the wall conditions of the two systems: no-slip u,
Neumann P (dP/dr = 0), pseudo-vacuum B (tangential B = 0 and
d(r^2 B_r)/dr = 0) and Dirichlet P_b.  Right-hand sides are the continuous
operators applied to them, differentiated symbolically with sympy.
"""
import numpy as np
import sympy as sp

X, Y, Z = sp.symbols("x y z", real=True)
R = sp.sqrt(X**2 + Y**2 + Z**2)


def _lap(f):
    return sp.diff(f, X, 2) + sp.diff(f, Y, 2) + sp.diff(f, Z, 2)


def _div(v):
    return sp.diff(v[0], X) + sp.diff(v[1], Y) + sp.diff(v[2], Z)


def fields(kind, ri, ro):
    s = (R - ri) / (ro - ri)
    nx, ny, nz = X / R, Y / R, Z / R
    if kind == 0:
        w = (R - ri) * (ro - R)
        u = [w * (sp.sin(Y) + Z), w * sp.cos(X) * Z, w * X * Y]
        p = sp.cos(sp.pi * s) * (nx * ny + nz)
    else:
        g = 1 + nx * nz + ny
        h = sp.cos(sp.pi * s)
        w2 = ((R - ri) * (ro - R)) ** 2
        t = [sp.sin(Y), Z * X, sp.cos(X + Z)]
        n = [nx, ny, nz]
        u = [g * h * n[a] / R**2 + w2 * t[a] for a in range(3)]
        p = sp.sin(sp.pi * s) * (nx * ny + nz)
    return u, p


def rhs_exprs(kind, ri, ro, dt, ekman, pm):
    u, p = fields(kind, ri, ro)
    if kind == 0:
        cor = [-u[1], u[0], 0]
        bu = [u[a] - dt * (ekman * _lap(u[a]) - 2 * cor[a]) for a in range(3)]
    else:
        bu = [u[a] - dt * ekman / pm * _lap(u[a]) for a in range(3)]
    bp = _div(u) - dt * _lap(p)
    return u + [p], bu + [bp]


def evaluate(exprs, xyz):
    out = []
    for e in exprs:
        f = sp.lambdify((X, Y, Z), e, "numpy")
        v = f(xyz[..., 0], xyz[..., 1], xyz[..., 2])
        out.append(np.broadcast_to(v, xyz.shape[:-1]).astype(np.float64))
    return np.stack(out, -1)
