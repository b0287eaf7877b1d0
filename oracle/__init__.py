"""Plain FP64 CPU oracle for the cubed-sphere shell solver (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``csdyn_ref.c`` (plain C, no
shared code with the HIP path) through ctypes, plus a few NumPy helpers.

Every function follows a passage of Yin et al., arXiv 2009.02171:
the grid and metric (Sec. 3.2), the finite-volume operators (Sec. 3.2,
eq. divdiscretization), the two systems of the approximate factorization
(Sec. 3.1), the RAS / two-level preconditioners (Sec. 3.3, eq. onelevel,
twolevel) and right-preconditioned restarted GMRES (Sec. 3.3).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csdyn_ref.c")
_LIB = os.path.join(_HERE, "libcsdyn_ref.so")

OK, ENOTCONV, EINVAL, EZEROPIVOT, ENOMEM, EBREAKDOWN = 0, 1, -1, -3, -4, -5
RI, RO = 7.0 / 13.0, 20.0 / 13.0   # Sec. 2: r_i = 7/13, r_o = 20/13


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("nr", C.c_int32), ("ri", C.c_double), ("ro", C.c_double)]


class Op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dt", C.c_double), ("ekman", C.c_double), ("pm", C.c_double),
                ("ra", C.c_double), ("pr", C.c_double)]


class RasOpts(C.Structure):
    _fields_ = [("sub", C.c_int32 * 3), ("overlap", C.c_int32), ("levels", C.c_int32),
                ("coarse_rtol", C.c_double), ("coarse_restart", C.c_int32), ("coarse_maxit", C.c_int32),
                ("precision", C.c_int32)]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("flexible", C.c_int32),
                ("rtol", C.c_double), ("atol", C.c_double)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("inner_iters", C.c_int64),
                ("relres_true", C.c_double), ("relres_est", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER
        d, i32, i64 = P(C.c_double), P(C.c_int32), P(C.c_int64)
        _lib.ref_cell_geometry.argtypes = [P(Grid), d, d]
        _lib.ref_metric.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, d, d, d]
        _lib.ref_seam_tables.argtypes = [P(Grid), i32, i32, i32, i32, d, i32, i32, i32]
        _lib.ref_operator_apply.argtypes = [P(Grid), P(Op), d, d]
        _lib.ref_operator_rows.argtypes = [P(Grid), P(Op), d, C.c_int64, i64, d]
        _lib.ref_assemble.argtypes = [P(Grid), P(Op), i64, i32, d]
        _lib.ref_pc_setup.argtypes = [P(Grid), P(Op), P(RasOpts), P(C.c_void_p)]
        _lib.ref_pc_destroy.argtypes = [C.c_void_p]
        _lib.ref_pc_destroy.restype = None
        _lib.ref_pc_apply.argtypes = [C.c_void_p, d, d]
        _lib.ref_pc_subdomain.argtypes = [C.c_void_p, C.c_int, C.c_int, i64, i64, i64, i32, i64, i32, d]
        _lib.ref_pc_count.argtypes = [C.c_void_p, C.c_int]
        _lib.ref_pc_inner.argtypes = [C.c_void_p]
        _lib.ref_pc_inner.restype = C.c_void_p
        _lib.ref_pc_inner_iters.argtypes = [C.c_void_p]
        _lib.ref_pc_inner_iters.restype = C.c_int64
        _lib.ref_ilu0_csr.argtypes = [C.c_int64, i64, i32, d]
        _lib.ref_subdomain_solve.argtypes = [P(Grid), P(Op), i32, C.c_int, C.c_int, d, d]
        _lib.ref_subdomain_solve_p.argtypes = [P(Grid), P(Op), i32, C.c_int, C.c_int, C.c_int, d, d]
        _lib.ref_project.argtypes = [P(Grid), P(Op), d, d]
        _lib.ref_advect.argtypes = [P(Grid), C.c_int32, d, C.c_int32, d, C.c_int32, d]
        _lib.ref_gmres_solve.argtypes = [P(Grid), P(Op), C.c_void_p, P(GmresOpts), d, d, P(GmresStats)]
        _lib.ref_gmres_solve_hist.argtypes = [P(Grid), P(Op), C.c_void_p, P(GmresOpts), d, d, P(GmresStats), d,
                                              C.c_int]
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")
    return rc


@dataclass(frozen=True)
class Problem:
    """A grid (N x N x Nr cells per panel, Sec. 3.2) and one of the two systems."""
    n: int
    nr: int
    kind: int = 0            # 0 velocity-pressure, 1 magnetic / pseudo-pressure, 2 velocity-temperature
    dt: float = 1e-4
    ekman: float = 1e-3
    pm: float = 5.0
    ri: float = RI
    ro: float = RO
    ra: float = 100.0        # modified Rayleigh number (VT only)
    pr: float = 1.0          # Prandtl number (VT only)

    def grid(self):
        return Grid(self.n, self.nr, self.ri, self.ro)

    def op(self):
        return Op(self.kind, self.dt, self.ekman, self.pm, self.ra, self.pr)

    @property
    def ncell(self):
        return 6 * self.n * self.n * self.nr

    @property
    def nunk(self):
        return 4 * self.ncell

    def shape(self):
        return (6, self.nr, self.n, self.n, 4)


def cell_geometry(pb: Problem):
    """Cell-centre Cartesian coordinates [6,Nr,N,N,3] and volumes V = sqrt(g) hs^2 hr."""
    xyz = np.zeros((6, pb.nr, pb.n, pb.n, 3))
    vol = np.zeros((6, pb.nr, pb.n, pb.n))
    _check(lib().ref_cell_geometry(C.byref(pb.grid()), _dp(xyz), _dp(vol)), "geometry")
    return xyz, vol


def metric(p: int, xi: float, eta: float, r: float):
    sg = C.c_double()
    gcov = np.zeros(9)
    gcon = np.zeros(9)
    lib().ref_metric(p, xi, eta, r, C.byref(sg), _dp(gcov), _dp(gcon))
    return sg.value, gcov.reshape(3, 3), gcon.reshape(3, 3)


def seam_tables(pb: Problem):
    n = pb.n
    gq, gfix, gidx, gm0 = (np.zeros(24 * n, np.int32) for _ in range(4))
    gw = np.zeros(24 * n * 4)
    fq, feq, ftq = (np.zeros(24 * n, np.int32) for _ in range(3))
    _check(lib().ref_seam_tables(C.byref(pb.grid()), _ip(gq), _ip(gfix), _ip(gidx), _ip(gm0), _dp(gw),
                                 _ip(fq), _ip(feq), _ip(ftq)), "seam tables")
    sh = (6, 4, n)
    return dict(q=gq.reshape(sh), fix_i=gfix.reshape(sh), idx=gidx.reshape(sh), m0=gm0.reshape(sh),
                w=gw.reshape(6, 4, n, 4), face_q=fq.reshape(sh), face_e=feq.reshape(sh), face_t=ftq.reshape(sh))


def apply(pb: Problem, x: np.ndarray) -> np.ndarray:
    """y = A x row by row from the stencil definition (Sec. 3.2)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.zeros_like(x)
    _check(lib().ref_operator_apply(C.byref(pb.grid()), C.byref(pb.op()), _dp(x), _dp(y)), "apply")
    return y.reshape(pb.shape())


def apply_rows(pb: Problem, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(A x)[rows] for selected flat row indices (sampled checks at full size)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.zeros(rows.size)
    _check(lib().ref_operator_rows(C.byref(pb.grid()), C.byref(pb.op()), _dp(x), rows.size, _lp(rows), _dp(y)),
           "apply_rows")
    return y


def project(pb: Problem, x: np.ndarray) -> np.ndarray:
    """Step 3 (Sec. 3.1): (u~ - dt grad_h P, D_f F) from a solution x = (u~, P)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    out = np.zeros_like(x)
    _check(lib().ref_project(C.byref(pb.grid()), C.byref(pb.op()), _dp(x), _dp(out)), "project")
    return out.reshape(pb.shape())


def assemble(pb: Problem):
    """Global CSR (scipy) of A with the structural pattern."""
    import scipy.sparse as sp
    nrow = pb.nunk
    rp = np.zeros(nrow + 1, np.int64)
    _check(lib().ref_assemble(C.byref(pb.grid()), C.byref(pb.op()), _lp(rp), None, None), "assemble")
    ci = np.zeros(rp[-1], np.int32)
    v = np.zeros(rp[-1])
    _check(lib().ref_assemble(C.byref(pb.grid()), C.byref(pb.op()), _lp(rp), _ip(ci), _dp(v)), "assemble")
    return sp.csr_matrix((v, ci, rp), shape=(nrow, nrow))


class Preconditioner:
    """One-level RAS / two-level hybrid RAS with ILU(0) (Sec. 3.3); levels=3 repeats the
    hybrid construction on the coarse grid (its coarse solve is FGMRES preconditioned by
    the coarse grid's own two-level hybrid, with sub/4 boxes on the coarsest grid)."""

    def __init__(self, pb: Problem, sub=(4, 4, 4), overlap=1, levels=1, coarse_rtol=0.1,
                 coarse_restart=30, coarse_maxit=200, precision=0):
        self.pb = pb
        o = RasOpts((C.c_int32 * 3)(*sub), overlap, levels, coarse_rtol, coarse_restart, coarse_maxit, precision)
        h = C.c_void_p()
        rc = lib().ref_pc_setup(C.byref(pb.grid()), C.byref(pb.op()), C.byref(o), C.byref(h))
        self.status = rc
        _check(rc, "pc setup")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ref_pc_destroy(h)
            self.h = None

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        y = np.zeros_like(x)
        lib().ref_pc_apply(self.h, _dp(x), _dp(y))
        return y.reshape(self.pb.shape())

    def count(self, coarse=False):
        return lib().ref_pc_count(self.h, int(coarse))

    def inner_iters(self):
        """Coarse-solve iterations accumulated by apply() calls since the last solve started."""
        return lib().ref_pc_inner_iters(self.h)

    def inner_apply(self, x):
        """levels=3: the coarse grid's two-level hybrid applied to a coarse-grid vector."""
        ih = lib().ref_pc_inner(self.h)
        if not ih:
            raise ValueError("no inner preconditioner (levels < 3)")
        pc = Problem(self.pb.n // 2, self.pb.nr // 2, self.pb.kind, self.pb.dt, self.pb.ekman, self.pb.pm, self.pb.ri,
                     self.pb.ro)
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        y = np.zeros_like(x)
        lib().ref_pc_apply(C.c_void_p(ih), _dp(x), _dp(y))
        return y.reshape(pc.shape())

    def subdomain(self, s, coarse=False):
        """Local cells, owned flags and the ILU(0) factors (L strictly lower, U upper) as CSR."""
        import scipy.sparse as sp
        nloc, nnz = C.c_int64(), C.c_int64()
        _check(lib().ref_pc_subdomain(self.h, int(coarse), s, C.byref(nloc), C.byref(nnz), None, None, None, None,
                                      None), "subdomain")
        gcell = np.zeros(nloc.value, np.int64)
        owned = np.zeros(nloc.value, np.int32)
        rp = np.zeros(4 * nloc.value + 1, np.int64)
        ci = np.zeros(nnz.value, np.int32)
        v = np.zeros(nnz.value)
        lib().ref_pc_subdomain(self.h, int(coarse), s, C.byref(nloc), C.byref(nnz), _lp(gcell), _ip(owned), _lp(rp),
                               _ip(ci), _dp(v))
        m = 4 * nloc.value
        return gcell, owned.astype(bool), sp.csr_matrix((v, ci, rp), shape=(m, m))


def subdomain_solve(pb: Problem, sub, s, x, overlap=1, precision=0):
    """Owned part of one subdomain's ILU(0) solve, (L_s U_s)^{-1} R_s x, written into a
    NaN-filled full vector (only subdomain s is built; for sampled checks at full size).
    precision=1: FP32 factors and FP32 sweeps."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.full_like(x, np.nan)
    sb = np.array(sub, dtype=np.int32)
    _check(lib().ref_subdomain_solve_p(C.byref(pb.grid()), C.byref(pb.op()), _ip(sb), overlap, s, precision, _dp(x),
                                       _dp(y)), "subdomain_solve")
    return y.reshape(pb.shape())


def gmres(pb: Problem, b, x0=None, pc: Preconditioner | None = None, restart=30, maxit=1000, flexible=False,
          rtol=1e-8, atol=0.0, history=False):
    """Right-preconditioned restarted (F)GMRES (Sec. 3.3).  Returns (x, stats, status); with
    history=True, stats["hist"] holds the residual estimate after every Arnoldi step."""
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    st = GmresStats()
    o = GmresOpts(restart, maxit, int(flexible), rtol, atol)
    hist = np.full(maxit, np.nan)
    rc = lib().ref_gmres_solve_hist(C.byref(pb.grid()), C.byref(pb.op()), pc.h if pc else None, C.byref(o), _dp(b),
                                    _dp(x), C.byref(st), _dp(hist) if history else None, maxit if history else 0)
    stats = dict(iters=st.iters, restarts=st.restarts, inner_iters=st.inner_iters, relres_true=st.relres_true,
                 relres_est=st.relres_est)
    if history:
        stats["hist"] = hist[:st.iters].copy()
    return x.reshape(pb.shape()), stats, rc


def ilu0(a):
    """ILU(0) of a scipy CSR matrix (sorted indices); returns (status, factors as CSR)."""
    a = a.tocsr().copy()
    a.sort_indices()
    rp = a.indptr.astype(np.int64)
    ci = a.indices.astype(np.int32)
    v = a.data.astype(np.float64).copy()
    rc = lib().ref_ilu0_csr(a.shape[0], _lp(rp), _ip(ci), _dp(v))
    import scipy.sparse as sp
    return rc, sp.csr_matrix((v, ci, rp), shape=a.shape)


def advect(n: int, nr: int, kind_a: int, a: np.ndarray, kind_b: int, b: np.ndarray, scalar: bool = False) -> np.ndarray:
    """(a . grad) b in the conservative form div(a b_c) per Cartesian component
    (Sec. 3.2, eq. nonlinearint), a with the ghost rules of system kind_a, b
    with those of kind_b; the vector part of b (scalar part of the result 0),
    or with scalar=True the scalar part (vector part of the result 0)."""
    g = Grid(n, nr, RI, RO)
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    out = np.zeros_like(a)
    _check(lib().ref_advect(C.byref(g), kind_a, _dp(a), kind_b, _dp(b), int(scalar), _dp(out)), "advect")
    return out.reshape(6, nr, n, n, 4)


def nonlinear(n: int, nr: int, u: np.ndarray, B: np.ndarray, cB: float, T: np.ndarray | None = None):
    """Sec. 3.1, eq. nonlinearoperator: f1 = -(u.grad)u + cB (B.grad)B,
    f3 = (B.grad)u - (u.grad)B (u: no-slip ghosts, B: pseudo-vacuum); with
    the velocity-temperature state T = (u, Theta) also f2 = -(u.grad)Theta
    (isothermal Theta ghosts) in the scalar slot."""
    f1 = -advect(n, nr, 0, u, 0, u) + cB * advect(n, nr, 1, B, 1, B)
    f3 = advect(n, nr, 1, B, 0, u) - advect(n, nr, 0, u, 1, B)
    if T is None:
        return f1, f3
    f1 = f1 - advect(n, nr, 0, u, 2, T, scalar=True)
    return f1, f3


def cn_rhs(pb: Problem, xhat: np.ndarray, fn: np.ndarray, c1: float, fm=None, c2: float = 0.0, gf=None,
           c3: float = 0.0) -> np.ndarray:
    """Sec. 3.1, eqs. tsvelocity / tsmag in this system's scaling: the vector
    part of (I + (Delta t/2) L) xhat = 2 xhat - A xhat (the vector rows of A are
    I - (Delta t/2) L and do not read the scalar part), plus the explicit terms;
    scalar part 0."""
    x = np.array(xhat, dtype=np.float64).reshape(pb.shape())
    out = 2.0 * x - apply(pb, x) + c1 * np.asarray(fn).reshape(pb.shape())
    if fm is not None and c2 != 0.0:
        out += c2 * np.asarray(fm).reshape(pb.shape())
    if gf is not None and c3 != 0.0:
        out += c3 * np.asarray(gf).reshape(pb.shape())
    if pb.kind != 2:       # VP, BP: the divergence rows; VT keeps its Theta row (eq. tstemperature)
        out[..., 3] = 0.0
    return out


def vector_rows(pb: Problem, x: np.ndarray) -> np.ndarray:
    """((A x)_vec, 0): Step 2's right-hand side after a VT Step 1 (Sec. 3.1, eq. tsp)."""
    out = apply(pb, x)
    out[..., 3] = 0.0
    return out


def step3_state(pb: Problem, x: np.ndarray) -> np.ndarray:
    """Sec. 3.1, eq. ubtilde: (u~ - dt grad_h P, P) from a solution (u~, P)."""
    out = project(pb, x)
    out[..., 3] = np.asarray(x).reshape(pb.shape())[..., 3]
    return out


def project_pressure(pb: Problem, b):
    """Zero volume-weighted mean of the scalar component (Neumann solvability)."""
    _, vol = cell_geometry(pb)
    b = np.array(b, dtype=np.float64).reshape(pb.shape())
    b[..., 3] -= (vol * b[..., 3]).sum() / vol.sum()
    return b
