"""Thin ctypes binding of libcsdyn (include/csdyn.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory (workspaces, vectors) and the
current stream.  The library must be built (``python -m
paper_2009_02171_amd.build``); importing this module on a machine where it
is missing raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsdyn.so")

OK, ENOTCONV, EINVAL, EHIP, EZEROPIVOT, ENOMEM, EBREAKDOWN = 0, 1, -1, -2, -3, -4, -5
VP, BP, VT = 0, 1, 2
RI, RO = 7.0 / 13.0, 20.0 / 13.0


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("nr", C.c_int32), ("ri", C.c_double), ("ro", C.c_double)]


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dt", C.c_double), ("ekman", C.c_double), ("pm", C.c_double),
                ("ra", C.c_double), ("pr", C.c_double)]


class RasOpts(C.Structure):
    _fields_ = [("sub", C.c_int32 * 3), ("overlap", C.c_int32), ("levels", C.c_int32),
                ("coarse_rtol", C.c_double), ("coarse_restart", C.c_int32), ("coarse_maxit", C.c_int32),
                ("precision", C.c_int32), ("storage", C.c_int32), ("values", C.c_int32)]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("flexible", C.c_int32),
                ("rtol", C.c_double), ("atol", C.c_double), ("orth", C.c_int32), ("rhs_relative", C.c_int32),
                ("timing", C.c_int32), ("device_steps", C.c_int32)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("inner_iters", C.c_int64),
                ("relres_true", C.c_double), ("relres_est", C.c_double), ("res0", C.c_double),
                ("res_true", C.c_double), ("bnorm", C.c_double), ("t_ms", C.c_double * 6),
                ("t_span_ms", C.c_double), ("inner2_iters", C.c_int64)]

# phases of GmresStats.t_ms (CSDYN_T_* in csdyn.h)
PHASES = ("op", "pc_fine", "pc_coarse", "pc_interp", "orth", "other")


class RasInfo(C.Structure):
    _fields_ = [("nsd_fine", C.c_int32), ("nsd_coarse", C.c_int32), ("nnz_fine", C.c_int64),
                ("nnz_coarse", C.c_int64), ("box_cells_fine", C.c_int64), ("box_cells_coarse", C.c_int64),
                ("owned_cells_fine", C.c_int64), ("owned_cells_coarse", C.c_int64), ("stored_fine", C.c_int64),
                ("stored_coarse", C.c_int64), ("max_levels_fine", C.c_int32), ("max_levels_coarse", C.c_int32),
                ("precision", C.c_int32), ("lds_fine", C.c_int32), ("lds_coarse", C.c_int32),
                ("box_in_lds_fine", C.c_int32), ("box_in_lds_coarse", C.c_int32), ("threads_fine", C.c_int32),
                ("threads_coarse", C.c_int32), ("structures_fine", C.c_int32), ("structures_coarse", C.c_int32),
                ("blocks_per_cu_fine", C.c_int32), ("blocks_per_cu_coarse", C.c_int32), ("packed_fine", C.c_int32),
                ("packed_coarse", C.c_int32)]


class ConvShape(C.Structure):
    _fields_ = [("batch", C.c_int32), ("d", C.c_int32), ("h", C.c_int32), ("w", C.c_int32), ("cin", C.c_int32),
                ("cout", C.c_int32)]


class GuessInfo(C.Structure):
    _fields_ = [("res_extrap", C.c_double), ("res_net", C.c_double), ("res_guess", C.c_double),
                ("alpha", C.c_double)]


class ProfileEntry(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("size", C.c_int64), ("count", C.c_int64), ("total_ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


# Exported symbols and their signatures, as declared in include/csdyn.h.
_P = C.POINTER
SIGNATURES = {
    "csdyn_op_workspace_bytes": (C.c_int32, [_P(Grid), _P(C.c_size_t)]),
    "csdyn_op_setup": (C.c_int32, [_P(Grid), _P(OpDesc), C.c_void_p, C.c_size_t, C.c_void_p, _P(C.c_void_p)]),
    "csdyn_operator_apply": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_op_destroy": (None, [C.c_void_p]),
    "csdyn_project": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_op_set_tile": (C.c_int32, [C.c_void_p, C.c_int32]),
    "csdyn_ras_workspace_bytes": (C.c_int32, [C.c_void_p, _P(RasOpts), _P(C.c_size_t)]),
    "csdyn_ras_setup": (C.c_int32, [C.c_void_p, _P(RasOpts), C.c_void_p, C.c_size_t, C.c_void_p, _P(C.c_void_p)]),
    "csdyn_ras_apply": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_ras_destroy": (None, [C.c_void_p]),
    "csdyn_ras_inspect": (C.c_int32, [_P(Grid), _P(OpDesc), _P(C.c_int32), C.c_int32, C.c_int32, _P(C.c_int64),
                                      _P(C.c_int64), _P(C.c_int32), _P(C.c_int32), _P(C.c_int64), _P(C.c_int32),
                                      _P(C.c_double)]),
    "csdyn_gmres_workspace_bytes": (C.c_int32, [C.c_void_p, _P(GmresOpts), _P(C.c_size_t)]),
    "csdyn_residual_workspace_bytes": (C.c_int32, [C.c_void_p, _P(C.c_size_t)]),
    "csdyn_batch_workspace_bytes": (C.c_int32, [C.c_int32, _P(C.c_void_p), _P(GmresOpts), _P(C.c_size_t)]),
    "csdyn_batch_setup": (C.c_int32, [C.c_int32, _P(C.c_void_p), _P(C.c_void_p), _P(GmresOpts), C.c_void_p,
                                      C.c_size_t, _P(C.c_void_p)]),
    "csdyn_gmres_solve_batched": (C.c_int32, [C.c_void_p, _P(C.c_void_p), _P(C.c_void_p), C.c_int32, C.c_void_p,
                                              _P(GmresStats)]),
    "csdyn_batch_destroy": (None, [C.c_void_p]),
    "csdyn_batch_modes": (C.c_int32, [C.c_void_p, _P(C.c_int32)]),
    "csdyn_residual_norm": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                        _P(C.c_double)]),
    "csdyn_residual_norm_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, _P(C.c_double)]),
    "csdyn_gmres_solve": (C.c_int32, [C.c_void_p, C.c_void_p, _P(GmresOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_size_t, C.c_void_p, _P(GmresStats)]),
    "csdyn_ras_get_info": (C.c_int32, [C.c_void_p, _P(RasInfo)]),
    "csdyn_profile_begin": (C.c_int32, [C.c_int32]),
    "csdyn_profile_select": (C.c_int32, [C.c_char_p, C.c_int32]),
    "csdyn_profile_end": (C.c_int32, [_P(ProfileEntry), C.c_int32, _P(C.c_int32)]),
    "csdyn_conv3d_sizes": (C.c_int32, [_P(ConvShape), _P(C.c_int64), _P(C.c_int64), _P(C.c_size_t)]),
    "csdyn_conv3d_pack": (C.c_int32, [_P(ConvShape), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_conv3d_fwd": (C.c_int32, [_P(ConvShape), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_conv3d_bwd_data": (C.c_int32, [_P(ConvShape), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p]),
    "csdyn_conv3d_bwd_weight": (C.c_int32, [_P(ConvShape), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_size_t, C.c_void_p]),
    "csdyn_adam_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                    C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "csdyn_net_param_count": (C.c_int32, [_P(C.c_int32), _P(C.c_int64)]),
    "csdyn_net_workspace_bytes": (C.c_int32, [C.c_int32, C.c_int32, _P(C.c_int32), _P(C.c_size_t)]),
    "csdyn_net_setup": (C.c_int32, [C.c_int32, C.c_int32, _P(C.c_int32), C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p, _P(C.c_void_p)]),
    "csdyn_net_get_params": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_net_predict": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_net_loss_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        _P(C.c_double), C.c_void_p]),
    "csdyn_net_train_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                         _P(C.c_double), C.c_void_p]),
    "csdyn_net_destroy": (None, [C.c_void_p]),
    "csdyn_guess_workspace_bytes": (C.c_int32, [C.c_void_p, _P(C.c_size_t)]),
    "csdyn_guess": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                C.c_void_p, C.c_size_t, C.c_void_p, _P(GuessInfo)]),
    "csdyn_march_rhs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "csdyn_nonlinear_workspace_bytes": (C.c_int32, [C.c_void_p, _P(C.c_size_t)]),
    "csdyn_nonlinear": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "csdyn_cn_rhs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                 C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "csdyn_step3_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_vector_rows": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csdyn_last_error": (C.c_char_p, []),
}

_lib = None


def lib(path: str = LIB_PATH):
    """Load libcsdyn.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libcsdyn.so not built at {path}: run python -m paper_2009_02171_amd.build")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CsdynError(RuntimeError):
    def __init__(self, status, what):
        msg = lib().csdyn_last_error().decode()
        super().__init__(f"{what}: status {status}: {msg}")
        self.status = status


def _check(rc, what):
    if rc < 0:
        raise CsdynError(rc, what)
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Operator:
    """y = A x for one system on one grid (csdyn_op_setup / csdyn_operator_apply)."""

    def __init__(self, n, nr, kind=VP, dt=1e-4, ekman=1e-3, pm=5.0, ri=RI, ro=RO, device="cuda", ra=100.0, pr=1.0):
        self.n, self.nr, self.kind = n, nr, kind
        self.dt, self.ekman, self.pm = dt, ekman, pm
        self.device = torch.device(device)
        self.grid = Grid(n, nr, ri, ro)
        self.desc = OpDesc(kind, dt, ekman, pm, ra, pr)
        nb = C.c_size_t()
        _check(lib().csdyn_op_workspace_bytes(C.byref(self.grid), C.byref(nb)), "csdyn_op_workspace_bytes")
        self.ws = _workspace(nb.value, self.device)
        h = C.c_void_p()
        _check(lib().csdyn_op_setup(C.byref(self.grid), C.byref(self.desc), _ptr(self.ws), nb.value, _stream(),
                                    C.byref(h)), "csdyn_op_setup")
        self.h = h

    @property
    def shape(self):
        return (6, self.nr, self.n, self.n, 4)

    def empty(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def apply(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
        y = self.empty() if y is None else y
        _check(lib().csdyn_operator_apply(self.h, _ptr(x), _ptr(y), _stream(stream)), "csdyn_operator_apply")
        return y

    def set_tile(self, tile: int):
        """Stencil workgroup shape: 0 by N, 1: 32x8, 2: 16x16, 3: 64x4, 4: 16x8, 5: 32x4,
        6: FP64 layers requested straight into LDS (16x16; N > 16)."""
        _check(lib().csdyn_op_set_tile(self.h, tile), "csdyn_op_set_tile")

    def project(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        """Step 3: (u~ - dt grad_h P, divergence of the corrected face fluxes)."""
        out = self.empty() if out is None else out
        _check(lib().csdyn_project(self.h, _ptr(x), _ptr(out), _stream(stream)), "csdyn_project")
        return out

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.csdyn_op_destroy(h)
            self.h = None


class RAS:
    """One- or two-level RAS / ILU(0) preconditioner (csdyn_ras_setup / csdyn_ras_apply)."""

    def __init__(self, op: Operator, sub=(4, 4, 4), overlap=1, levels=1, coarse_rtol=0.1, coarse_restart=30,
                 coarse_maxit=200, precision=0, storage=0, values=0):
        self.op = op
        self.opts = RasOpts((C.c_int32 * 3)(*sub), overlap, levels, coarse_rtol, coarse_restart, coarse_maxit,
                            precision, storage, values)
        nb = C.c_size_t()
        _check(lib().csdyn_ras_workspace_bytes(op.h, C.byref(self.opts), C.byref(nb)), "csdyn_ras_workspace_bytes")
        self.ws = _workspace(nb.value, op.device)
        h = C.c_void_p()
        _check(lib().csdyn_ras_setup(op.h, C.byref(self.opts), _ptr(self.ws), nb.value, _stream(), C.byref(h)),
               "csdyn_ras_setup")
        self.h = h

    def apply(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
        y = self.op.empty() if y is None else y
        _check(lib().csdyn_ras_apply(self.h, _ptr(x), _ptr(y), _stream(stream)), "csdyn_ras_apply")
        return y

    def info(self):
        inf = RasInfo()
        _check(lib().csdyn_ras_get_info(self.h, C.byref(inf)), "csdyn_ras_get_info")
        return {k: getattr(inf, k) for k, _ in RasInfo._fields_}

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.csdyn_ras_destroy(h)
            self.h = None


def ras_inspect(n, nr, kind, sub, s, overlap=1, dt=1e-4, ekman=1e-3, pm=5.0, ri=RI, ro=RO):
    """Host-side subdomain data (csdyn_ras_inspect): (gcell, owned, scipy CSR of the ILU(0) factors)."""
    import numpy as np
    import scipy.sparse as sp
    g, d = Grid(n, nr, ri, ro), OpDesc(kind, dt, ekman, pm)
    sb = (C.c_int32 * 3)(*sub)
    nloc, nnz = C.c_int64(), C.c_int64()
    L = lib()
    _check(L.csdyn_ras_inspect(C.byref(g), C.byref(d), sb, overlap, s, C.byref(nloc), C.byref(nnz), None, None, None,
                               None, None), "csdyn_ras_inspect")
    gc = np.zeros(nloc.value, np.int32)
    ow = np.zeros(nloc.value, np.int32)
    rp = np.zeros(4 * nloc.value + 1, np.int64)
    ci = np.zeros(nnz.value, np.int32)
    v = np.zeros(nnz.value)
    P = C.POINTER
    _check(L.csdyn_ras_inspect(C.byref(g), C.byref(d), sb, overlap, s, C.byref(nloc), C.byref(nnz),
                               gc.ctypes.data_as(P(C.c_int32)), ow.ctypes.data_as(P(C.c_int32)),
                               rp.ctypes.data_as(P(C.c_int64)), ci.ctypes.data_as(P(C.c_int32)),
                               v.ctypes.data_as(P(C.c_double))), "csdyn_ras_inspect")
    m = 4 * nloc.value
    return gc.astype(np.int64), ow.astype(bool), sp.csr_matrix((v, ci, rp), shape=(m, m))


class Solver:
    """Restarted (F)GMRES with a workspace kept across solves (csdyn_gmres_solve)."""

    def __init__(self, op: Operator, pc: RAS | None = None, restart=30, maxit=1000, flexible=False, rtol=1e-8,
                 atol=0.0, orth=0, rhs_relative=False, timing=False, device_steps=0):
        self.op, self.pc = op, pc
        self.opts = GmresOpts(restart, maxit, int(flexible), rtol, atol, orth, int(rhs_relative), int(timing),
                              int(device_steps))
        nb = C.c_size_t()
        _check(lib().csdyn_gmres_workspace_bytes(op.h, C.byref(self.opts), C.byref(nb)),
               "csdyn_gmres_workspace_bytes")
        self.ws = _workspace(nb.value, op.device)
        self.nbytes = nb.value

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, stream=None):
        """Solves in place into x (x holds x0 on entry).  Returns (x, stats dict, status)."""
        x = torch.zeros_like(b) if x is None else x
        st = GmresStats()
        rc = lib().csdyn_gmres_solve(self.op.h, self.pc.h if self.pc else None, C.byref(self.opts), _ptr(b), _ptr(x),
                                     _ptr(self.ws), self.nbytes, _stream(stream), C.byref(st))
        _check(rc, "csdyn_gmres_solve")
        stats = dict(iters=st.iters, restarts=st.restarts, inner_iters=st.inner_iters, relres_true=st.relres_true,
                     relres_est=st.relres_est, res0=st.res0, res_true=st.res_true, bnorm=st.bnorm,
                     inner2_iters=st.inner2_iters)
        if self.opts.timing:
            stats["t_ms"] = dict(zip(PHASES, list(st.t_ms)))
            stats["t_span_ms"] = st.t_span_ms
        return x, stats, rc


class Batch:
    """Lock-step batched FGMRES over shells of different sizes (csdyn_batch_*)."""

    def __init__(self, ops, pcs=None, restart=30, maxit=1000, rtol=1e-8, atol=0.0, rhs_relative=False):
        self.ops, self.pcs = list(ops), list(pcs) if pcs is not None else None
        ns = len(self.ops)
        self.opts = GmresOpts(restart, maxit, 1, rtol, atol, 0, int(rhs_relative))
        self._oh = (C.c_void_p * ns)(*[o.h for o in self.ops])
        self._ph = (C.c_void_p * ns)(*[p.h if p is not None else None for p in self.pcs]) if self.pcs else None
        nb = C.c_size_t()
        _check(lib().csdyn_batch_workspace_bytes(ns, self._oh, C.byref(self.opts), C.byref(nb)),
               "csdyn_batch_workspace_bytes")
        self.ws = _workspace(nb.value, self.ops[0].device)
        h = C.c_void_p()
        _check(lib().csdyn_batch_setup(ns, self._oh, self._ph, C.byref(self.opts), _ptr(self.ws), nb.value,
                                       C.byref(h)), "csdyn_batch_setup")
        self.h = h

    # how a lock-step Arnoldi step runs (csdyn_gmres_solve_batched's use_graph)
    EAGER, GRAPH, PHASES, PERSISTENT = 0, 1, 2, 3

    def available(self, mode):
        v = C.c_int32()
        _check(lib().csdyn_batch_modes(self.h, C.byref(v)), "csdyn_batch_modes")
        return bool(v.value >> mode & 1)

    @property
    def persistent_available(self):
        return self.available(self.PERSISTENT)

    def solve(self, bs, xs, use_graph=True, stream=None):
        """use_graph: False/0 eager, True/1 graph of per-shell branches, 2 one launch per phase for
        all shells, 3 persistent step."""
        ns = len(self.ops)
        for t in list(bs) + list(xs):
            _need(t, torch.float64, "batch vectors")
        bp = (C.c_void_p * ns)(*[_ptr(t).value for t in bs])
        xp = (C.c_void_p * ns)(*[_ptr(t).value for t in xs])
        st = (GmresStats * ns)()
        rc = lib().csdyn_gmres_solve_batched(self.h, bp, xp, int(use_graph), _stream(stream), st)
        _check(rc, "csdyn_gmres_solve_batched")
        stats = [dict(iters=s.iters, restarts=s.restarts, relres_true=s.relres_true, relres_est=s.relres_est,
                      res0=s.res0, res_true=s.res_true, bnorm=s.bnorm) for s in st]
        return stats, rc

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.csdyn_batch_destroy(h)


class Residual:
    """||b - A x|| of a candidate initial guess (csdyn_residual_norm)."""

    def __init__(self, op: Operator):
        self.op = op
        nb = C.c_size_t()
        _check(lib().csdyn_residual_workspace_bytes(op.h, C.byref(nb)), "csdyn_residual_workspace_bytes")
        self.ws = _workspace(nb.value, op.device)
        self.nbytes = nb.value

    def __call__(self, b, x, stream=None):
        out = C.c_double()
        _check(lib().csdyn_residual_norm(self.op.h, _ptr(b), _ptr(x), _ptr(self.ws), self.nbytes, _stream(stream),
                                         C.byref(out)), "csdyn_residual_norm")
        return out.value


def residual_norm_noalloc(op: Operator, b, x, stream=None):
    """||b - A x|| without a workspace (csdyn_residual_norm_noalloc; shells of at most
    6 x 32^3 cells)."""
    out = C.c_double()
    _check(lib().csdyn_residual_norm_noalloc(op.h, _ptr(b), _ptr(x), _stream(stream), C.byref(out)),
           "csdyn_residual_norm_noalloc")
    return out.value


class Profile:
    """Context manager around csdyn_profile_begin/end: per-kernel launch counts
    and summed HIP-event durations, recorded on the launch streams.  select:
    kernel names to time, every: one launch in `every` of each of them
    (csdyn_profile_select); select=None times every launch."""

    def __init__(self, max_launches=200000, select=None, every=1):
        self.max_launches = max_launches
        self.select = select
        self.every = every
        self.result = {}

    def __enter__(self):
        names = ",".join(self.select).encode() if self.select else None
        _check(lib().csdyn_profile_select(names, self.every), "csdyn_profile_select")
        _check(lib().csdyn_profile_begin(self.max_launches), "csdyn_profile_begin")
        return self

    def __exit__(self, *exc):
        buf = (ProfileEntry * 256)()
        n = C.c_int32()
        _check(lib().csdyn_profile_end(buf, 256, C.byref(n)), "csdyn_profile_end")
        self.result = {(buf[i].name.decode(), buf[i].size): dict(count=buf[i].count, ms=buf[i].total_ms,
                                                                  bytes=buf[i].bytes, flops=buf[i].flops)
                       for i in range(min(n.value, 256))}
        return False


# ------------------------------------------------------- learned initial guess
def _need(t, dtype, what):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    return t


def conv_sizes(shape):
    s = ConvShape(*shape)
    wf, wb, ws = C.c_int64(), C.c_int64(), C.c_size_t()
    _check(lib().csdyn_conv3d_sizes(C.byref(s), C.byref(wf), C.byref(wb), C.byref(ws)), "csdyn_conv3d_sizes")
    return wf.value, wb.value, ws.value


def conv_pack(shape, w: torch.Tensor, stream=None):
    """Packed BF16 forward and data-gradient weights of FP32 w [cout][27][cin]."""
    s = ConvShape(*shape)
    _need(w, torch.float32, "conv_pack weights")
    nf, nb, _ = conv_sizes(shape)
    wf = torch.empty(nf, dtype=torch.bfloat16, device=w.device)
    wb = torch.empty(nb, dtype=torch.bfloat16, device=w.device)
    _check(lib().csdyn_conv3d_pack(C.byref(s), _ptr(w), _ptr(wf), _ptr(wb), _stream(stream)), "csdyn_conv3d_pack")
    return wf, wb


def conv_fwd(shape, x, wf, bias=None, residual=None, relu=False, out32=False, stream=None):
    """shape = (batch, d, h, w, cin, cout); x BF16 [batch, d, h, w, cin8]."""
    s = ConvShape(*shape)
    _need(x, torch.bfloat16, "conv_fwd input"), _need(wf, torch.bfloat16, "conv_fwd weights")
    _need(bias, torch.float32, "conv_fwd bias"), _need(residual, torch.bfloat16, "conv_fwd residual")
    b, d, h, w_, ci, co = shape
    co8 = (co + 7) // 8 * 8
    if out32:
        y, y32 = None, torch.empty((b, d, h, w_, co), dtype=torch.float32, device=x.device)
    else:
        y, y32 = torch.empty((b, d, h, w_, co8), dtype=torch.bfloat16, device=x.device), None
    _check(lib().csdyn_conv3d_fwd(C.byref(s), _ptr(x), _ptr(wf), _ptr(bias) if bias is not None else None,
                                  _ptr(residual) if residual is not None else None, int(relu),
                                  _ptr(y) if y is not None else None, _ptr(y32) if y32 is not None else None,
                                  _stream(stream)), "csdyn_conv3d_fwd")
    return y32 if out32 else y


def conv_bwd_data(shape, dy, wb, mask=None, stream=None):
    s = ConvShape(*shape)
    _need(dy, torch.bfloat16, "conv_bwd_data dy"), _need(wb, torch.bfloat16, "conv_bwd_data weights")
    _need(mask, torch.bfloat16, "conv_bwd_data mask")
    b, d, h, w_, ci, co = shape
    dx = torch.empty((b, d, h, w_, (ci + 7) // 8 * 8), dtype=torch.bfloat16, device=dy.device)
    _check(lib().csdyn_conv3d_bwd_data(C.byref(s), _ptr(dy), _ptr(wb), _ptr(mask) if mask is not None else None,
                                       _ptr(dx), _stream(stream)), "csdyn_conv3d_bwd_data")
    return dx


def conv_bwd_weight(shape, x, dy, stream=None):
    s = ConvShape(*shape)
    _need(x, torch.bfloat16, "conv_bwd_weight x"), _need(dy, torch.bfloat16, "conv_bwd_weight dy")
    b, d, h, w_, ci, co = shape
    _, _, nws = conv_sizes(shape)
    ws = _workspace(nws, x.device)
    dw = torch.empty((co, 27, ci), dtype=torch.float32, device=x.device)
    db = torch.empty(co, dtype=torch.float32, device=x.device)
    _check(lib().csdyn_conv3d_bwd_weight(C.byref(s), _ptr(x), _ptr(dy), _ptr(dw), _ptr(db), _ptr(ws), nws,
                                         _stream(stream)), "csdyn_conv3d_bwd_weight")
    return dw, db


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for t in (p, g, m, v):
        _need(t, torch.float32, "adam_step")
    _check(lib().csdyn_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), step, lr, beta1, beta2, eps,
                                 _stream(stream)), "csdyn_adam_step")


class Net:
    """The learned-guess network on an N x N x Nr shell (csdyn_net_*)."""

    def __init__(self, n, nr, params: torch.Tensor, widths=(32, 48, 64, 128), stream=None):
        self.n, self.nr = n, nr
        self.widths = (C.c_int32 * 4)(*widths)
        cnt = C.c_int64()
        _check(lib().csdyn_net_param_count(self.widths, C.byref(cnt)), "csdyn_net_param_count")
        self.nparam = cnt.value
        if params.numel() != self.nparam or params.dtype != torch.float32:
            raise ValueError(f"expected {self.nparam} FP32 parameters")
        nb = C.c_size_t()
        _check(lib().csdyn_net_workspace_bytes(n, nr, self.widths, C.byref(nb)), "csdyn_net_workspace_bytes")
        self.ws = _workspace(nb.value, params.device)
        h = C.c_void_p()
        _check(lib().csdyn_net_setup(n, nr, self.widths, _ptr(params), _ptr(self.ws), nb.value, _stream(stream),
                                     C.byref(h)), "csdyn_net_setup")
        self.h = h

    def params(self, stream=None):
        out = torch.empty(self.nparam, dtype=torch.float32, device=self.ws.device)
        _check(lib().csdyn_net_get_params(self.h, _ptr(out), _stream(stream)), "csdyn_net_get_params")
        return out

    def predict(self, x1, x2, out=None, stream=None):
        _need(x1, torch.float64, "predict"), _need(x2, torch.float64, "predict")
        out = torch.empty_like(x1) if out is None else out
        _check(lib().csdyn_net_predict(self.h, _ptr(x1), _ptr(x2), _ptr(out), _stream(stream)), "csdyn_net_predict")
        return out

    def loss_grad(self, x2, x1, xn, stream=None):
        g = torch.empty(self.nparam, dtype=torch.float32, device=self.ws.device)
        loss = C.c_double()
        _check(lib().csdyn_net_loss_grad(self.h, _ptr(x2), _ptr(x1), _ptr(xn), _ptr(g), C.byref(loss),
                                         _stream(stream)), "csdyn_net_loss_grad")
        return loss.value, g

    def train_step(self, x2, x1, xn, lr=1e-3, want_loss=True, stream=None):
        loss = C.c_double()
        _check(lib().csdyn_net_train_step(self.h, _ptr(x2), _ptr(x1), _ptr(xn), lr,
                                          C.byref(loss) if want_loss else None, _stream(stream)),
               "csdyn_net_train_step")
        return loss.value if want_loss else None

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.csdyn_net_destroy(h)


GUESS_EXTRAPOLATE, GUESS_FALLBACK, GUESS_MINRES = 0, 1, 2


class Guess:
    """Initial guesses of a time march (csdyn_guess): extrapolation, the network with the
    residual fallback, or the minimal-residual step along the network's correction."""

    def __init__(self, op: Operator):
        self.op = op
        nb = C.c_size_t()
        _check(lib().csdyn_guess_workspace_bytes(op.h, C.byref(nb)), "csdyn_guess_workspace_bytes")
        self.ws = _workspace(nb.value, op.device)
        self.nbytes = nb.value

    def __call__(self, x1, x2, mode=GUESS_EXTRAPOLATE, net=None, b=None, out=None, stream=None):
        """Returns (guess, info dict)."""
        out = self.op.empty() if out is None else out
        inf = GuessInfo()
        _check(lib().csdyn_guess(net.h if net is not None else None, self.op.h, _ptr(b) if b is not None else None,
                                 _ptr(x1), _ptr(x2), mode, _ptr(out), _ptr(self.ws), self.nbytes, _stream(stream),
                                 C.byref(inf)), "csdyn_guess")
        return out, {k: getattr(inf, k) for k, _ in GuessInfo._fields_}


def march_rhs(op: Operator, v, f, dt, out=None, stream=None):
    """b = (v + dt f, 0) on the device (csdyn_march_rhs)."""
    out = op.empty() if out is None else out
    _check(lib().csdyn_march_rhs(op.h, _ptr(v), _ptr(f), dt, _ptr(out), _stream(stream)), "csdyn_march_rhs")
    return out


class Nonlinear:
    """f1 = -(u.grad)u + cB (B.grad)B and f3 = (B.grad)u - (u.grad)B
    (csdyn_nonlinear), with the ghost workspace kept across calls."""

    def __init__(self, vp: Operator, bp: Operator):
        self.vp, self.bp = vp, bp
        nb = C.c_size_t()
        _check(lib().csdyn_nonlinear_workspace_bytes(vp.h, C.byref(nb)), "csdyn_nonlinear_workspace_bytes")
        self.ws = _workspace(nb.value, vp.device)
        self.nbytes = nb.value

    def __call__(self, u, B, cB, f1=None, f3=None, T=None, stream=None):
        """T: the velocity-temperature state (u, Theta); then f1's scalar slot is f2."""
        f1 = self.vp.empty() if f1 is None else f1
        f3 = self.vp.empty() if f3 is None else f3
        _check(lib().csdyn_nonlinear(self.vp.h, self.bp.h, _ptr(u), _ptr(B), _ptr(T) if T is not None else None, cB,
                                     _ptr(f1), _ptr(f3), _ptr(self.ws), self.nbytes, _stream(stream)),
               "csdyn_nonlinear")
        return f1, f3


def cn_rhs(op: Operator, xhat, fn, c1, fm=None, c2=0.0, gf=None, c3=0.0, out=None, stream=None):
    """(2 xhat - A xhat + c1 fn + c2 fm + c3 gf, 0) on the device (csdyn_cn_rhs)."""
    out = op.empty() if out is None else out
    _check(lib().csdyn_cn_rhs(op.h, _ptr(xhat), _ptr(fn), _ptr(fm) if fm is not None else None,
                              _ptr(gf) if gf is not None else None, c1, c2, c3, _ptr(out), _stream(stream)),
           "csdyn_cn_rhs")
    return out


def step3_state(op: Operator, x, out=None, stream=None):
    """(x_vec - dt grad_h P, P) on the device (csdyn_step3_state)."""
    out = op.empty() if out is None else out
    _check(lib().csdyn_step3_state(op.h, _ptr(x), _ptr(out), _stream(stream)), "csdyn_step3_state")
    return out


def vector_rows(op: Operator, x, out=None, stream=None):
    """((A x)_vec, 0) on the device (csdyn_vector_rows)."""
    out = op.empty() if out is None else out
    _check(lib().csdyn_vector_rows(op.h, _ptr(x), _ptr(out), _stream(stream)), "csdyn_vector_rows")
    return out
