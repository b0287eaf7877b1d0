"""The entry point without a workspace (csdyn_residual_norm_noalloc): its
temporaries live in a static device array of the library.  Checked through the
C-ABI against csdyn_residual_norm on two calls in a row, the second on a
smaller shell, and for its size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2009_02171_amd import inputs

pytestmark = pytest.mark.gpu


def _case(n, nr, kind, seed):
    import torch
    from paper_2009_02171_amd import csdyn
    op = csdyn.Operator(n, nr, kind=kind)
    b = torch.from_numpy(inputs.rhs(n, nr, seed=seed)).cuda()
    x = torch.from_numpy(0.9 * inputs.rhs(n, nr, seed=seed + 1)).cuda()
    return op, b, x


def test_noalloc_matches_workspace_entry_point():
    import torch
    from paper_2009_02171_amd import csdyn
    L = csdyn.lib()
    for n, nr, kind, seed in ((32, 32, 0, 3), (16, 8, 1, 5)):   # the maximum size, then a smaller shell
        print(f"[noalloc] n={n} nr={nr} kind={kind}", flush=True)
        op, b, x = _case(n, nr, kind, seed)
        ref = csdyn.Residual(op)(b, x)
        out = C.c_double(-1.0)
        s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = L.csdyn_residual_norm_noalloc(op.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), s,
                                           C.byref(out))
        assert rc == 0, L.csdyn_last_error()
        print(f"[noalloc] norm {out.value!r} workspace entry point {ref!r}", flush=True)
        assert out.value > 0 and abs(out.value - ref) <= 1e-14 * ref


def test_noalloc_rejects_sizes_beyond_its_array():
    from paper_2009_02171_amd import csdyn
    op, b, x = _case(40, 8, 0, 7)      # 76,800 cells: fits
    assert np.isclose(csdyn.residual_norm_noalloc(op, b, x), csdyn.Residual(op)(b, x), rtol=1e-14, atol=0)
    op, b, x = _case(40, 24, 0, 7)     # 230,400 cells > 196,608
    with pytest.raises(csdyn.CsdynError):
        csdyn.residual_norm_noalloc(op, b, x)
