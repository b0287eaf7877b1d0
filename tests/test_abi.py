"""The C-ABI library loads on a machine without a GPU and exports every
function that include/csdyn.h declares (no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "csdyn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(csdyn_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("csdyn_operator_apply", "csdyn_ras_setup", "csdyn_ras_apply", "csdyn_gmres_solve",
                     "csdyn_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2009_02171_amd import csdyn
    lib = ctypes.CDLL(csdyn.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(csdyn.SIGNATURES)


def test_last_error_is_empty_string_initially():
    from paper_2009_02171_amd import csdyn
    assert isinstance(csdyn.lib().csdyn_last_error(), bytes)


def test_conv_sizes_and_network_parameter_count_host_only():
    """Host-side sizing of the network entries (no device work)."""
    import ctypes as C
    from paper_2009_02171_amd import csdyn, inputs
    lib = csdyn.lib()
    s = csdyn.ConvShape(6, 8, 8, 8, 48, 32)
    wf, wb, ws = C.c_int64(), C.c_int64(), C.c_size_t()
    assert lib.csdyn_conv3d_sizes(C.byref(s), C.byref(wf), C.byref(wb), C.byref(ws)) == 0
    kpad = (27 * 48 + 31) // 32 * 32            # forward K, padded to the MFMA K-slab
    kbpad = (27 * 32 + 31) // 32 * 32           # data-gradient K (input channels = 32)
    assert wf.value == 32 * kpad and wb.value == 48 * kbpad
    assert ws.value > 0
    bad = csdyn.ConvShape(6, 8, 8, 8, 48, 129)  # more than 128 output channels
    assert lib.csdyn_conv3d_sizes(C.byref(bad), C.byref(wf), C.byref(wb), C.byref(ws)) == csdyn.EINVAL
    widths = (C.c_int32 * 4)(32, 48, 64, 128)
    cnt = C.c_int64()
    assert lib.csdyn_net_param_count(widths, C.byref(cnt)) == 0
    assert cnt.value == len(inputs.net_params(0)) == 701988
    nb = C.c_size_t()
    assert lib.csdyn_net_workspace_bytes(16, 12, widths, C.byref(nb)) == csdyn.EINVAL  # Nr not a multiple of 8
    assert lib.csdyn_net_workspace_bytes(16, 16, widths, C.byref(nb)) == 0 and nb.value > 0


def test_autotune_candidates():
    from paper_2009_02171_amd import autotune
    assert autotune.candidate_subdomains(80, 80) == [8, 16, 20]
    assert autotune.candidate_subdomains(72, 72) == [8, 12, 24]
    assert autotune.candidate_subdomains(24, 24) == [8, 12, 24]
    assert set(autotune.TILES) == {1, 2, 3, 4, 5, 6}
