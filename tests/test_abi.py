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
