"""The C ABI library loads and exports every entry point the header declares
(no compute calls: runs on the CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adaptgrav.h")
LIB = os.path.join(ROOT, "paper_2010_13792_amd", "libadaptgrav.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ag_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["ag_tree_build", "ag_grav_eval", "ag_grav_timestep", "ag_grav_predict",
                 "ag_grav_backward", "ag_adaptive_select", "ag_grav_direct"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_entry_point():
    import paper_2010_13792_amd as ag
    assert sorted(ag.ENTRY_POINTS) == declared_functions()
    lib = ag.load_library()
    assert lib.ag_last_error() is not None


def test_error_codes_match_header():
    import paper_2010_13792_amd as ag
    src = open(HEADER).read()
    for name in ["AG_OK", "AG_EINVAL", "AG_ENOMEM", "AG_EHIP", "AG_ESTATE", "AG_ENONFINITE",
                 "AG_EDEVICE", "AG_FP64", "AG_FP32_PAIRS"]:
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", src)
        assert m, name
        assert getattr(ag, name) == int(m.group(1)), name
