"""The C ABI library builds, loads without a GPU and exports every function
that include/sdsl.h declares (no compute calls here)."""
import ctypes as C
import os
import re

import paper_2604_23979_amd as sd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "sdsl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdsl_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("sdsl_setup", "sdsl_refactor", "sdsl_update_values", "sdsl_solve", "sdsl_solve_batch",
                 "sdsl_destroy", "sdsl_get_info", "sdsl_last_error", "sdsl_default_options"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(sd.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(header_functions()) == set(sd.SIGNATURES)


def test_default_options_and_footprint_host_only():
    o = sd._binding.COptions()
    sd.lib().sdsl_default_options(C.byref(o))
    assert o.method == sd.BJ and o.pivot == sd.PIVOT_SHIFT and o.max_iter == 100000 and o.check_every == 16
    assert abs(o.inner_tol - 1e-4) < 1e-18
    import numpy as np
    rp = np.array([0, 1, 2], dtype=np.int64)
    A = sd._binding.CSR(2, 2, rp.ctypes.data_as(C.c_void_p), None, None, sd._binding.MEM_HOST)
    bp = np.array([0, 2], dtype=np.int32)
    part = sd._binding.Partition(1, bp.ctypes.data_as(C.c_void_p), 0)
    assert sd.lib().sdsl_footprint_bytes(C.byref(A), C.byref(part), C.byref(o), None) > 0


def test_setup_rejects_bad_arguments_without_touching_the_device():
    o = sd._binding.COptions()
    sd.lib().sdsl_default_options(C.byref(o))
    h = C.c_void_p()
    assert sd.lib().sdsl_setup(None, None, C.byref(o), None, None, C.byref(h)) == sd.E_INVALID
    assert b"null" in sd.lib().sdsl_last_error(None)
    assert not h.value
