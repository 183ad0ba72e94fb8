"""The C-ABI library loads and exports every function include/smcgw.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smcgw.h")
LIB = os.path.join(ROOT, "paper_2601_02336_amd", "lib", "libsmcgw.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smcgw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("smcgw_loglike_grad", "smcgw_nuts_step", "smcgw_smc_reweight_resample", "smcgw_mass_matrix",
                     "smcgw_create", "smcgw_destroy", "smcgw_add_event"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    lib = ctypes.CDLL(LIB)
    lib.smcgw_status_string.restype = ctypes.c_char_p
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.smcgw_status_string(code).decode() != "unknown status"
    assert lib.smcgw_status_string(99).decode() == "unknown status"


def test_invalid_arguments_rejected_without_gpu():
    """Argument checks run before any HIP call."""
    lib = ctypes.CDLL(LIB)
    assert lib.smcgw_create(None, 0, None) == -1
    assert lib.smcgw_loglike_grad(None, 1, None, None, None, None, 1) == -1
    assert lib.smcgw_mass_matrix(None, 2, 2, None, ctypes.c_double(0.0), None, None, None) == -1
    assert lib.smcgw_autotune_nuts(None, 1, 1, None, None, None, None, None, 1, 1, None, None) == -1
    assert lib.smcgw_nuts_step(None, 1, 1, None, None, None, None, None, None, None, 1, None, None, None, None) == -1
    assert lib.smcgw_set_option(None, 0, ctypes.c_int64(4)) == -1
    assert lib.smcgw_local_metric(None, 1, 1, None, ctypes.c_double(1.0), None, None, None, None, None) == -1
    assert lib.smcgw_smc_reweight_resample_async(None, 1, 1, ctypes.c_double(0.0), ctypes.c_double(0.5),
                                                 ctypes.c_uint64(0), ctypes.c_uint64(0), None, None, None, None,
                                                 None, None) == -1
    assert lib.smcgw_recycle(None, 1, 1, None, None, None, ctypes.c_uint64(0), None, None, None, None) == -1
    assert lib.smcgw_ps_reweight_resample(None, 1, 1, 1, None, None, None, None, None, ctypes.c_double(0.5),
                                          ctypes.c_uint64(0), ctypes.c_uint64(0), None, None, None, None, None,
                                          None) == -1
