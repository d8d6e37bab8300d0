"""The C-ABI library loads without a GPU and exports every entry point that
include/bsw.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bsw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsw_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("bsw_operator_apply", "bsw_step_begin", "bsw_jacobian_linearize", "bsw_jacobian_apply",
                 "bsw_precond_apply", "bsw_stage_update", "bsw_solve", "bsw_mesh_upload", "bsw_disc_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2301_11238_amd import bsw
    if not os.path.exists(bsw.LIB_PATH):
        pytest.fail("libbsw.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(bsw.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding covers the same names
    assert set(declared_symbols()) == set(bsw.SIGNATURES)


def test_request_footprint_is_host_arithmetic():
    """bsw_request_footprint needs no device: it grows with the mesh and the
    restart length, and FP32 state takes less than FP64."""
    from paper_2301_11238_amd import bsw
    a = bsw.request_footprint(1000, 2, bsw.BSW_FP64)
    assert a > 1000 * 42 * 8 * 41  # state and 41 work vectors at least
    assert bsw.request_footprint(2000, 2, bsw.BSW_FP64) > a
    assert bsw.request_footprint(1000, 2, bsw.BSW_FP32) < a
    assert bsw.request_footprint(1000, 2, bsw.BSW_FP64, gmres_m=10) < a
    assert bsw.request_footprint(1000, 3, bsw.BSW_FP64) > a
    assert bsw.request_footprint(1000, 5, bsw.BSW_FP64) == -1
