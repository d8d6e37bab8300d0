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


def _fake_disc(dtype):
    """A Disc whose attributes describe a 2-D P2 discretisation of 10
    elements on cuda:0, without creating one (no GPU here)."""
    import types
    from paper_2301_11238_amd import bsw
    d = object.__new__(bsw.Disc)
    d.ctx = types.SimpleNamespace(device=0, h=None)
    d.h = None
    d.dim, d.P, d.np, d.nf, d.n_el = 2, 2, 6, 7, 10
    d.dtype = dtype
    return d


def test_binding_refuses_bad_device_arguments():
    """Host tensors, a wrong dtype, a non-contiguous view or a short buffer are
    refused with ValueError before the library sees a pointer."""
    import torch
    from paper_2301_11238_amd import bsw
    good = dict(device=0, dtype=torch.float64, min_numel=420)
    with pytest.raises(ValueError, match="cuda:0"):
        bsw.check_tensor(torch.zeros(420, dtype=torch.float64), name="W", **good)
    with pytest.raises(ValueError, match="torch tensor"):
        bsw.check_tensor([0.0] * 420, name="W", **good)
    d = _fake_disc(torch.float64)
    W = torch.zeros((7, 6, 10), dtype=torch.float64)
    b = torch.zeros((3, 6, 10), dtype=torch.float64)
    prm = bsw.make_params(_params())
    for call in (lambda: d.operator_apply(prm, 0.1, W, b, W.clone()),
                 lambda: d.step_begin(prm, 0.1, W, b),
                 lambda: d.jacobian_linearize(prm, 0.1, W),
                 lambda: d.jacobian_apply(W, W.clone()),
                 lambda: d.precond_apply(W, W.clone()),
                 lambda: d.stage_update(prm, W, W.clone()),
                 lambda: d.norm2(W),
                 lambda: d.solve(prm, bsw.Options(), W)):
        with pytest.raises(ValueError):
            call()


def _params():
    import workloads as wl
    return wl.Params()


def test_check_tensor_rules_without_a_device(monkeypatch):
    """The dtype, contiguity and length rules, with the device test stubbed
    so that CPU tensors stand in for device ones."""
    import torch
    from paper_2301_11238_amd import bsw
    monkeypatch.setattr(torch.Tensor, "is_cuda", property(lambda self: True))
    monkeypatch.setattr(torch.Tensor, "device", property(lambda self: torch.device("cuda", 0)))
    monkeypatch.setattr(bsw, "_ptr", lambda t: "ok")
    ok = torch.zeros((7, 6, 10), dtype=torch.float64)
    assert bsw.check_tensor(ok, 0, torch.float64, 420) == "ok"
    with pytest.raises(ValueError, match="dtype"):
        bsw.check_tensor(ok.float(), 0, torch.float64, 420)
    with pytest.raises(ValueError, match="contiguous"):
        bsw.check_tensor(ok.transpose(0, 2), 0, torch.float64, 420)
    with pytest.raises(ValueError, match="at least"):
        bsw.check_tensor(ok[:6], 0, torch.float64, 420)
    with pytest.raises(ValueError, match="cuda:1"):
        bsw.check_tensor(ok, 1, torch.float64, 420)
    d = _fake_disc(torch.float64)
    with pytest.raises(ValueError, match="b_old"):
        d.operator_apply(bsw.make_params(_params()), 0.1, ok, torch.zeros((2, 6, 10), dtype=torch.float64),
                         ok.clone())
