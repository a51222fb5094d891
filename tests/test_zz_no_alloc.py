"""gs_score_all_static (the allocation-free entry point) against gs_score_all, through the
C ABI, on the GPU: identical tables on consecutive calls with a smaller second input,
the device status code, a plan switch back, and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from datagen import config_data, linear_gaussian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _static(gs, plan, X, what):
    """One gs_score_all_static call through the C ABI; returns (table, status code)."""
    n, m = X.shape
    out = torch.full((gs.num_families(m),), float("nan"), dtype=torch.float32, device="cuda")
    code = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    w = {"bic": 0, "rss": 1}[what]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = gs.lib().gs_score_all_static(plan.handle, ctypes.c_void_p(X.data_ptr()), n, m, X.stride(0),
                                     ctypes.c_void_p(out.data_ptr()), w,
                                     ctypes.c_void_p(code.data_ptr()), stream)
    assert r == gs.GS_OK, gs.last_error()
    torch.cuda.synchronize()
    return out, int(code.item())


def _reference(gs, plan, X, what):
    out = torch.full((gs.num_families(X.shape[1]),), float("nan"), dtype=torch.float32,
                     device="cuda")
    gs.score_all(X, plan=plan, what=what, precision="fp32", out=out)
    torch.cuda.synchronize()
    return out


def test_static_matches_score_all_on_consecutive_calls(gs):
    big = torch.as_tensor(config_data("c2_m20_n1000"), device="cuda")
    small = torch.as_tensor(linear_gaussian(12, 300, 0.3, 0.5, 1.5, seed=12), device="cuda")
    pb, ps = gs.Plan(20), gs.Plan(12)
    for X, p in ((big, pb), (small, ps), (big, pb)):
        for what in ("bic", "rss"):
            print(f"static call m={X.shape[1]} n={X.shape[0]} {what}", flush=True)
            got, code = _static(gs, p, X, what)
            want = _reference(gs, p, X, what)
            assert code == gs.GS_OK
            assert not torch.isnan(got).any().item()
            assert torch.equal(got, want), f"m={X.shape[1]} {what}: tables differ"


def test_static_status_and_no_device_allocation(gs):
    X = linear_gaussian(9, 120, 0.3, 0.5, 1.5, seed=9)
    X[:, 5] = X[:, 2]
    Xd = torch.as_tensor(X, device="cuda")
    p = gs.Plan(9)
    _static(gs, p, Xd, "rss")  # warm: module and plan tables resident
    free0, _ = torch.cuda.mem_get_info()
    _, code = _static(gs, p, Xd, "rss")
    free1, _ = torch.cuda.mem_get_info()
    assert code == gs.GS_ERANK
    assert free1 == free0, f"device free memory changed by {free0 - free1} bytes"


def test_static_rejects_plans_beyond_the_array(gs):
    m, n = 28, 500
    X = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    out = torch.empty(gs.num_families(m), dtype=torch.float32, device="cuda")
    p = gs.Plan(m)
    r = gs.lib().gs_score_all_static(p.handle, ctypes.c_void_p(X.data_ptr()), n, m, m,
                                     ctypes.c_void_p(out.data_ptr()), 0, None, None)
    assert r == gs._abi.GS_ENOMEM and "static" in gs.last_error()
