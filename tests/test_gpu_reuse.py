"""Backward calls that reuse R0 and the segment anchors of the plan's last call on the
same data (gs_plan_set_reuse): the result must be bit-identical to a backward that forms
them again, and every call that changed the plan's buffers in between (other data,
another walk precision, gs_qr_r0) must make the backward form them again."""
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


def _dscores(gs, X, plan, precision):
    """Cotangents of the loss sum_c logsumexp_S(-BIC(c, S)) from the scores of X."""
    m = X.shape[1]
    bic = gs.score_all(X, plan=plan, precision=precision)
    d = -torch.softmax(-bic.view(m, -1).double(), dim=1).reshape(-1)
    return d.to(bic.dtype).contiguous()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_reuse_is_bit_identical(gs, precision):
    X = torch.as_tensor(config_data("c5_m14_n500"), device="cuda")
    plan = gs.Plan(X.shape[1])
    print(f"\nreuse vs full backward, c5_m14_n500, {precision}", flush=True)
    ds = _dscores(gs, X, plan, precision)
    full = gs.score_backward(X, ds, plan=plan, precision=precision, reuse_front=False)
    gs.score_all(X, plan=plan, precision=precision)
    again = gs.score_backward(X, ds, plan=plan, precision=precision, reuse_front=True)
    assert torch.equal(full, again)
    # the reused R0 and anchors are the forward's: after X is changed in place (which the
    # caller must not do) the result differs from a backward that forms them again
    gs.score_all(X, plan=plan, precision=precision)
    X.mul_(1.5)
    stale = gs.score_backward(X, ds, plan=plan, precision=precision, reuse_front=True)
    fresh = gs.score_backward(X, ds, plan=plan, precision=precision, reuse_front=False)
    assert not torch.equal(stale, fresh)


def test_reuse_falls_back_when_the_buffers_changed(gs):
    m, n = 12, 300
    X1 = torch.as_tensor(linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=31), device="cuda")
    X2 = torch.as_tensor(linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=32), device="cuda")
    plan = gs.Plan(m)
    plan.set_reuse(True)
    print(f"\nreuse fallbacks, m={m} n={n}", flush=True)
    ds = _dscores(gs, X2, plan, "fp32")
    ref = gs.score_backward(X2, ds, plan=plan, reuse_front=False)
    ds64 = _dscores(gs, X2, plan, "fp64")
    ref64 = gs.score_backward(X2, ds64, plan=plan, precision="fp64", reuse_front=False)
    # other data
    gs.score_all(X1, plan=plan)
    assert torch.equal(gs.score_backward(X2, ds, plan=plan), ref)
    # the same data scored by the other walk precision
    gs.score_all(X2, plan=plan, precision="fp64")
    assert torch.equal(gs.score_backward(X2, ds, plan=plan), ref)
    gs.score_all(X2, plan=plan)
    assert torch.equal(gs.score_backward(X2, ds64, plan=plan, precision="fp64"), ref64)
    # R0 rewritten from other data after the forward on X2
    gs.score_all(X2, plan=plan)
    gs.qr_r0(X1, plan=plan)
    assert torch.equal(gs.score_backward(X2, ds, plan=plan), ref)
    # a view of the same memory with fewer rows
    gs.score_all(X2, plan=plan)
    Xs = X2[: n - 50]
    ref_s = gs.score_backward(Xs, ds, plan=plan, reuse_front=False)
    gs.score_all(X2, plan=plan)
    assert torch.equal(gs.score_backward(Xs, ds, plan=plan), ref_s)


def test_autograd_reuses_and_matches(gs):
    """GivScore's backward reuses the forward's R0 and anchors; its gradient equals the
    one of a backward that forms them again."""
    X = torch.as_tensor(config_data("c5_m14_n500"), device="cuda").requires_grad_(True)
    plan = gs.Plan(X.shape[1])
    bic = gs.givscore(X, plan=plan)
    loss = -torch.logsumexp(-bic.view(X.shape[1], -1).double(), dim=1).sum()
    loss.backward()
    bic2 = gs.score_all(X.detach(), plan=plan).requires_grad_(True)
    l2 = -torch.logsumexp(-bic2.view(X.shape[1], -1).double(), dim=1).sum()
    (d,) = torch.autograd.grad(l2, [bic2])
    ref = gs.score_backward(X.detach(), d.contiguous(), plan=plan, reuse_front=False)
    assert torch.equal(X.grad, ref)
