"""The hand-written backward at sizes where the whole-table oracle is out of reach
(m = 22: anchor-QR adjoints over 24 columns; m = 26: segments of k = 13, whose reverse
walk starts from the end-state anchors, and anchor-QR adjoints padded to 32 columns).
Checked against a difference quotient of the FP64 forward along a seeded random
direction V of unit Frobenius norm, L(X) = sum_c logsumexp_S(-BIC(c, S)):
    (-L(X + 2hV) + 8 L(X + hV) - 8 L(X - hV) + L(X - 2hV)) / 12h  vs  <dL/dX, V>,
the fourth-order central quotient (truncation O(h^4)) at h = 1e-3.  The FP64 backward
is accurate to about 1e-14 in the element-wise adjoint tests, so its comparison shows
the quotient's own error; bounds 1e-6 relative for the FP64 backward and 1e-4 for the
FP32 one (the bound of the element-wise adjoint tests)."""
import numpy as np
import pytest
import torch

from datagen import config_data, linear_gaussian

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-6, "fp32": 1e-4}
H = 1e-3


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _loss(gs, X, plan):
    m = X.shape[1]
    bic = gs.score_all(X, plan=plan, precision="fp64").view(m, -1)
    return torch.logsumexp(-bic, dim=1).sum().item()


@pytest.mark.parametrize("m,n", [(22, 2000), (26, 5000)])
def test_backward_matches_finite_difference(gs, m, n):
    if m == 26:
        Xh = config_data("c3_m26_n5000")
    else:
        Xh = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=22)
    X = torch.as_tensor(Xh, device="cuda")
    plan = gs.Plan(m)
    print(f"\nbackward vs finite difference, m={m} n={n} k={plan.info['k']}", flush=True)
    rng = np.random.default_rng(7)
    V = rng.standard_normal(Xh.shape)
    V /= np.linalg.norm(V)
    Vd = torch.as_tensor(V, device="cuda")
    L = {t: _loss(gs, X + (t * H) * Vd, plan) for t in (-2, -1, 1, 2)}
    fd = (-L[2] + 8 * L[1] - 8 * L[-1] + L[-2]) / (12 * H)
    bic = gs.score_all(X, plan=plan, precision="fp64").view(m, -1)
    d64 = (-torch.softmax(-bic, dim=1)).reshape(-1).contiguous()
    del bic
    for prec in ("fp64", "fp32"):
        ds = d64 if prec == "fp64" else d64.float().contiguous()
        dX = gs.score_backward(X, ds, plan=plan, precision=prec, reuse_front=False)
        dd = float((dX * Vd).sum().item())
        rel = abs(dd - fd) / abs(fd)
        print(f"  {prec}: <dX, V> = {dd:.12e}, difference quotient {fd:.12e}, rel {rel:.3e}",
              flush=True)
        assert rel <= TOL[prec], f"{prec}: relative difference {rel:.3e}"
        del dX
    torch.cuda.synchronize()
