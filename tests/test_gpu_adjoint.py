"""GPU parity of the hand-written adjoint (gs_score_backward) against the FP64 oracle's
closed-form gradient dL/dX = 2 X A (itself pinned by finite differences in
test_oracle_grad.py).  Same dscores on both sides.

Tolerances, on max |dX_gpu - dX_oracle| / max |dX_oracle|:
  FP64 replay and undo of the walk: 1e-10;
  FP32 replay and undo: 1e-4 (the undone walk drifts by the FP32 rounding of each step;
  measured values are printed)."""
import numpy as np
import pytest
import torch

import oracle
from datagen import CONFIGS, config_data, linear_gaussian

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _check(gs, X, plan, what, precision, dscores):
    n, m = X.shape
    Xd = torch.as_tensor(X, device="cuda")
    dt = torch.float32 if precision == "fp32" else torch.float64
    ds = torch.as_tensor(dscores, dtype=dt, device="cuda")
    got = gs.score_backward(Xd, ds, plan=plan, what=what, precision=precision).cpu().numpy()
    if what == "bic":
        rss = oracle.score_all(X, oracle.OUT_RSS)
        # the FP32 side sees dscores rounded to FP32: give the oracle the same values
        gbar = np.asarray(ds.double().cpu().numpy()) * (n / rss)
    else:
        gbar = np.asarray(ds.double().cpu().numpy())
    want, _ = oracle.grad_from_gbar(X, gbar)
    err = np.abs(got - want).max() / np.abs(want).max()
    return err


PLANS = [(5, 30, 0, 0), (6, 40, 6, 3), (8, 60, 8, 5), (9, 70, 9, 3), (10, 90, 7, 4),
         (11, 100, 9, 5), (12, 120, 12, 6), (14, 500, 0, 0), (14, 500, 11, 5)]


@pytest.mark.parametrize("m,n,k,ks", PLANS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_logsumexp_bic(gs, m, n, k, ks, precision):
    X = linear_gaussian(m, n, 0.25, 0.5, 1.5, seed=100 + m + n)
    bic = oracle.score_all(X, oracle.OUT_BIC)
    _, dbic = oracle.logsumexp_loss(bic, m)
    err = _check(gs, X, gs.Plan(m, k, ks), "bic", precision, dbic)
    print(f"\nm={m} n={n} k={k} ks={ks} {precision}: max rel dX err {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_linear_rss(gs, precision):
    m, n = 10, 80
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=77)
    g = np.random.default_rng(5).standard_normal(oracle.num_families(m))
    err = _check(gs, X, gs.Plan(m, 8, 4), "rss", precision, g)
    assert err <= TOL[precision]


def test_c5_autograd_and_determinism(gs):
    """Differentiation workload: m=14, n=500, FP32; loss = sum_c logsumexp_S(-BIC)."""
    name = "c5_m14_n500"
    X = config_data(name)
    m = CONFIGS[name].m
    Xd = torch.as_tensor(X, device="cuda").requires_grad_(True)
    for precision in ("fp32", "fp64"):
        scores = gs.givscore(Xd, precision=precision)
        L = torch.logsumexp(-scores.double().view(m, -1), dim=1).sum()
        (dX,) = torch.autograd.grad(L, Xd)
        L_or, dX_or, _, _ = oracle.loss_and_grad(X)
        err = (dX.cpu().numpy() - dX_or).__abs__().max() / np.abs(dX_or).max()
        print(f"\nC5 {precision}: loss {L.item():.6f} (oracle {L_or:.6f}), max rel dX err {err:.3e}")
        assert abs(L.item() - L_or) <= 1e-3 * abs(L_or)
        assert err <= TOL[precision]
    ds = torch.as_tensor(oracle.logsumexp_loss(oracle.score_all(X, oracle.OUT_BIC), m)[1],
                         dtype=torch.float32, device="cuda")
    a = gs.score_backward(Xd.detach(), ds)
    b = gs.score_backward(Xd.detach(), ds)
    assert torch.equal(a, b)
