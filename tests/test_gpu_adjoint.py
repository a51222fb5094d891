"""GPU parity of the hand-written adjoint (gs_score_backward) against the FP64 oracle's
closed-form gradient dL/dX = 2 X A (itself pinned by finite differences in
test_oracle_grad.py).  Same dscores on both sides.

Tolerances, on max |dX_gpu - dX_oracle| / max |dX_oracle| (normwise):
  FP64 replay and undo of the walk: 1e-10;
  FP32 replay and undo: 1e-4 (the undone walk drifts by the FP32 rounding of each step;
  measured values are printed).
Element by element, on the entries with |dX_oracle| >= 1e-3 max |dX_oracle| (each
relative to itself): 1e-8 (FP64) and 1e-2 (FP32); an entry at 1e-3 of the largest
carries up to 1e3 times the normwise relative error."""
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
    return _errors(got, want, precision)


ELEM_TOL = {"fp64": 1e-8, "fp32": 1e-2}


def _errors(got, want, precision, scale=1.0):
    """Normwise error; asserts the element-wise bound on the significant entries."""
    want = want * scale
    err = np.abs(got - want).max() / np.abs(want).max()
    big = np.abs(want) >= 1e-3 * np.abs(want).max()
    elem = float((np.abs(got - want)[big] / np.abs(want)[big]).max())
    print(f" [element-wise on {int(big.sum())} of {big.size} entries: {elem:.3e}]", end="")
    assert elem <= ELEM_TOL[precision], f"element-wise dX error {elem:.3e}"
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
        err = _errors(dX.cpu().numpy(), dX_or, precision)
        print(f"\nC5 {precision}: loss {L.item():.6f} (oracle {L_or:.6f}), max rel dX err {err:.3e}")
        assert abs(L.item() - L_or) <= 1e-3 * abs(L_or)
        assert err <= TOL[precision]
    ds = torch.as_tensor(oracle.logsumexp_loss(oracle.score_all(X, oracle.OUT_BIC), m)[1],
                         dtype=torch.float32, device="cuda")
    a = gs.score_backward(Xd.detach(), ds)
    b = gs.score_backward(Xd.detach(), ds)
    assert torch.equal(a, b)


@pytest.mark.parametrize("e", [200, -200])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_extreme_scales(gs, e, precision):
    """Data at 2^e (e = +-200: squares far outside the FP32 range).  Every BIC moves by
    the same constant 2 n ln a under X -> a X, so the logsumexp loss's gradient at a X is
    the gradient at X divided by a; RSS is homogeneous of degree 2, so a linear RSS loss's
    gradient at a X is a times the one at X.  Both against the oracle on X."""
    m, n = 8, 60
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=88)
    Xa = np.ldexp(X, e)
    plan = gs.Plan(m, 6, 3)
    bic = oracle.score_all(X, oracle.OUT_BIC)
    _, dbic = oracle.logsumexp_loss(bic, m)
    dt = torch.float32 if precision == "fp32" else torch.float64
    ds = torch.as_tensor(dbic, dtype=dt, device="cuda")
    got = gs.score_backward(torch.as_tensor(Xa, device="cuda"), ds, plan=plan, what="bic",
                            precision=precision).cpu().numpy()
    rss = oracle.score_all(X, oracle.OUT_RSS)
    want, _ = oracle.grad_from_gbar(X, ds.double().cpu().numpy() * (n / rss))
    err = _errors(got, want, precision, scale=2.0 ** -e)
    print(f"\nBIC adjoint at 2^{e} {precision}: max rel dX err {err:.3e}")
    assert err <= TOL[precision]
    g = np.random.default_rng(9).standard_normal(oracle.num_families(m))
    ds = torch.as_tensor(g, dtype=dt, device="cuda")
    got = gs.score_backward(torch.as_tensor(Xa, device="cuda"), ds, plan=plan, what="rss",
                            precision=precision).cpu().numpy()
    want, _ = oracle.grad_from_gbar(X, ds.double().cpu().numpy())
    err = _errors(got, want, precision, scale=2.0 ** e)
    print(f"\nRSS adjoint at 2^{e} {precision}: max rel dX err {err:.3e}")
    assert err <= TOL[precision]
