"""Pins for the gradient oracle (CPU): the closed form dL/dX = 2 X A against central
finite differences of the oracle's own loss, for the differentiation workload's loss
L = sum_c logsumexp_S(-BIC(c,S)) and for a linear loss on the RSS table."""
import numpy as np
import pytest

import oracle
from datagen import linear_gaussian


def _loss(X):
    m = X.shape[1]
    return oracle.logsumexp_loss(oracle.score_all(X, oracle.OUT_BIC, threads=4), m)[0]


@pytest.mark.parametrize("m,n,seed", [(5, 30, 1), (7, 50, 2), (8, 80, 3)])
def test_logsumexp_bic_gradient_vs_central_fd(m, n, seed):
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=seed)
    L, dX, _, _ = oracle.loss_and_grad(X, threads=4)
    assert np.isclose(L, _loss(X))
    rng = np.random.default_rng(seed)
    h = 1e-3
    for _ in range(24):
        i, j = int(rng.integers(0, n)), int(rng.integers(0, m))
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        fd = (_loss(Xp) - _loss(Xm)) / (2 * h)
        # central differences with h = 1e-3: truncation O(h^2 * third derivative)
        assert abs(fd - dX[i, j]) <= 1e-5 * max(1.0, abs(dX[i, j])), (i, j, fd, dX[i, j])


def test_linear_rss_loss_gradient():
    """L = sum g(c,S) RSS(c,S) with fixed weights g: dL/dX = 2 X A, A symmetric."""
    m, n = 6, 40
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=7)
    g = np.random.default_rng(7).standard_normal(oracle.num_families(m))
    dX, A = oracle.grad_from_gbar(X, g, threads=3)
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())

    def loss(Y):
        return float(g @ oracle.score_all(Y, oracle.OUT_RSS, threads=4))
    h = 1e-4
    for (i, j) in [(0, 0), (3, 5), (39, 2), (20, 4)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        fd = (loss(Xp) - loss(Xm)) / (2 * h)
        assert abs(fd - dX[i, j]) <= 1e-6 * max(1.0, abs(dX[i, j]))


def test_gradient_of_single_family_is_residual_outer_product():
    """One family: dRSS/dX = 2 r w^T (r = residual, w = e_c - beta)."""
    m, n = 5, 30
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=9)
    c, S = 2, [0, 4]
    g = np.zeros(oracle.num_families(m))
    g[oracle.family_index(m, c, 0b10001)] = 1.0
    dX, _ = oracle.grad_from_gbar(X, g, threads=1)
    beta = np.linalg.lstsq(X[:, S], X[:, c], rcond=None)[0]
    w = np.zeros(m)
    w[c] = 1.0
    w[S] = -beta
    r = X @ w
    assert np.allclose(dX, 2 * np.outer(r, w), atol=1e-10)


@pytest.mark.slow
def test_c5_gradient_vs_central_fd_all_columns():
    """The differentiation workload itself (m = 14, n = 500): the closed form against
    central differences, h = 1e-3 in FP64, on 70 seeded entries of X, five in each of
    the 14 columns.  The loss is evaluated on the oracle's normal-equations route
    (pinned to the Householder route in test_oracle_pins.py), which keeps the 140 loss
    evaluations cheap."""
    from datagen import config_data
    X = config_data("c5_m14_n500")
    n, m = X.shape
    L, dX, _, _ = oracle.loss_and_grad(X)

    def loss(Y):
        return oracle.logsumexp_loss(oracle.score_all_gram(Y, oracle.OUT_BIC), m)[0]

    assert abs(loss(X) - L) <= 1e-9 * abs(L)
    rng = np.random.default_rng(14)
    h = 1e-3
    worst = 0.0
    for j in range(m):
        for i in rng.choice(n, size=5, replace=False):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, j] += h
            Xm[i, j] -= h
            fd = (loss(Xp) - loss(Xm)) / (2 * h)
            err = abs(fd - dX[i, j]) / max(1.0, abs(dX[i, j]))
            worst = max(worst, err)
            assert err <= 1e-5, (i, j, fd, dX[i, j])
    print(f"\nC5 central differences, 70 entries: max error {worst:.3e}")
