"""Regression coefficients of every family (gs_score_beta) on the GPU (marked gpu): the
walk's FP64 back-substitution against the oracle's per-family Householder solution
(itself pinned to numpy's least squares), whole tables, and at m = 20 through the
residual it leaves.

Tolerance: per family, max |d beta| <= 1e-9 max(1, max |beta|) (FP64 rotations and
back-substitution on data with VIFs below about 1e3: the coefficients' sensitivity is
of the order of the condition of the parents' columns times eps; measured values are
printed); rows of families without parents are exact zeros; the output is pre-filled
with NaN, so a row the kernel never writes fails."""
import numpy as np
import pytest
import torch

import oracle
from datagen import config_data, linear_gaussian
from parity import sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _beta(gs, X):
    n, m = X.shape
    out = torch.full((gs.num_families(m), m), float("nan"), dtype=torch.float64, device="cuda")
    gs.score_beta(torch.as_tensor(X, device="cuda"), out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES = [(1, 6), (2, 9), (5, 40), (8, 200), (10, 120), (12, 300), (14, 500)]


@pytest.mark.parametrize("m,n", CASES)
def test_beta_whole_table(gs, m, n):
    X = config_data("c1_m8_n200") if (m, n) == (8, 200) else (
        config_data("c5_m14_n500") if (m, n) == (14, 500) else
        linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=300 + m))
    got = _beta(gs, X)
    want = oracle.beta_all(X)
    assert np.isfinite(got).all(), "unwritten or non-finite rows"
    scale = np.maximum(1.0, np.abs(want).max(axis=1))
    err = float((np.abs(got - want).max(axis=1) / scale).max())
    print(f"\nm={m} n={n}: max beta err {err:.3e} over {got.shape[0]} families")
    assert err <= 1e-9
    for c in range(m):
        assert np.all(got[oracle.family_index(m, c, 0)] == 0.0)


def test_beta_c2_residuals(gs):
    """m = 20, n = 1000 (1.7 GB of coefficients): on 4,096 sampled families the residual
    x_c - X beta has the oracle's RSS, and the coefficients match the oracle's."""
    X = config_data("c2_m20_n1000")
    n, m = X.shape
    got = _beta(gs, X)
    assert np.isfinite(got).all()
    idx = sample_indices(m, 4096, 20)
    rss = oracle.score_indices(X, idx, oracle.OUT_RSS)
    worst = 0.0
    for t, i in enumerate(idx):
        c, _ = oracle.family_decode(m, int(i))
        r = X[:, c] - X @ got[i]
        worst = max(worst, abs(float(r @ r) - rss[t]) / rss[t])
    print(f"\nC2: max rel RSS err of the coefficients' residuals {worst:.3e}")
    assert worst <= 1e-10
