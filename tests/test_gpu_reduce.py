"""The fused consumer gs_score_reduce on the GPU (marked gpu): per child the minimum BIC
with a parent set reaching it, ln sum_S exp(-BIC), and the top-k parent sets, folded in
the walk without writing the table.

Against the oracle's per-child reduction of its own BIC table (whole tables):
  - minimum: within the BIC tolerance of the FP32 walk;
  - the returned parent set: its oracle BIC within twice that tolerance of the oracle
    minimum (near-ties may resolve either way);
  - logsumexp: within the largest BIC tolerance of the child (the soft minimum moves by
    at most the largest change of its arguments) plus 1e-4 for the FP32 summation;
  - top-k: distinct valid masks, ascending scores, each score within tolerance of the
    oracle BIC of its mask, and the j-th within twice the tolerance of the oracle's j-th.
At the full m = 26 size, against gs_score_all's table reduced by torch: the same FP32
values, so the minimum and the top-k scores are equal bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from datagen import CONFIGS, config_data, linear_gaussian
from parity import bic_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


CASES = [("c1_m8_n200", 0, 0), ("c5_m14_n500", 0, 0), ("c5_m14_n500", 14, 5),
         (None, 10, 4), (None, 6, 3)]


def _data(name, seed):
    if name:
        return config_data(name)
    return linear_gaussian(11, 150, 0.3, 0.5, 1.5, seed=seed)


@pytest.mark.parametrize("name,k,ks", CASES)
def test_reduce_against_oracle(gs, name, k, ks):
    X = _data(name, 40 + k)
    n, m = X.shape
    plan = gs.Plan(m, k, ks)
    got = gs.score_reduce(torch.as_tensor(X, device="cuda"), plan=plan, top_k=8)
    got = {key: v.cpu().numpy() for key, v in got.items()}
    table = oracle.score_all(X, oracle.OUT_BIC)
    ref = oracle.reduce_table(table, m, top_k=8)
    tol = bic_tol(n, table, "fp32")
    worst = 0.0
    for c in range(m):
        r = ref[c]
        blk = slice(c << (m - 1), (c + 1) << (m - 1))
        tmax = float(tol[blk].max())
        t0 = float(bic_tol(n, np.array([r["min"]]), "fp32")[0])
        assert abs(got["best_score"][c] - r["min"]) <= t0
        bm = int(got["best_parents"][c]) & 0xffffffff
        assert not (bm >> c) & 1 and bm < (1 << m)
        assert table[oracle.family_index(m, c, bm)] - r["min"] <= 2 * t0
        dl = abs(got["logsumexp"][c] - r["logsumexp"])
        worst = max(worst, dl)
        assert dl <= tmax + 1e-4, (c, got["logsumexp"][c], r["logsumexp"])
        tm = [int(x) & 0xffffffff for x in got["top_parents"][c]]
        ts = got["top_score"][c]
        assert len(set(tm)) == 8 and all(not (x >> c) & 1 and x < (1 << m) for x in tm)
        assert np.all(np.diff(ts) >= 0)
        for j in range(8):
            ob = table[oracle.family_index(m, c, tm[j])]
            assert abs(ts[j] - ob) <= t0 + float(bic_tol(n, np.array([ob]), "fp32")[0])
            assert ob - r["top_scores"][j] <= 2 * float(bic_tol(n, np.array([ob]), "fp32")[0])
    print(f"\nm={m} n={n} k={plan.info['k']}: max |d logsumexp| {worst:.3e}")


def test_reduce_full_size_against_table(gs):
    """m = 26, n = 5000 with the default plan: the fused results against the FP32 table
    of gs_score_all reduced by torch."""
    X = torch.as_tensor(config_data("c3_m26_n5000"), device="cuda")
    m = X.shape[1]
    plan = gs.Plan(m)
    got = gs.score_reduce(X, plan=plan, top_k=8)
    again = gs.score_reduce(X, plan=plan, top_k=8)
    for key in got:
        assert torch.equal(got[key], again[key]), f"{key} not reproducible"
    table = gs.score_all(X, plan=plan).view(m, -1)
    half = 1 << (m - 1)
    for c in range(m):
        row = table[c]
        mn = row.min()
        assert got["best_score"][c].item() == mn.item()
        bm = int(got["best_parents"][c].item()) & 0xffffffff
        assert row[gs.family_index(m, c, bm) - c * half].item() == mn.item()
        lse = torch.logsumexp(-row.double(), dim=0).item()
        assert abs(got["logsumexp"][c].item() - lse) <= 1e-4 + 1e-9 * abs(lse)
        vals = torch.topk(row, 8, largest=False).values
        assert torch.equal(got["top_score"][c], vals)
        for j in range(8):
            tmk = int(got["top_parents"][c, j].item()) & 0xffffffff
            assert row[gs.family_index(m, c, tmk) - c * half].item() == got["top_score"][c, j].item()
    del table
    torch.cuda.empty_cache()
