"""Batched scoring (gs_score_batched) on the GPU (marked gpu).

A batch runs the same kernels as one dataset at a time, with the datasets'
pointers read from device tables: each dataset's table must equal, bit for bit,
what gs_score_all writes for it with the same plan (inner block 5, default k), and
must match the FP64 oracle within the FP32 tolerance.  The bootstrap workload is
256 resamples with m in 12..18 and n in 200..2000.
"""
import numpy as np
import pytest
import torch

import oracle
from datagen import bootstrap_batch, linear_gaussian
from parity import TOL, assert_bic, assert_rss, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _nan_outs(gs, Xs):
    return [torch.full((gs.num_families(X.shape[1]),), float("nan"), dtype=torch.float32,
                       device="cuda") for X in Xs]


def _single(gs, X, what):
    m = X.shape[1]
    plan = gs.Plan(m, 0, 5)
    return gs.score_all(torch.as_tensor(X, device="cuda"), plan=plan, what=what, precision="fp32")


def _small_batch():
    # uneven sizes, every m from 5 to 14, n from m + 1 upwards, one n above 128 x 16
    Xs = bootstrap_batch(count=20, m_range=(5, 14), n_range=(20, 700), root_seed=77)
    Xs.append(linear_gaussian(6, 7, 0.3, 0.5, 1.5, seed=5))
    Xs.append(linear_gaussian(9, 2100, 0.3, 0.5, 1.5, seed=6))
    return Xs


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("what", ["rss", "bic"])
def test_batched_equals_single(gs, what, use_graph):
    Xs = _small_batch()
    print(f"batched vs single: {len(Xs)} datasets, {what}, graph={use_graph}", flush=True)
    b = gs.Batch([(X.shape[1], X.shape[0]) for X in Xs])
    Xd = [torch.as_tensor(X, device="cuda") for X in Xs]
    outs = b.score(Xd, what=what, outs=_nan_outs(gs, Xs), use_graph=use_graph)
    torch.cuda.synchronize()
    for i, X in enumerate(Xs):
        ref = _single(gs, X, what)
        torch.cuda.synchronize()
        assert not torch.isnan(outs[i]).any().item(), f"dataset {i}: unwritten entries"
        assert torch.equal(outs[i], ref), f"dataset {i} (m={X.shape[1]}, n={X.shape[0]}) differs"
    b.close()


def test_batched_small_vs_oracle_whole_tables(gs):
    Xs = _small_batch()
    b = gs.Batch([(X.shape[1], X.shape[0]) for X in Xs])
    Xd = [torch.as_tensor(X, device="cuda") for X in Xs]
    rss = [o.cpu().numpy() for o in b.score(Xd, what="rss", outs=_nan_outs(gs, Xs))]
    bic = [o.cpu().numpy() for o in b.score(Xd, what="bic", outs=_nan_outs(gs, Xs))]
    for i, X in enumerate(Xs):
        n = X.shape[0]
        assert_rss(rss[i], oracle.score_all(X, oracle.OUT_RSS), TOL["fp32"], f"dataset {i} rss")
        assert_bic(bic[i], oracle.score_all(X, oracle.OUT_BIC), n, "fp32", f"dataset {i} bic")
    b.close()


def test_graph_replay_with_new_data(gs):
    """Replays with other data pointers and other values, then the first data again:
    every replay must give the eager (non-graph) result of its own data."""
    Xs = _small_batch()[:8]
    shapes = [(X.shape[1], X.shape[0]) for X in Xs]
    b = gs.Batch(shapes)
    eager = gs.Batch(shapes)
    A = [torch.as_tensor(X, device="cuda") for X in Xs]
    B = [torch.as_tensor(2.0 * X[::-1].copy(), device="cuda") for X in Xs]
    for rep, data in enumerate([A, B, A, B]):
        got = b.score(data, what="bic", use_graph=True)
        want = eager.score(data, what="bic", use_graph=False)
        torch.cuda.synchronize()
        for i in range(len(Xs)):
            assert torch.equal(got[i], want[i]), f"replay {rep} dataset {i}"
        # eager work on the device between replays
        torch.cuda.synchronize()
        _ = sum(float(x.sum()) for x in data)
    b.close()
    eager.close()


def test_bootstrap_256_sampled_vs_oracle(gs):
    Xs = bootstrap_batch()
    assert len(Xs) == 256
    print("bootstrap 256 datasets, m 12..18, n 200..2000", flush=True)
    b = gs.Batch([(X.shape[1], X.shape[0]) for X in Xs])
    info = b.info
    assert info["total_families"] == sum(X.shape[1] * 2 ** (X.shape[1] - 1) for X in Xs)
    Xd = [torch.as_tensor(X, device="cuda") for X in Xs]
    outs = b.score(Xd, what="bic", outs=_nan_outs(gs, Xs), use_graph=True)
    torch.cuda.synchronize()
    for i, X in enumerate(Xs):
        assert not torch.isnan(outs[i]).any().item(), f"dataset {i}: unwritten entries"
    for i in range(0, 256, 3):
        X = Xs[i]
        m, n = X.shape[1], X.shape[0]
        idx = sample_indices(m, 48, 1000 + i)
        ref = oracle.score_indices(X, idx, oracle.OUT_BIC)
        got = outs[i][torch.as_tensor(idx, device="cuda")].cpu().numpy()
        assert_bic(got, ref, n, "fp32", f"dataset {i} (m={m}, n={n})")
    for i in (0, 101, 255):
        assert torch.equal(outs[i], _single(gs, Xs[i], "bic")), f"dataset {i} batched != single"
    b.close()


def test_batched_status_per_dataset(gs):
    good = linear_gaussian(7, 100, 0.3, 0.5, 1.5, seed=1)
    nan = good.copy()
    nan[3, 2] = np.nan
    rank = linear_gaussian(8, 100, 0.3, 0.5, 1.5, seed=2)
    rank[:, 5] = rank[:, 1] - 2.0 * rank[:, 3]
    Xs = [good, nan, rank, good]
    b = gs.Batch([(X.shape[1], X.shape[0]) for X in Xs])
    outs = b.score([torch.as_tensor(X, device="cuda") for X in Xs], what="rss",
                   check_status=False)
    st = b.status()
    assert st == [gs.GS_OK, gs.GS_ENOTFINITE, gs.GS_ERANK, gs.GS_OK]
    ref = oracle.score_all(good, oracle.OUT_RSS)
    for i in (0, 3):
        assert_rss(outs[i].cpu().numpy(), ref, TOL["fp32"], f"dataset {i}")
    with pytest.raises(gs.GivScoreError):
        b.score([torch.as_tensor(X, device="cuda") for X in Xs], what="rss")
    b.close()


def test_batched_argument_errors(gs):
    Xs = [linear_gaussian(6, 50, 0.3, 0.5, 1.5, seed=3)]
    b = gs.Batch([(6, 50)])
    with pytest.raises(ValueError):
        b.score([torch.as_tensor(Xs[0][:40], device="cuda")])
    out = torch.empty(6 * 32 + 1, dtype=torch.float32, device="cuda")[1:]
    with pytest.raises(gs.GivScoreError):  # misaligned table
        b.score([torch.as_tensor(Xs[0], device="cuda")], outs=[out])
    b.close()
