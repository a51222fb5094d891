"""GPU tests of gs_score_all_many: many datasets of one shape with several in flight
must give, dataset by dataset, the same tables (bit for bit) and statuses as
gs_score_all on each one alone; the first of them is also checked against the
oracle."""
import numpy as np
import pytest
import torch

import oracle
from datagen import linear_gaussian
from parity import assert_rss

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _datasets(m, n, count, seed):
    return [torch.as_tensor(linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=seed + i), device="cuda")
            for i in range(count)]


@pytest.mark.parametrize("what", ["bic", "rss"])
@pytest.mark.parametrize("count,in_flight", [(5, 3), (2, 3), (4, 1), (9, 8)])
def test_many_matches_single_calls(gs, what, count, in_flight):
    m, n = 10, 200
    Xs = _datasets(m, n, count, 300 + count)
    plan = gs.Plan(m, 8, 5)
    outs = gs.score_all_many(Xs, plan=plan, what=what, in_flight=in_flight)
    assert plan.many_status() == [gs.GS_OK] * count
    single = gs.Plan(m, 8, 5)
    for X, got in zip(Xs, outs):
        want = gs.score_all(X, plan=single, what=what)
        assert torch.equal(got, want)
    if what == "rss":
        assert_rss(outs[0].cpu().numpy(), oracle.score_all(Xs[0].cpu().numpy(), oracle.OUT_RSS),
                   1e-4, "many, dataset 0")
    # a second call with fewer datasets reuses the slots and streams
    outs2 = gs.score_all_many(Xs[:2], plan=plan, what=what, in_flight=in_flight)
    for a, b in zip(outs[:2], outs2):
        assert torch.equal(a, b)


def test_many_reports_each_dataset_status(gs):
    """A rank-deficient dataset (a repeated column) among good ones: only its status
    is GS_ERANK, and the call with check_status raises naming it."""
    m, n = 8, 120
    Xs = _datasets(m, n, 4, 900)
    bad = Xs[2].clone()
    bad[:, 5] = bad[:, 1]
    Xs[2] = bad
    plan = gs.Plan(m)
    gs.score_all_many(Xs, plan=plan, in_flight=3, check_status=False)
    assert plan.many_status() == [gs.GS_OK, gs.GS_OK, gs.GS_ERANK, gs.GS_OK]
    with pytest.raises(gs.GivScoreError) as e:
        gs.score_all_many(Xs, plan=plan, in_flight=2)
    assert e.value.code == gs.GS_ERANK and "dataset 2" in str(e.value)


def test_many_on_a_side_stream(gs):
    """The call forks from and joins the caller's stream: work queued after it on that
    stream sees finished tables."""
    m, n = 9, 150
    Xs = _datasets(m, n, 3, 40)
    plan = gs.Plan(m)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = gs.score_all_many(Xs, plan=plan, in_flight=3, check_status=False)
        sums = torch.stack([o.double().sum() for o in outs])
    s.synchronize()
    want = torch.stack([gs.score_all(X).double().sum() for X in Xs])
    assert torch.equal(sums.cpu(), want.cpu())


def test_many_with_strided_rows(gs):
    """Datasets that are column slices of wider arrays (row stride > m)."""
    m, n = 7, 90
    wide = [torch.as_tensor(linear_gaussian(m + 3, n, 0.3, 0.5, 1.5, seed=60 + i), device="cuda")
            for i in range(3)]
    Xs = [w[:, :m] for w in wide]
    assert Xs[0].stride(0) == m + 3
    plan = gs.Plan(m)
    outs = gs.score_all_many(Xs, plan=plan, what="rss", in_flight=2)
    for X, got in zip(Xs, outs):
        assert torch.equal(got, gs.score_all(X.contiguous(), what="rss"))
