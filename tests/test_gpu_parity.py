"""GPU parity of the HIP walk against the FP64 CPU oracle (marked gpu).

Every comparison is element by element on the same seeded inputs: the whole table
where the oracle finishes in seconds, sampled table indices at the full sizes (the
m = 26, n = 5000 workload is run with the default plan, the launch configuration
the benchmark times).  The table is pre-filled with NaN so that an entry the
kernels never write fails the check.

Tolerances (relative RSS error against the FP64 oracle):
  FP64 walk: 1e-10;  FP32 walk (FP64 segment starts): 1e-4.
BIC = n ln(RSS/n) + (|S|+2) ln n moves by n ln(1 + tol) for a relative RSS error tol,
plus the rounding of the BIC value itself:
  |dBIC| <= n * tol + 8 * eps * |BIC| + n * ln2 * 2^-21 (FP32 hardware log2).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from datagen import CONFIGS, config_data, linear_gaussian
from parity import TOL, assert_bic, assert_rss, bic_tol, sample_indices

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def gs():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_07643_amd as g
    g.lib()
    return g


def _run(gs, X, what, precision, plan=None):
    Xd = torch.as_tensor(X, device="cuda")
    m = X.shape[1]
    dt = torch.float32 if precision == "fp32" else torch.float64
    out = torch.full((gs.num_families(m),), float("nan"), dtype=dt, device="cuda")
    gs.score_all(Xd, plan=plan, what=what, precision=precision, out=out)
    torch.cuda.synchronize()
    return out


_assert_rss, _assert_bic, _bic_tol = assert_rss, assert_bic, bic_tol


# ---------------------------------------------------------------- R0

@pytest.mark.parametrize("m,n", [(8, 200), (26, 5000), (5, 129), (30, 257)])
def test_r0(gs, m, n):
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=m * 1000 + n)
    R = gs.qr_r0(torch.as_tensor(X, device="cuda")).cpu().numpy()
    assert np.array_equal(R, np.triu(R)) and (np.diag(R) >= 0).all()
    # r_jj^2 is the RSS of variable j on the variables before it (Sec. 2)
    want = np.array([oracle.rss(X, j, (1 << j) - 1) for j in range(m)])
    _assert_rss(np.diag(R) ** 2, want, 1e-11, "diag")
    G = X.T @ X
    assert np.abs(R.T @ R - G).max() <= 1e-12 * np.abs(G).max()


# ---------------------------------------------------------------- whole tables

def test_c1_all_families(gs):
    c = CONFIGS["c1_m8_n200"]
    X = config_data("c1_m8_n200")
    ref_rss = oracle.score_all(X, oracle.OUT_RSS)
    ref_bic = oracle.score_all(X, oracle.OUT_BIC)
    for prec in ("fp64", "fp32"):
        got = _run(gs, X, "rss", prec).cpu().numpy()
        _assert_rss(got, ref_rss, TOL[prec], f"C1 rss {prec}")
        got = _run(gs, X, "bic", prec).cpu().numpy()
        _assert_bic(got, ref_bic, c.n, prec, f"C1 bic {prec}")


# (m, n, k, ks): plans that exercise one segment, many segments, middle blocks with
# every inner size, inactive half-waves, a lone segment and ragged row blocks.
WHOLE = [
    (1, 5, 0, 0), (2, 7, 0, 0), (3, 9, 0, 0), (4, 40, 4, 2), (5, 33, 5, 1), (6, 50, 0, 0),
    (7, 129, 7, 3), (8, 300, 8, 6), (9, 100, 9, 4), (10, 257, 10, 5), (11, 64, 8, 3),
    (12, 200, 12, 6), (12, 130, 9, 5), (13, 100, 13, 2), (14, 500, 11, 5), (14, 500, 0, 0),
]


@pytest.mark.parametrize("m,n,k,ks", WHOLE)
def test_whole_table(gs, m, n, k, ks):
    X = linear_gaussian(m, n, 0.25, 0.5, 1.5, seed=17 + 31 * m + n)
    plan = gs.Plan(m, k, ks)
    ref_rss = oracle.score_all(X, oracle.OUT_RSS)
    ref_bic = oracle.score_all(X, oracle.OUT_BIC)
    for prec in ("fp64", "fp32"):
        got = _run(gs, X, "rss", prec, plan).cpu().numpy()
        _assert_rss(got, ref_rss, TOL[prec], f"m={m} rss {prec}")
        got = _run(gs, X, "bic", prec, plan).cpu().numpy()
        _assert_bic(got, ref_bic, n, prec, f"m={m} bic {prec}")


# ---------------------------------------------------------------- full sizes, sampled

_sample = sample_indices


@pytest.mark.parametrize("name", ["c2_m20_n1000", "c3_m26_n5000"])
def test_full_size_sampled(gs, name):
    c = CONFIGS[name]
    X = config_data(name)
    idx = _sample(c.m, 4096, c.seed)
    ref_rss = oracle.score_indices(X, idx, oracle.OUT_RSS)
    ref_bic = oracle.score_indices(X, idx, oracle.OUT_BIC)
    it = torch.as_tensor(idx, device="cuda")
    for prec in ("fp32", "fp64"):
        out = _run(gs, X, "rss", prec)
        assert not torch.isnan(out).any().item(), f"{name} {prec}: unwritten entries"
        _assert_rss(out[it].cpu().numpy(), ref_rss, TOL[prec], f"{name} rss {prec}")
        del out
        out = _run(gs, X, "bic", prec)
        assert not torch.isnan(out).any().item(), f"{name} {prec}: unwritten entries"
        _assert_bic(out[it].cpu().numpy(), ref_bic, c.n, prec, f"{name} bic {prec}")
        del out
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_c2_whole_table(gs, prec):
    """m = 20, n = 1000: all 10,485,760 families of both walks, RSS and BIC, against the
    oracle's normal-equations route (pinned to its per-family Householder route on
    whole tables and to exact rational Gram determinant ratios)."""
    c = CONFIGS["c2_m20_n1000"]
    X = config_data("c2_m20_n1000")
    print(f"\nC2 whole table, {prec}", flush=True)
    ref_rss = oracle.score_all_gram(X, oracle.OUT_RSS)
    ref_bic = oracle.score_all_gram(X, oracle.OUT_BIC)
    got = _run(gs, X, "rss", prec).cpu().numpy()
    err = _assert_rss(got, ref_rss, TOL[prec], f"C2 rss {prec}")
    got = _run(gs, X, "bic", prec).cpu().numpy()
    _assert_bic(got, ref_bic, c.n, prec, f"C2 bic {prec}")
    print(f"C2 whole table {prec}: max rel RSS err {err:.3e}, "
          f"max |dBIC| {np.abs(got - ref_bic).max():.3e}")


@pytest.mark.parametrize("name", ["c2_m20_n1000", "c3_m26_n5000"])
def test_fp32_walk_vs_fp64_walk_whole_table(gs, name):
    """Every entry of the FP32 walk against the FP64 walk of the same plan (the FP64
    walk is itself pinned to the oracle above and in the whole-table tests)."""
    X = config_data(name)
    a = _run(gs, X, "rss", "fp32")
    b = _run(gs, X, "rss", "fp64")
    worst = 0.0
    for lo in range(0, a.numel(), 1 << 27):
        hi = min(a.numel(), lo + (1 << 27))
        rel = ((a[lo:hi].double() - b[lo:hi]).abs() / b[lo:hi]).max().item()
        worst = max(worst, rel)
    print(f"\n{name}: max rel RSS err FP32 walk vs FP64 walk = {worst:.3e}")
    assert worst <= TOL["fp32"]


@pytest.mark.parametrize("n", [48, 1000])
def test_max_m(gs, n):
    """m = 30, the largest supported size (64 GB FP32 table), sampled, with the default
    plan (segments of 2^13 - 14 Givens steps).  n = 48 is the small-sample case: the
    regressions on large parent sets have few residual degrees of freedom; its largest
    VIF (22) keeps it inside the FP32 walk's measured regime (the envelope test)."""
    m = 30
    X = linear_gaussian(m, n, 0.1, 0.3, 1.0, seed=30)
    idx = _sample(m, 1024, 30)
    ref = oracle.score_indices(X, idx, oracle.OUT_RSS)
    plan = gs.Plan(m)
    out = _run(gs, X, "rss", "fp32", plan)
    for lo in range(0, out.numel(), 1 << 30):
        assert not torch.isnan(out[lo:lo + (1 << 30)]).any().item()
    vif = plan.vif()
    err = _assert_rss(out[torch.as_tensor(idx, device="cuda")].cpu().numpy(), ref, TOL["fp32"],
                      f"m=30 n={n}")
    print(f"\nm=30 n={n}: max VIF {vif.max():.3g}, max rel RSS err {err:.3e}")
    del out
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- edge cases

def test_strided_rows(gs):
    m, n = 9, 77
    Xw = linear_gaussian(m + 4, n, 0.3, 0.5, 1.5, seed=4)
    X = Xw[:, :m]
    Xd = torch.as_tensor(Xw, device="cuda")[:, :m]
    assert Xd.stride(0) == m + 4
    ref = oracle.score_all(np.ascontiguousarray(X), oracle.OUT_RSS)
    out = gs.score_all(Xd, what="rss", precision="fp64").cpu().numpy()
    _assert_rss(out, ref, TOL["fp64"], "strided")


@pytest.mark.parametrize("scale", [1e150, 1e-150])
def test_extreme_scales_fp64(gs, scale):
    """FP64 path on data near the ends of the double range: 1e150 puts the QR steps'
    squared norms above 1e300 (the library square root and division then replace the
    refined hardware ones), 1e-150 keeps every value normal but tiny."""
    m, n = 7, 60
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=7) * scale
    print(f"extreme scale {scale:g}: m={m} n={n}", flush=True)
    for what, out_kind in (("rss", oracle.OUT_RSS), ("bic", oracle.OUT_BIC)):
        ref = oracle.score_all(X, out_kind)
        got = _run(gs, X, what, "fp64").cpu().numpy()
        if what == "rss":
            _assert_rss(got, ref, TOL["fp64"], f"scale {scale:g}")
        else:
            _assert_bic(got, ref, n, "fp64", f"scale {scale:g}")


def test_minimal_samples(gs):
    """n = m + 1: one residual degree of freedom for the full parent sets (largest VIF
    about 1e3); both walks stay inside their tolerances."""
    m = 10
    X = linear_gaussian(m, m + 1, 0.3, 0.5, 1.5, seed=5)
    ref = oracle.score_all(X, oracle.OUT_RSS)
    for prec in ("fp64", "fp32"):
        out = _run(gs, X, "rss", prec).cpu().numpy()
        err = _assert_rss(out, ref, TOL[prec], f"n=m+1 {prec}")
        print(f"\nn=m+1 {prec}: max rel RSS err {err:.3e}")


def test_nonfinite_and_rank_status(gs):
    X = linear_gaussian(6, 40, 0.3, 0.5, 1.5, seed=6)
    Xn = X.copy()
    Xn[3, 2] = np.nan
    with pytest.raises(gs.GivScoreError) as e:
        gs.score_all(torch.as_tensor(Xn, device="cuda"))
    assert e.value.code == gs.GS_ENOTFINITE
    Xr = X.copy()
    Xr[:, 4] = Xr[:, 1]
    plan = gs.Plan(6)
    out = gs.score_all(torch.as_tensor(Xr, device="cuda"), plan=plan, what="rss",
                       precision="fp64", check_status=False)
    assert plan.status() == gs.GS_ERANK
    # families that do not hold both copies of the duplicated column are unaffected
    ref = oracle.score_all(Xr, oracle.OUT_RSS)
    keep = []
    for i in range(ref.size):
        c, mask = oracle.family_decode(6, i)
        allv = mask | (1 << c)
        if not ((allv >> 1) & 1 and (allv >> 4) & 1):
            keep.append(i)
    keep = np.array(keep)
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    err = _assert_rss(got[keep], ref[keep], TOL["fp64"], "rank-deficient")
    print(f"\nrank-deficient X, families without both copies: max rel RSS err {err:.3e}")
    vif = plan.vif()
    n = X.shape[0]
    assert vif[1] * (n * 2.0 ** -52) ** 2 >= 1 and vif[4] * (n * 2.0 ** -52) ** 2 >= 1
    # a clean call afterwards reports OK again
    gs.score_all(torch.as_tensor(X, device="cuda"), plan=plan)
    assert plan.status() == gs.GS_OK


def test_deterministic_and_timing(gs):
    X = config_data("c2_m20_n1000")
    plan = gs.Plan(20)
    plan.set_timing(True)
    a = _run(gs, X, "bic", "fp32", plan)
    b = _run(gs, X, "bic", "fp32", plan)
    assert torch.equal(a, b)
    ms, cnt = plan.timing()
    assert cnt == 2 and all(x > 0 for x in ms) and ms[3] >= ms[2]


# ---------------------------------------------------------------- range and conditioning

def _expect_status(gs, X, what, precision, code):
    plan = gs.Plan(X.shape[1])
    out = _run_plan_nocheck(gs, X, what, precision, plan)
    assert plan.status() == code, f"status {plan.status()} != {code}"
    return out


def _run_plan_nocheck(gs, X, what, precision, plan):
    Xd = torch.as_tensor(X, device="cuda")
    dt = torch.float32 if precision == "fp32" else torch.float64
    out = torch.full((gs.num_families(X.shape[1]),), float("nan"), dtype=dt, device="cuda")
    gs.score_all(Xd, plan=plan, what=what, precision=precision, out=out, check_status=False)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("scale", [1e20, 1e-20, 1e150, 1e-150])
def test_extreme_scales_fp32(gs, scale):
    """FP32 walk on data whose squares leave the FP32 range: the walk scores the
    column-equilibrated data, so the BIC table matches the oracle; an RSS table cannot
    hold these values in FP32 and the call reports GS_ERANGE."""
    m, n = 7, 60
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=7) * scale
    print(f"\nFP32 walk at data scale {scale:g}: m={m} n={n}", flush=True)
    ref = oracle.score_all(X, oracle.OUT_BIC)
    got = _run(gs, X, "bic", "fp32").cpu().numpy()
    _assert_bic(got, ref, n, "fp32", f"bic scale {scale:g}")
    _expect_status(gs, X, "rss", "fp32", gs.GS_ERANGE)


@pytest.mark.parametrize("scale", [1e15, 1e-15])
def test_large_scales_fp32_rss(gs, scale):
    """RSS values inside the FP32 range but far from 1: exact after the 2^(2 e_c)
    factor."""
    m, n = 7, 60
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=7) * scale
    ref = oracle.score_all(X, oracle.OUT_RSS)
    got = _run(gs, X, "rss", "fp32").cpu().numpy()
    err = _assert_rss(got, ref, TOL["fp32"], f"rss scale {scale:g}")
    print(f"\nFP32 RSS at data scale {scale:g}: max rel err {err:.3e}")


@pytest.mark.parametrize("e", [1000, -1000, 400, -400])
def test_full_double_range(gs, e):
    """Data at 2^e, near the ends of the double range, where the oracle's own squares
    overflow or underflow: compared through the exact scaling laws of the definitions,
    RSS(a X) = a^2 RSS(X) and BIC(a X) = BIC(X) + 2 n ln a, against the oracle on X."""
    m, n = 7, 60
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=7)
    Xa = np.ldexp(X, e)
    lna = e * math.log(2.0)
    ref_bic = oracle.score_all(X, oracle.OUT_BIC) + 2 * n * lna
    ref_rss = np.ldexp(oracle.score_all(X, oracle.OUT_RSS), 2 * e)
    for prec in ("fp32", "fp64"):
        got = _run(gs, Xa, "bic", prec).cpu().numpy()
        _assert_bic(got, ref_bic, n, prec, f"bic 2^{e} {prec}")
    if abs(2 * e) < 1000:
        got = _run(gs, Xa, "rss", "fp64").cpu().numpy()
        err = _assert_rss(got, ref_rss, TOL["fp64"], f"rss 2^{e} fp64")
        print(f"\nFP64 RSS at 2^{e}: max rel err {err:.3e}")
    else:
        _expect_status(gs, Xa, "rss", "fp64", gs.GS_ERANGE)


@pytest.mark.parametrize("n", [700, 20000])
def test_row_blocks_at_different_scales(gs, n):
    """Column c of the 128-row block b of X scaled by 2^s_bc, s_bc in [-20, 20]: the
    first QR pass scales every block by its own powers of two and the next pass brings
    the blocks to one scale, exactly.  R0 of X and of X 2^t (t an integer per column)
    must then differ by exactly the factors 2^t, R0^T R0 must equal X^T X to rounding,
    and the FP64 table must match the oracle.  (n = 20000 takes three passes, so the
    rescaling pass is not the last one.)"""
    m = 6
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=n)
    rng = np.random.default_rng(n)
    nb = (n + 127) // 128
    s = rng.integers(-20, 21, size=(nb, m))
    Xs = np.ldexp(X, np.repeat(s, 128, axis=0)[:n])
    t = rng.integers(-300, 301, size=m)
    R = gs.qr_r0(torch.as_tensor(Xs, device="cuda")).cpu().numpy()
    Rt = gs.qr_r0(torch.as_tensor(np.ldexp(Xs, t[None, :]), device="cuda")).cpu().numpy()
    assert np.array_equal(np.ldexp(R, t[None, :]), Rt)
    G = Xs.T @ Xs
    d = np.sqrt(np.diag(G))
    assert (np.abs(R.T @ R - G) / np.outer(d, d)).max() <= 1e-12
    ref = oracle.score_all(Xs, oracle.OUT_RSS)
    got = _run(gs, Xs, "rss", "fp64").cpu().numpy()
    err = _assert_rss(got, ref, TOL["fp64"], f"block scales n={n} fp64")
    print(f"\nrow blocks at 2^[-20, 20], n={n}: FP64 max rel RSS err {err:.3e}")


def test_column_zero_in_some_row_blocks(gs):
    """A column that is exactly zero in the first two 128-row blocks (the first QR pass
    then has no exponent for it there) and another that is zero outside them: the
    rescaling pass must keep those rows at zero.  Both walks against the oracle."""
    m, n = 6, 700
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=71)
    X[:256, 2] = 0.0
    X[256:, 4] = 0.0
    ref = oracle.score_all(X, oracle.OUT_RSS)
    for prec in ("fp64", "fp32"):
        got = _run(gs, X, "rss", prec).cpu().numpy()
        err = _assert_rss(got, ref, TOL[prec], f"zero column blocks {prec}")
        print(f"\ncolumns zero in some row blocks, {prec}: max rel RSS err {err:.3e}")


def test_tiny_column_is_not_rank_deficient(gs):
    """One column in units 1e-13 smaller than the others: well posed (the rank test is
    scale free), both walks within their tolerances."""
    m, n = 7, 60
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=7)
    X[:, 3] *= 1e-13
    ref = oracle.score_all(X, oracle.OUT_RSS)
    for prec in ("fp64", "fp32"):
        plan = gs.Plan(m)
        got = _run_plan_nocheck(gs, X, "rss", prec, plan)
        assert plan.status() == gs.GS_OK
        err = _assert_rss(got.cpu().numpy(), ref, TOL[prec], f"tiny column {prec}")
        print(f"\ntiny column {prec}: max rel RSS err {err:.3e}")


@pytest.mark.parametrize("name", ["c1_m8_n200", "c2_m20_n1000", "c5_m14_n500"])
def test_column_vif(gs, name):
    """gs_column_vif: ||x_c||^2 / RSS(c | all other columns), checked against the
    oracle's RSS of the full parent set and against the diagonal of (X^T X)^-1."""
    X = config_data(name)
    n, m = X.shape
    plan = gs.Plan(m)
    _run_plan_nocheck(gs, X, "bic", "fp32", plan)
    vif = plan.vif()
    full = (1 << m) - 1
    want = np.array([float(X[:, c] @ X[:, c]) / oracle.rss(X, c, full & ~(1 << c))
                     for c in range(m)])
    G = X.T @ X
    want2 = np.diag(G) * np.diag(np.linalg.inv(G))
    assert np.abs(vif / want - 1).max() <= 1e-9
    assert np.abs(vif / want2 - 1).max() <= 1e-9


# FP32 walk precision envelope (relative RSS error against the FP64 oracle), fitted with
# a margin of at least 1.3 to measurements of segments of L Givens steps on data of
# largest VIF V (collinearity sweeps at m = 12 and 14, the m = 20 and m = 26 workloads):
#   E(L, V) = u (A sqrt(L) + sqrt(V) (B0 + B1 sqrt(L))),  u = 2^-24,
# with A = 6, B0 = 2.5, B1 = 0.2.  1e-4 then holds at the default segment length
# (L = 8178) for V <= 3.0e3, at L = 120 for V <= 1.2e5.
ENV_A, ENV_B0, ENV_B1 = 6.0, 2.5, 0.2


def fp32_envelope(L, V):
    u = 2.0 ** -24
    return u * (ENV_A * math.sqrt(L) + math.sqrt(V) * (ENV_B0 + ENV_B1 * math.sqrt(L)))


@pytest.mark.parametrize("delta", [1.0, 0.1, 0.01, 1e-3, 1e-4])
def test_fp32_precision_envelope(gs, delta):
    """Collinearity sweep: column 11 = column 0 + delta (a unit-scaled independent
    column), largest VIF about 1/delta^2, segments of 26 to 2^11 - 12 Givens steps.
    The measured error of the FP32 walk stays under the envelope E(L, V), with L from
    the plan and V from gs_column_vif; where E <= 1e-4 the 1e-4 tolerance holds."""
    m, n = 12, 300
    X = linear_gaussian(m, n, 0.2, 0.5, 1.5, seed=1212)
    v = X[:, 11] / np.linalg.norm(X[:, 11]) * np.linalg.norm(X[:, 0])
    X[:, 11] = X[:, 0] + delta * v
    X -= X.mean(axis=0)
    ref = oracle.score_all(X, oracle.OUT_RSS)
    for k in (5, 8, 11):
        plan = gs.Plan(m, k, 5)
        got = _run_plan_nocheck(gs, X, "rss", "fp32", plan).cpu().numpy().astype(np.float64)
        V = float(plan.vif().max())
        L = plan.info["swaps_per_segment"]
        err = float(np.max(np.abs(got - ref) / ref))
        env = fp32_envelope(L, V)
        print(f"\ndelta {delta:g} k {k} L {L} max VIF {V:.3e}: err {err:.3e} envelope {env:.3e}")
        assert err <= env
        if env <= TOL["fp32"]:
            assert err <= TOL["fp32"]


# ---------------------------------------------------------------- exactly once, on the device

@pytest.mark.parametrize("name,k,ks", [("c3_m26_n5000", 0, 0), ("c2_m20_n1000", 0, 0),
                                       ("c2_m20_n1000", 13, 5), ("c2_m20_n1000", 9, 3),
                                       ("c5_m14_n500", 14, 6), ("c1_m8_n200", 4, 2)])
def test_device_writes_exactly_once(gs, name, k, ks):
    """The walk's own store path with each write turned into an atomic +1 (gs_count_writes):
    every table entry must be written exactly once -- the split of Sec. 6 covers every
    family once -- at the default m = 26 plan the benchmark times, and at plans with
    other segment and inner-block sizes (lane-owned stores for inner blocks other than 5)."""
    X = config_data(name)
    m = X.shape[1]
    plan = gs.Plan(m, k, ks)
    print(f"\n{name} k={plan.info['k']} ks={plan.info['ks']}", flush=True)
    cnt = gs.count_writes(torch.as_tensor(X, device="cuda"), plan=plan)
    ones = int((cnt == 1).sum().item())
    assert ones == cnt.numel(), (f"{cnt.numel() - ones} entries not written exactly once "
                                 f"(min {cnt.min().item()}, max {cnt.max().item()})")
    del cnt
    torch.cuda.empty_cache()


def test_workspace_cap(gs, monkeypatch):
    """GS_WORKSPACE_LIMIT one byte below the plan's workspace gives GS_ENOMEM on a fresh
    plan; at the limit the call succeeds and matches the oracle."""
    X = config_data("c1_m8_n200")
    n, m = X.shape
    Xd = torch.as_tensor(X, device="cuda")
    plan = gs.Plan(m)
    need = plan.workspace_bytes(n)
    monkeypatch.setenv("GS_WORKSPACE_LIMIT", str(need - 1))
    with pytest.raises(gs.GivScoreError) as e:
        gs.score_all(Xd, plan=plan, what="rss", precision="fp64")
    assert e.value.code == gs._abi.GS_ENOMEM
    monkeypatch.setenv("GS_WORKSPACE_LIMIT", str(need))
    got = gs.score_all(Xd, plan=plan, what="rss", precision="fp64").cpu().numpy()
    _assert_rss(got, oracle.score_all(X, oracle.OUT_RSS), TOL["fp64"], "capped workspace")


@pytest.mark.parametrize("delta", [1.0, 1e-2, 3e-4, 1e-4, 1e-5])
def test_fp64_walk_across_conditioning(gs, delta):
    """The FP64 walk keeps 1e-10 from well-conditioned data to a largest VIF of about
    1e11 (delta = 1e-5; the walks take their guarded steps above 1e8), with
    R0^T R0 = X^T X to rounding throughout."""
    m, n = 12, 300
    X = linear_gaussian(m, n, 0.2, 0.5, 1.5, seed=1212)
    v = X[:, 11] / np.linalg.norm(X[:, 11]) * np.linalg.norm(X[:, 0])
    X[:, 11] = X[:, 0] + delta * v
    X -= X.mean(axis=0)
    plan = gs.Plan(m)
    got = _run_plan_nocheck(gs, X, "rss", "fp64", plan).cpu().numpy()
    V = float(plan.vif().max())
    err = _assert_rss(got, oracle.score_all(X, oracle.OUT_RSS), TOL["fp64"], f"delta {delta:g}")
    R = gs.qr_r0(torch.as_tensor(X, device="cuda"), plan=plan).cpu().numpy()
    G = X.T @ X
    gerr = np.abs(R.T @ R - G).max() / np.abs(G).max()
    print(f"\ndelta {delta:g}: max VIF {V:.3e}, FP64 walk max rel RSS err {err:.3e}, "
          f"|R0^T R0 - X^T X| / |X^T X| {gerr:.2e}")
    assert gerr <= 1e-14
