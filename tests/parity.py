"""Tolerances and comparison helpers shared by the GPU parity tests.

Tolerances (relative RSS error against the FP64 oracle):
  FP64 walk: 1e-10;  FP32 walk (FP64 segment starts): 1e-4.
BIC = n ln(RSS/n) + (|S|+2) ln n moves by n ln(1 + tol) for a relative RSS error tol,
plus the rounding of the BIC value itself:
  |dBIC| <= n * tol + 8 * eps * |BIC| + n * ln2 * 2^-21 (FP32 hardware log2).
"""
import math

import numpy as np

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def assert_rss(got, want, tol, label=""):
    got = np.asarray(got, dtype=np.float64)
    assert np.isfinite(got).all(), f"{label}: unwritten or non-finite entries"
    rel = np.abs(got - want) / want
    worst = int(np.argmax(rel))
    assert rel.max() <= tol, f"{label}: max rel RSS err {rel.max():.3e} at {worst}"
    return float(rel.max())


def bic_tol(n, bic, precision):
    eps = 2.0 ** -23 if precision == "fp32" else 2.0 ** -52
    t = n * TOL[precision] + 8 * eps * np.abs(bic)
    if precision == "fp32":
        t = t + n * math.log(2) * 2.0 ** -21
    return t


def assert_bic(got, want, n, precision, label=""):
    got = np.asarray(got, dtype=np.float64)
    assert np.isfinite(got).all(), f"{label}: unwritten or non-finite entries"
    err = np.abs(got - want)
    tol = bic_tol(n, want, precision)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{label}: {bad.size} BIC entries off, first {bad[:5]} err {err[bad[:5]]}"


def sample_indices(m, count, seed):
    """Random table indices plus the first, last, middle and end-of-child-0 entries."""
    rng = np.random.default_rng(seed)
    N = m * 2 ** (m - 1)
    idx = rng.choice(N, size=min(count, N), replace=False)
    return np.unique(np.concatenate([idx, [0, N - 1, N // 2, 2 ** (m - 1) - 1]])).astype(np.int64)
