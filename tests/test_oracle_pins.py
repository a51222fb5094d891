"""Pins for the FP64 oracle against facts fixed by the mathematics (CPU only).

Each test checks the oracle's RSS / BIC against something other than itself:
an exact rational computation, a different library routine, a closed form or an
invariant, chosen so that a dropped term, a wrong index or a transposed operand
in the oracle fails at least one of them."""
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle
from datagen import linear_gaussian


def _families(m):
    for c in range(m):
        others = [v for v in range(m) if v != c]
        for r in range(len(others) + 1):
            for S in combinations(others, r):
                yield c, S


def _mask(S):
    return sum(1 << v for v in S)


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 11])
def test_family_index_bijection(m):
    N = oracle.num_families(m)
    assert N == m * 2 ** (m - 1)
    seen = np.zeros(N, dtype=np.int64)
    for c, S in _families(m):
        i = oracle.family_index(m, c, _mask(S))
        assert oracle.family_decode(m, i) == (c, _mask(S))
        seen[i] += 1
    assert (seen == 1).all()
    # within a child's block the index is the parent mask with bit c removed
    assert oracle.family_index(m, 0, 0) == 0
    if m >= 3:
        assert oracle.family_index(m, 1, 0b101) == 2 ** (m - 1) + 0b11


def _det_fraction(M):
    M = [row[:] for row in M]
    n = len(M)
    det = Fraction(1)
    for j in range(n):
        p = next((i for i in range(j, n) if M[i][j] != 0), None)
        if p is None:
            return Fraction(0)
        if p != j:
            M[j], M[p] = M[p], M[j]
            det = -det
        det *= M[j][j]
        for i in range(j + 1, n):
            f = M[i][j] / M[j][j]
            for k in range(j, n):
                M[i][k] -= f * M[j][k]
    return det


def test_rss_exact_gram_determinant_ratio():
    """RSS(c,S) = det(G[S+c]) / det(G[S]) with G = X^T X, computed in exact rationals
    on integer data (a textbook identity of least squares)."""
    rng = np.random.default_rng(11)
    n, m = 9, 5
    Xi = rng.integers(-6, 7, size=(n, m))
    X = Xi.astype(np.float64)
    G = [[Fraction(int(v)) for v in row] for row in (Xi.T @ Xi)]
    for c, S in _families(m):
        idx = list(S) + [c]
        num = _det_fraction([[G[a][b] for b in idx] for a in idx])
        den = _det_fraction([[G[a][b] for b in S] for a in S]) if S else Fraction(1)
        exact = float(num / den)
        got = oracle.rss(X, c, _mask(S))
        assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), (c, S, got, exact)


@pytest.mark.parametrize("m,n", [(4, 12), (6, 40)])
def test_rss_matches_lstsq(m, n):
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=100 + m)
    table = oracle.score_all(X, oracle.OUT_RSS, threads=2)
    for c, S in _families(m):
        y = X[:, c]
        if S:
            A = X[:, list(S)]
            beta = np.linalg.lstsq(A, y, rcond=None)[0]
            r = y - A @ beta
        else:
            r = y
        want = float(r @ r)
        got = table[oracle.family_index(m, c, _mask(S))]
        assert abs(got - want) <= 1e-11 * want


def test_rss_closed_forms_and_invariants():
    m, n = 7, 60
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=5)
    T = oracle.score_all(X, oracle.OUT_RSS, threads=2)
    Ginv = np.linalg.inv(X.T @ X)
    full = (1 << m) - 1
    for c in range(m):
        # empty parent set: the squared norm of the child
        assert T[oracle.family_index(m, c, 0)] == pytest.approx(X[:, c] @ X[:, c], rel=1e-13)
        # all other variables as parents: 1 / [(X^T X)^-1]_cc
        assert T[oracle.family_index(m, c, full & ~(1 << c))] == pytest.approx(1.0 / Ginv[c, c],
                                                                               rel=1e-10)
    # adding a parent never increases the RSS
    for c, S in _families(m):
        base = T[oracle.family_index(m, c, _mask(S))]
        for v in range(m):
            if v != c and v not in S:
                more = T[oracle.family_index(m, c, _mask(S) | (1 << v))]
                assert more <= base * (1 + 1e-12)


def test_rss_relabeling_invariance():
    """Permuting the columns of X relabels the families and leaves each RSS unchanged."""
    m, n = 6, 50
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=9)
    perm = np.array([3, 0, 5, 1, 4, 2])  # new column j holds old variable perm[j]
    Xp = X[:, perm]
    T = oracle.score_all(X, oracle.OUT_RSS, threads=2)
    Tp = oracle.score_all(Xp, oracle.OUT_RSS, threads=2)
    inv = np.argsort(perm)
    for c, S in _families(m):
        a = T[oracle.family_index(m, c, _mask(S))]
        b = Tp[oracle.family_index(m, int(inv[c]), _mask([int(inv[v]) for v in S]))]
        assert a == pytest.approx(b, rel=1e-12)


def test_rss_constructed_residual():
    """x_c = X_S beta + e with e orthogonal to span(X_S): RSS(c, S) = ||e||^2."""
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, 3))
    e = rng.standard_normal(n)
    Q, _ = np.linalg.qr(A)
    e = e - Q @ (Q.T @ e)
    y = A @ np.array([0.7, -1.3, 2.0]) + e
    X = np.column_stack([A, y, rng.standard_normal(n)])
    got = oracle.rss(X, 3, 0b0111)
    assert got == pytest.approx(float(e @ e), rel=1e-12)
    # an extra unrelated regressor can only lower it
    assert oracle.rss(X, 3, 0b10111) <= got * (1 + 1e-12)


def test_bic_is_gaussian_likelihood_penalty():
    """BIC(c,S) = -2 max log-likelihood of the Gaussian regression + (|S|+2) ln n, with
    the parameter-free constant n(1 + ln 2 pi) dropped."""
    from scipy.stats import norm
    m, n = 5, 80
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=21)
    T = oracle.score_all(X, oracle.OUT_BIC, threads=2)
    for c, S in [(0, ()), (2, (0, 4)), (4, (0, 1, 2, 3)), (1, (3,))]:
        y = X[:, c]
        if S:
            beta = np.linalg.lstsq(X[:, list(S)], y, rcond=None)[0]
            r = y - X[:, list(S)] @ beta
        else:
            r = y
        sigma = np.sqrt(r @ r / n)
        loglik = norm.logpdf(r, scale=sigma).sum()
        want = -2 * loglik + (len(S) + 2) * np.log(n) - n * (1 + np.log(2 * np.pi))
        assert T[oracle.family_index(m, c, _mask(S))] == pytest.approx(want, rel=1e-10, abs=1e-9)


def test_oracle_threads_agree():
    X = linear_gaussian(9, 100, 0.3, 0.5, 1.5, seed=1)
    a = oracle.score_all(X, oracle.OUT_RSS, threads=1)
    b = oracle.score_all(X, oracle.OUT_RSS, threads=5)
    assert np.array_equal(a, b)
    idx = np.array([5, 17, 0, 2303, 1000])
    assert np.array_equal(oracle.score_indices(X, idx, oracle.OUT_RSS, threads=3), a[idx])


# ---- the normal-equations route (or_score_all_gram): the same pins, plus agreement
# with the Householder route on whole tables

def test_gram_route_exact_determinant_ratio():
    rng = np.random.default_rng(12)
    n, m = 9, 5
    Xi = rng.integers(-6, 7, size=(n, m))
    X = Xi.astype(np.float64)
    G = [[Fraction(int(v)) for v in row] for row in (Xi.T @ Xi)]
    T = oracle.score_all_gram(X, oracle.OUT_RSS, threads=2)
    for c, S in _families(m):
        idx = list(S) + [c]
        num = _det_fraction([[G[a][b] for b in idx] for a in idx])
        den = _det_fraction([[G[a][b] for b in S] for a in S]) if S else Fraction(1)
        exact = float(num / den)
        got = T[oracle.family_index(m, c, _mask(S))]
        assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), (c, S, got, exact)


def test_gram_route_matches_lstsq_and_closed_forms():
    m, n = 6, 40
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=106)
    T = oracle.score_all_gram(X, oracle.OUT_RSS, threads=2)
    Ginv = np.linalg.inv(X.T @ X)
    full = (1 << m) - 1
    for c, S in _families(m):
        y = X[:, c]
        r = y - X[:, list(S)] @ np.linalg.lstsq(X[:, list(S)], y, rcond=None)[0] if S else y
        assert T[oracle.family_index(m, c, _mask(S))] == pytest.approx(float(r @ r), rel=1e-11)
    for c in range(m):
        assert T[oracle.family_index(m, c, 0)] == pytest.approx(X[:, c] @ X[:, c], rel=1e-13)
        assert T[oracle.family_index(m, c, full & ~(1 << c))] == pytest.approx(1 / Ginv[c, c],
                                                                               rel=1e-10)


@pytest.mark.parametrize("m,n,seed", [(8, 200, 8), (10, 11, 5), (12, 300, 3)])
def test_gram_route_agrees_with_householder(m, n, seed):
    X = linear_gaussian(m, n, 0.3, 0.5, 1.5, seed=seed)
    for what in (oracle.OUT_RSS, oracle.OUT_BIC):
        a = oracle.score_all(X, what, threads=4)
        b = oracle.score_all_gram(X, what, threads=3)
        if what == oracle.OUT_RSS:
            assert np.max(np.abs(a - b) / a) <= 1e-12
        else:
            assert np.max(np.abs(a - b)) <= 1e-9


# ---- the per-child reduction of a table (the fused consumer's reference)

def test_reduce_table_pins():
    """Minimum and argmin by brute force over the families, logsumexp against scipy,
    top-k against a full sort, on the oracle's own BIC table."""
    from scipy.special import logsumexp
    m, n = 6, 50
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=31)
    T = oracle.score_all(X, oracle.OUT_BIC, threads=2)
    red = oracle.reduce_table(T, m, top_k=5)
    for c in range(m):
        vals = {_mask(S): T[oracle.family_index(m, c, _mask(S))] for cc, S in _families(m) if cc == c}
        mn = min(vals.values())
        assert red[c]["min"] == mn
        assert sorted(red[c]["argmin_masks"]) == sorted(k for k, v in vals.items() if v == mn)
        assert red[c]["logsumexp"] == pytest.approx(logsumexp([-v for v in vals.values()]), rel=1e-14)
        srt = sorted(vals.items(), key=lambda kv: (kv[1], kv[0]))[:5]
        assert red[c]["top_masks"] == [k for k, _ in srt]
        assert red[c]["top_scores"] == [v for _, v in srt]
    # ties: every mask reaching the minimum is reported
    T2 = np.zeros(oracle.num_families(3))
    T2[[0, 3]] = -1.0
    r2 = oracle.reduce_table(T2, 3, top_k=2)
    assert r2[0]["argmin_masks"] == [0, 0b110] and r2[0]["top_masks"] == [0, 0b110]
    assert r2[1]["logsumexp"] == pytest.approx(np.log(4.0))


# ---- regression coefficients (beta_all)

@pytest.mark.parametrize("m,n,seed", [(1, 9, 1), (4, 12, 2), (6, 40, 3), (8, 120, 4)])
def test_beta_all_matches_lstsq(m, n, seed):
    """Every family's coefficients against numpy's least squares, whole tables at m <= 8;
    zeros outside the parent set; and the residual they leave is the oracle's RSS."""
    X = linear_gaussian(m, n, 0.4, 0.5, 1.5, seed=seed)
    B = oracle.beta_all(X, threads=3)
    rss = oracle.score_all(X, oracle.OUT_RSS, threads=2)
    for c, S in _families(m):
        i = oracle.family_index(m, c, _mask(S))
        want = np.zeros(m)
        if S:
            want[list(S)] = np.linalg.lstsq(X[:, list(S)], X[:, c], rcond=None)[0]
        assert np.allclose(B[i], want, rtol=1e-10, atol=1e-12 * max(1.0, np.abs(want).max()))
        r = X[:, c] - X @ B[i]
        assert float(r @ r) == pytest.approx(rss[i], rel=1e-10)
