"""FP64 CPU oracle for the all-families regression scores -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU library never imports, links or calls it.

`oracle.c` solves each family on its own by Householder QR (the brute-force
route of Sec. 1.1 of the paper); `walk.py` holds the integer reference for the
swap sequences of Sec. 3 and Sec. 6.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OUT_BIC = 0
OUT_RSS = 1


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.or_num_families.argtypes = [ctypes.c_int]
        lib.or_num_families.restype = i64
        lib.or_family_index.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        lib.or_family_index.restype = i64
        lib.or_family_decode.argtypes = [ctypes.c_int, i64, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_uint64)]
        lib.or_family_decode.restype = ctypes.c_int
        lib.or_bic.argtypes = [dbl, i64, ctypes.c_int]
        lib.or_bic.restype = dbl
        lib.or_rss.argtypes = [vp, i64, ctypes.c_int, i64, ctypes.c_int, ctypes.c_uint64]
        lib.or_rss.restype = dbl
        lib.or_score_all.argtypes = [vp, i64, ctypes.c_int, i64, vp, ctypes.c_int, ctypes.c_int]
        lib.or_score_all.restype = ctypes.c_int
        lib.or_score_indices.argtypes = [vp, i64, ctypes.c_int, i64, vp, i64, vp, ctypes.c_int,
                                         ctypes.c_int]
        lib.or_score_indices.restype = ctypes.c_int
        lib.or_score_all_gram.argtypes = [vp, i64, ctypes.c_int, i64, vp, ctypes.c_int,
                                          ctypes.c_int]
        lib.or_score_all_gram.restype = ctypes.c_int
        lib.or_beta_all.argtypes = [vp, i64, ctypes.c_int, i64, vp, ctypes.c_int]
        lib.or_beta_all.restype = ctypes.c_int
        lib.or_grad_from_gbar.argtypes = [vp, i64, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int]
        lib.or_grad_from_gbar.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _as_X(X):
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim != 2:
        raise ValueError("X must be 2-D (n, m)")
    return X


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1)


def num_families(m: int) -> int:
    return int(_lib().or_num_families(m))


def family_index(m: int, child: int, mask: int) -> int:
    return int(_lib().or_family_index(m, child, mask))


def family_decode(m: int, idx: int):
    c = ctypes.c_int()
    mk = ctypes.c_uint64()
    if _lib().or_family_decode(m, idx, ctypes.byref(c), ctypes.byref(mk)) != 0:
        raise ValueError("index out of range")
    return c.value, mk.value


def bic(rss: float, n: int, nparents: int) -> float:
    return float(_lib().or_bic(rss, n, nparents))


def rss(X, child: int, mask: int) -> float:
    X = _as_X(X)
    n, m = X.shape
    return float(_lib().or_rss(X.ctypes.data, n, m, m, child, mask))


def score_all(X, what: int = OUT_BIC, threads: int | None = None) -> np.ndarray:
    X = _as_X(X)
    n, m = X.shape
    out = np.empty(num_families(m), dtype=np.float64)
    st = _lib().or_score_all(X.ctypes.data, n, m, m, out.ctypes.data, what,
                             threads or default_threads())
    if st != 0:
        raise RuntimeError(f"oracle score_all failed ({st})")
    return out


def score_all_gram(X, what: int = OUT_BIC, threads: int | None = None) -> np.ndarray:
    """Every family by the normal equations (Gram matrix in extended precision, one
    Cholesky elimination per family): an independent second route, O(|S|^3) per
    family, for whole tables too large for the per-family Householder QR."""
    X = _as_X(X)
    n, m = X.shape
    out = np.empty(num_families(m), dtype=np.float64)
    st = _lib().or_score_all_gram(X.ctypes.data, n, m, m, out.ctypes.data, what,
                                  threads or default_threads())
    if st != 0:
        raise RuntimeError(f"oracle score_all_gram failed ({st})")
    return out


def score_indices(X, idx, what: int = OUT_BIC, threads: int | None = None) -> np.ndarray:
    X = _as_X(X)
    n, m = X.shape
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.shape[0], dtype=np.float64)
    st = _lib().or_score_indices(X.ctypes.data, n, m, m, idx.ctypes.data, idx.shape[0],
                                 out.ctypes.data, what, threads or default_threads())
    if st != 0:
        raise RuntimeError(f"oracle score_indices failed ({st})")
    return out


def beta_all(X, threads: int | None = None) -> np.ndarray:
    """Regression coefficients of every family (Sec. 1.1: back-substitution on the R of
    the family's own Householder QR), (m * 2^(m-1), m) in table order: row idx holds
    beta_v for the parents v of family idx and zeros elsewhere (the child included)."""
    X = _as_X(X)
    n, m = X.shape
    out = np.empty((num_families(m), m), dtype=np.float64)
    st = _lib().or_beta_all(X.ctypes.data, n, m, m, out.ctypes.data, threads or default_threads())
    if st != 0:
        raise RuntimeError(f"oracle beta_all failed ({st})")
    return out


def grad_from_gbar(X, gbar, threads: int | None = None):
    """dL/dX = 2 X A with A = sum gbar(c,S) w w^T (gbar = dL/dRSS in table order).
    Returns (dX (n, m), A (m, m))."""
    X = _as_X(X)
    n, m = X.shape
    gbar = np.ascontiguousarray(np.asarray(gbar, dtype=np.float64))
    if gbar.shape != (num_families(m),):
        raise ValueError("gbar must hold one value per family")
    A = np.empty((m, m), dtype=np.float64)
    dX = np.empty((n, m), dtype=np.float64)
    st = _lib().or_grad_from_gbar(X.ctypes.data, n, m, m, gbar.ctypes.data, A.ctypes.data,
                                 dX.ctypes.data, threads or default_threads())
    if st != 0:
        raise RuntimeError(f"oracle gradient failed ({st})")
    return dX, A


def logsumexp_loss(bic: np.ndarray, m: int):
    """L = sum over children of logsumexp over parent sets of -BIC, and dL/dBIC."""
    t = np.asarray(bic, dtype=np.float64).reshape(m, -1)
    z = -t
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    ssum = e.sum(axis=1, keepdims=True)
    L = float((zmax[:, 0] + np.log(ssum[:, 0])).sum())
    dbic = -(e / ssum)
    return L, dbic.reshape(-1)


def loss_and_grad(X, threads: int | None = None):
    """The differentiation workload's loss on the oracle's BIC table and its gradient
    dL/dX by the closed form.  Returns (L, dX, dL/dBIC, RSS table)."""
    X = _as_X(X)
    n, m = X.shape
    rss_t = score_all(X, OUT_RSS, threads)
    bic_t = score_all(X, OUT_BIC, threads)
    L, dbic = logsumexp_loss(bic_t, m)
    gbar = dbic * (n / rss_t)
    dX, _ = grad_from_gbar(X, gbar, threads)
    return L, dX, dbic, rss_t


def reduce_table(table: np.ndarray, m: int, top_k: int = 0):
    """Per-child reduction of a score table in table order (the consumers of Sec. 1):
    for every child c, the minimum score, every parent mask reaching it, the natural
    log of the sum of exp(-score) over all parent sets, and the top_k smallest scores
    with their parent masks (ascending; equal scores in ascending mask order).
    Plain loops over the table; returns a list of dicts, one per child."""
    t = np.asarray(table, dtype=np.float64).reshape(m, -1)
    out = []
    for c in range(m):
        row = t[c]
        masks = np.array([family_decode(m, c * row.size + i)[1] for i in range(row.size)],
                         dtype=np.int64)
        mn = row.min()
        best = [int(masks[i]) for i in range(row.size) if row[i] == mn]
        # ln sum exp(-s) = -min + ln sum exp(min - s): every term is at most 1
        lse = -mn + float(np.log(np.sum(np.exp(mn - row))))
        order = sorted(range(row.size), key=lambda i: (row[i], masks[i]))[:top_k]
        out.append({"min": float(mn), "argmin_masks": best, "logsumexp": lse,
                    "top_scores": [float(row[i]) for i in order],
                    "top_masks": [int(masks[i]) for i in order]})
    return out
