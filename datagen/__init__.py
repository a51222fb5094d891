"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This module only draws random data.  It contains none of the regression or
scoring arithmetic: it builds data matrices X (n samples x m variables) from a
random linear-Gaussian DAG, the kind of continuous Bayesian network whose local
scores the method computes (Sec. 1, Sec. 2 of the paper: continuous variables,
score of a child given a parent set as a function of its regression).

Recipe (the paper prints no data; these are stated readings):
  1. causal order pi = rng.permutation(m);
  2. for every pair a < b of positions in pi, an edge pi[a] -> pi[b] with
     probability p_edge, weight sign * U[lo, hi] with a fair random sign;
  3. x_v = sum_u w_uv x_u + N(0, 1), variables generated in causal order, FP64;
  4. each column centred (mean subtracted).
Column index = variable label, so the causal order is not visible in X.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["linear_gaussian", "bootstrap_batch", "CONFIGS", "Config", "config_data"]


def linear_gaussian(m: int, n: int, p_edge: float, lo: float, hi: float, seed) -> np.ndarray:
    """Return a centred (n, m) float64 C-contiguous data matrix."""
    if m < 1 or n < 1:
        raise ValueError("m and n must be positive")
    rng = np.random.default_rng(seed)
    order = rng.permutation(m)
    W = np.zeros((m, m), dtype=np.float64)  # W[u, v]: weight of edge u -> v
    for a in range(m):
        for b in range(a + 1, m):
            if rng.random() < p_edge:
                sign = 1.0 if rng.random() < 0.5 else -1.0
                W[order[a], order[b]] = sign * rng.uniform(lo, hi)
    noise = rng.standard_normal((n, m))
    X = np.zeros((n, m), dtype=np.float64)
    for v in order:
        X[:, v] = X @ W[:, v] + noise[:, v]
    X -= X.mean(axis=0, keepdims=True)
    return np.ascontiguousarray(X)


def bootstrap_batch(count: int = 256, m_range=(12, 18), n_range=(200, 2000),
                    p_edge: float = 0.2, lo: float = 0.5, hi: float = 1.5, root_seed: int = 256):
    """Uneven batch of bootstrap resamples: item b draws m_b in m_range (inclusive),
    n_b in n_range (inclusive), generates a dataset, resamples n_b rows with
    replacement and re-centres.  Returns a list of (n_b, m_b) float64 arrays."""
    out = []
    for child in np.random.SeedSequence(root_seed).spawn(count):
        rng = np.random.default_rng(child)
        mb = int(rng.integers(m_range[0], m_range[1] + 1))
        nb = int(rng.integers(n_range[0], n_range[1] + 1))
        X = linear_gaussian(mb, nb, p_edge, lo, hi, rng)
        rows = rng.integers(0, nb, size=nb)
        Xb = X[rows]
        Xb = Xb - Xb.mean(axis=0, keepdims=True)
        out.append(np.ascontiguousarray(Xb))
    return out


@dataclass(frozen=True)
class Config:
    name: str
    m: int
    n: int
    p_edge: float
    lo: float
    hi: float
    seed: int


# The five workloads: the small all-families case, the mid-size FP32 case, the
# headline m=26 case, and the shapes used by the batched and adjoint forms.
CONFIGS = {
    "c1_m8_n200": Config("c1_m8_n200", 8, 200, 0.3, 0.5, 1.5, 8),
    "c2_m20_n1000": Config("c2_m20_n1000", 20, 1000, 0.2, 0.5, 1.5, 20),
    "c3_m26_n5000": Config("c3_m26_n5000", 26, 5000, 0.15, 0.3, 1.0, 26),
    "c5_m14_n500": Config("c5_m14_n500", 14, 500, 0.2, 0.5, 1.5, 14),
}


def config_data(name: str) -> np.ndarray:
    c = CONFIGS[name]
    return linear_gaussian(c.m, c.n, c.p_edge, c.lo, c.hi, c.seed)
