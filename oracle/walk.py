"""Integer reference for the paper's swap sequences -- TEST INFRASTRUCTURE.

Plain Python, small m only.  Shares no code with the GPU library's planner.

Conventions: swap index i is 1-based as in the paper; GRC_i exchanges the
variables at positions i and i+1 (Sec. 1.3).  An ordering [p1..pm] is the QRD
of the data with its columns in that order; it solves the regressions
"{p1..pi} -> p_k" for 0 <= i < k <= m (Sec. 2, the [A,B,C] example).
"""
from __future__ import annotations

from itertools import combinations

__all__ = [
    "greedy_swaps", "swap_count", "walk_orderings", "models_of_ordering",
    "cumulative_model_counts", "greedy_by_choice", "runtime_T_recurrence",
    "runtime_T_closed", "seed_path", "emitted_families", "num_families",
]


def greedy_swaps(m: int) -> list[int]:
    """Upsilon(m), the shortest swap sequence of Sec. 3, built from what the section
    describes: with the last variable kept at the back, the first m - 1 variables are
    walked through their own sequence (every parent set of them is then a prefix once);
    the last variable is carried from the back to the front by m - 1 adjacent swaps
    (positions m - 1 down to 1); the first m - 1 are walked through their sequence once
    more, now one position further right, behind it (every parent set that holds it).
    The second walk's positions are shifted by one, as the text and the Sec. 5
    recurrence say.  One variable needs no swap; two need one."""
    if m < 1:
        raise ValueError("m >= 1")
    if m == 1:
        return []
    if m == 2:
        return [1]
    rest = greedy_swaps(m - 1)
    carry_to_front = list(range(m - 1, 0, -1))
    return rest + carry_to_front + [i + 1 for i in rest]


def swap_count(m: int) -> int:
    """|Upsilon(m)| = 2^m - m - 1 (Sec. 3, Sec. 5)."""
    return (1 << m) - m - 1


def walk_orderings(start: list, swaps: list[int]) -> list[list]:
    """All orderings visited: start, then one per GRC."""
    cur = list(start)
    out = [list(cur)]
    for i in swaps:
        cur[i - 1], cur[i] = cur[i], cur[i - 1]
        out.append(list(cur))
    return out


def models_of_ordering(order: list, include_empty: bool = False) -> set:
    """Regression models solved by the QRD of one ordering (Sec. 2)."""
    res = set()
    for k in range(len(order)):
        for i in range(0 if include_empty else 1, k + 1):
            res.add((order[k], frozenset(order[:i])))
    return res


def cumulative_model_counts(orderings: list[list], include_empty: bool = False) -> list[int]:
    seen = set()
    out = []
    for o in orderings:
        seen |= models_of_ordering(o, include_empty)
        out.append(len(seen))
    return out


def greedy_by_choice(m: int) -> list[int]:
    """The greedy rule of Sec. 3 run literally: at each step take the swap that adds
    the most new models, ties to the leftmost index; stop when all are covered."""
    order = list(range(m))
    seen = models_of_ordering(order)
    total = m * ((1 << (m - 1)) - 1)
    swaps = []
    while len(seen) < total:
        best, best_gain = None, 0
        for i in range(1, m):
            o = list(order)
            o[i - 1], o[i] = o[i], o[i - 1]
            gain = len(models_of_ordering(o) - seen)
            if gain > best_gain:
                best, best_gain = i, gain
        if best is None:
            raise RuntimeError("greedy stalled")
        order[best - 1], order[best] = order[best], order[best - 1]
        seen |= models_of_ordering(order)
        swaps.append(best)
    return swaps


def runtime_T_recurrence(m: int) -> int:
    """Flops of the walk by the recurrence of Sec. 5:
    T(m) = [T(m-1) + 6|Upsilon(m-1)|] + sum_{i=1}^{m-1} 6(m-i+1) + T(m-1).
    Base: T(2) = 12, one GRC at i = 1 costing 6(m-i+1) = 12."""
    if m <= 1:
        return 0
    if m == 2:
        return 12
    return (2 * runtime_T_recurrence(m - 1) + 6 * swap_count(m - 1)
            + sum(6 * (m - i + 1) for i in range(1, m)))


def runtime_T_closed(m: int) -> int:
    """Closed form of Sec. 5, read with its garbled middle term as 6 * 2^m:
    T(m) = 3 m 2^m + 6 2^m - 3 m^2 - 9 m - 6."""
    return 3 * m * (1 << m) + 6 * (1 << m) - 3 * m * m - 9 * m - 6


def seed_path(code_bits: list[int], m: int):
    """A processor's share of the walk (Sec. 6): its code fixes each of the outer
    variables k + 1 .. m (1-based labels, k = m - len(code)) either in front of the
    walked block, where it is a parent of every family the processor emits, or behind
    it, where it never is.  Variable i reads code bit m - i; 0 puts it in front (the
    polarity Alg. 2 prints).  The processor's initial ordering is the front set (later
    labels nearer the front), the walked variables 1 .. k, then the back set (in
    label order); it walks Upsilon(k) on the walked block, i.e. every swap index
    shifted by the size d of the front set.  Returns (initial ordering, swap list)."""
    k = m - len(code_bits)
    if k < 1:
        raise ValueError("code longer than m - 1")
    outer = list(range(k + 1, m + 1))
    front = [i for i in reversed(outer) if code_bits[m - i] == 0]
    back = [i for i in outer if code_bits[m - i] != 0]
    d = len(front)
    return front + list(range(1, k + 1)) + back, [d + s for s in greedy_swaps(k)]


def num_families(m: int) -> int:
    return m << (m - 1)


def emitted_families(order: list, swaps: list[int], first_prefix: int = 0,
                     last_prefix: int | None = None) -> list[tuple]:
    """Families (child, parent set) emitted along a walk with the rule
    "the initial QRD emits every prefix; after GRC_i only prefix_i is new, so emit
    prefix_i -> every later position" (the rule that reproduces the model counts
    of the Sec. 3 listing).  Prefix lengths outside [first_prefix, last_prefix]
    are not emitted (used for the segments of Sec. 6)."""
    m = len(order)
    if last_prefix is None:
        last_prefix = m - 1
    out = []
    cur = list(order)
    for i in range(first_prefix, last_prefix + 1):
        for kk in range(i, m):
            out.append((cur[kk], frozenset(cur[:i])))
    for i in swaps:
        cur[i - 1], cur[i] = cur[i], cur[i - 1]
        if first_prefix <= i <= last_prefix:
            for kk in range(i, m):
                out.append((cur[kk], frozenset(cur[:i])))
    return out


def all_families(m: int) -> set:
    res = set()
    for c in range(m):
        others = [v for v in range(m) if v != c]
        for r in range(len(others) + 1):
            for S in combinations(others, r):
                res.add((c, frozenset(S)))
    return res
