"""Pins for the integer side of the method, from the paper's own examples and counts
(CPU only).  These check the reference sequences in oracle/walk.py."""
import itertools

import pytest

from oracle import walk as W
from tests.conftest import read_golden


def test_upsilon_small():
    assert W.greedy_swaps(1) == []
    assert W.greedy_swaps(2) == [1]
    assert W.greedy_swaps(3) == [1, 2, 1, 2]
    assert W.greedy_swaps(4) == [1, 2, 1, 2, 3, 2, 1, 2, 3, 2, 3]


def test_sec2_three_variable_walk():
    rows = read_golden("paper_sec2_m3_walk.txt")
    walk_rows = [r for r in rows if r[0] != "models"]
    n_models = int([r for r in rows if r[0] == "models"][0][1])
    swaps = [int(r[1]) for r in walk_rows[1:]]
    assert swaps == W.greedy_swaps(3)
    orders = W.walk_orderings(list("ABC"), swaps)
    assert ["".join(o) for o in orders] == [r[0] for r in walk_rows]
    counts = W.cumulative_model_counts(orders)
    assert counts[-1] == n_models == 3 * (2 ** 2 - 1)


def test_sec3_four_variable_listing():
    rows = read_golden("paper_sec3_m4_listing.txt")
    orders = W.walk_orderings(list("ABCD"), W.greedy_swaps(4))
    assert ["".join(o) for o in orders] == [r[0] for r in rows]
    counts = W.cumulative_model_counts(orders)
    assert counts == [int(r[2]) for r in rows]
    # every printed count but the eleventh agrees with the distinct-model count
    printed = [int(r[1]) for r in rows]
    diff = [i for i, (a, b) in enumerate(zip(printed, counts)) if a != b]
    assert diff == [10]


@pytest.mark.parametrize("m", range(2, 15))
def test_upsilon_length(m):
    assert len(W.greedy_swaps(m)) == W.swap_count(m) == 2 ** m - m - 1


@pytest.mark.parametrize("m", range(3, 8))
def test_greedy_rule_equals_recursion(m):
    # Sec. 3: the greedy choice (most new models, leftmost on ties) follows the recursion
    assert W.greedy_by_choice(m) == W.greedy_swaps(m)


@pytest.mark.parametrize("m", range(2, 31))
def test_runtime_closed_form(m):
    assert W.runtime_T_recurrence(m) == W.runtime_T_closed(m)
    if m <= 16:
        # T(m) is the sum over the walk of the GRC cost 6(m-i+1) (Sec. 1.3)
        assert sum(6 * (m - i + 1) for i in W.greedy_swaps(m)) == W.runtime_T_closed(m)


@pytest.mark.parametrize("m", range(1, 11))
def test_emission_rule_exactly_once(m):
    fams = W.emitted_families(list(range(m)), W.greedy_swaps(m))
    assert len(fams) == len(set(fams)) == W.num_families(m)
    assert set(fams) == W.all_families(m)


def test_alg1_as_printed_double_covers():
    # Alg. 1 as printed appends [i | i in Upsilon(m-1)] without the "+1" the text has.
    def printed(m):
        if m == 2:
            return [1]
        p = printed(m - 1)
        return p + list(range(m - 1, 0, -1)) + list(p)
    fams = W.emitted_families(list(range(4)), printed(4))
    assert len(fams) == 38 and len(set(fams)) < W.num_families(4)


@pytest.mark.parametrize("m,kb", [(4, 1), (5, 2), (6, 3), (7, 2), (8, 4), (9, 3)])
def test_alg2_segments_cover_exactly_once(m, kb):
    """Sec. 6 / Alg. 2: 2^kb processors, each walks d + Upsilon(m - kb) from its own
    initial ordering; with emissions limited to prefix lengths d..d+k, the union
    covers every family exactly once, and each processor does 2^k - k - 1 swaps."""
    k = m - kb
    fams = []
    for code in itertools.product([0, 1], repeat=kb):
        order, swaps = W.seed_path(list(code), m)
        d = sum(1 for b in code if b == 0)
        assert len(swaps) == 2 ** k - k - 1
        fams += W.emitted_families(order, swaps, first_prefix=d, last_prefix=d + k)
    fams = [(c - 1, frozenset(v - 1 for v in S)) for c, S in fams]
    assert len(fams) == len(set(fams)) == W.num_families(m)


def test_alg2_printed_polarity_fails():
    # d = sum(P_id) as printed counts appended variables, not front ones.
    m, kb = 6, 2
    k = m - kb
    fams = []
    for code in itertools.product([0, 1], repeat=kb):
        order, _ = W.seed_path(list(code), m)
        d = sum(code)
        swaps = [d + s for s in W.greedy_swaps(k)]
        fams += W.emitted_families(order, swaps, first_prefix=d, last_prefix=d + k)
    assert len(set(fams)) < W.num_families(m)
