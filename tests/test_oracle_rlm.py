"""Pins for the RLM-sort step models (CPU only): multisequence selection
against brute force, the level's part sizes, the whole recursion against the
textbook mergesort, and planted mistakes that the pins must catch."""

import bisect
import itertools

import numpy as np
import pytest

import oracle
from oracle import rlm


def brute_element(seqs, k):
    """k-th smallest (1-based) of all (key, sequence, position) triples."""
    trip = sorted((int(v), i, t) for i, s in enumerate(seqs) for t, v in enumerate(s))
    return trip[k - 1]


def brute_split(seqs, k):
    trip = sorted((int(v), i, t) for i, s in enumerate(seqs) for t, v in enumerate(s))[:k]
    return [sum(1 for _, i2, _ in trip if i2 == i) for i in range(len(seqs))]


def random_cases(count, seed, max_p=5, max_len=8, values=4):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        p = int(rng.integers(1, max_p + 1))
        seqs = [sorted(int(v) for v in rng.integers(0, values, int(rng.integers(0, max_len + 1))))
                for _ in range(p)]
        if sum(len(s) for s in seqs):
            yield seqs


def test_multi_select_matches_brute_force():
    n_checked = 0
    for seqs in random_cases(300, 1):
        N = sum(len(s) for s in seqs)
        for k in range(1, N + 1):
            for seed in (1, 7):
                assert rlm.multi_select(seqs, k, seed) == brute_element(seqs, k), (seqs, k)
                n_checked += 1
    assert n_checked > 2000


def test_multi_select_exhaustive_two_sequences():
    # every pair of sorted sequences of length <= 3 over {0, 1, 2}
    pool = [list(c) for n in range(4) for c in itertools.combinations_with_replacement(range(3), n)]
    for a in pool:
        for b in pool:
            seqs = [a, b]
            for k in range(1, len(a) + len(b) + 1):
                assert rlm.multi_select(seqs, k, 3) == brute_element(seqs, k)


def test_split_positions_match_brute_force():
    for seqs in random_cases(200, 2, values=3):
        N = sum(len(s) for s in seqs)
        for k in range(0, N + 1):
            assert rlm.rank_split(seqs, k, 5) == brute_split(seqs, k), (seqs, k)


def test_rlm_parts_have_exact_sizes_and_order():
    rng = np.random.default_rng(3)
    for trial in range(40):
        p = int(rng.integers(1, 9))
        seqs = [sorted(int(v) for v in rng.integers(0, 20, int(rng.integers(0, 30))))
                for _ in range(p)]
        N = sum(len(s) for s in seqs)
        r = int(rng.integers(1, 7))
        cuts = rlm.rlm_splits(seqs, r, 11)
        ranks = rlm.part_ranks(N, r)
        for j in range(r):
            size = sum(cuts[j + 1][i] - cuts[j][i] for i in range(p))
            assert size == ranks[j + 1] - ranks[j]
            assert all(cuts[j][i] <= cuts[j + 1][i] for i in range(p))
        # every element of part j precedes every element of part j+1
        for j in range(r - 1):
            left = [(s[t], i, t) for i, s in enumerate(seqs) for t in range(cuts[j][i], cuts[j + 1][i])]
            right = [(s[t], i, t) for i, s in enumerate(seqs)
                     for t in range(cuts[j + 1][i], cuts[j + 2][i])]
            if left and right:
                assert max(left) < min(right)


@pytest.mark.parametrize("tile,r", [(4, 2), (8, 4), (16, 3), (32, 16)])
def test_rlm_sort_equals_mergesort(tile, r):
    rng = np.random.default_rng(4 + tile + r)
    for n in [0, 1, tile - 1, tile, tile + 1, 5 * tile + 3, 40 * tile + 7]:
        x = rng.integers(0, max(2, n // 3), n).astype(np.uint64)
        want, _ = oracle.oracle_sort(oracle.KEY_U64, x)
        assert rlm.rlm_sort(x, tile, r) == [int(v) for v in want], (n, tile, r)


def test_merge_pieces_is_stable_by_sequence():
    # equal keys: the lower sequence's element comes first
    a = [(1, 0), (2, 0)]
    b = [(1, 1), (2, 1)]
    merged = rlm._merge_pieces([a, b])
    assert merged == [(1, 0), (1, 1), (2, 0), (2, 1)]


def _select_variant(seqs, k, *, after_rule="left", own="t", cmp="ge", reduce_k=True):
    """multi_select with one planted mistake."""
    p = len(seqs)
    lo = [0] * p
    hi = [len(s) for s in seqs]
    rng = np.random.default_rng(5)
    for _ in range(1000):
        sizes = [hi[i] - lo[i] for i in range(p)]
        total = sum(sizes)
        if total == 1:
            i = next(i for i in range(p) if sizes[i])
            return (int(seqs[i][lo[i]]), i, lo[i])
        u = int(rng.integers(0, total))
        q = 0
        while u >= sizes[q]:
            u -= sizes[q]
            q += 1
        t = lo[q] + u
        x = seqs[q][t]
        j = []
        for i, s in enumerate(seqs):
            if i < q:
                c = bisect.bisect_right(s, x)
            elif i > q:
                c = bisect.bisect_right(s, x) if after_rule == "right" else bisect.bisect_left(s, x)
            else:
                c = bisect.bisect_left(s, x) if own == "value" else t
            j.append(min(max(c, lo[i]), hi[i]))
        left = sum(j[i] - lo[i] for i in range(p))
        if (left >= k) if cmp == "ge" else (left > k):
            hi = j
        else:
            if reduce_k:
                k -= left
            lo = j
    return None


def test_selection_pins_catch_planted_mistakes():
    cases = list(random_cases(150, 9, values=3))
    for seqs in cases[:20]:
        N = sum(len(s) for s in seqs)
        for k in range(1, N + 1):
            assert _select_variant(seqs, k) == brute_element(seqs, k)
    for name, kw in {"equal keys of later sequences counted first": dict(after_rule="right"),
                     "pivot's own sequence searched by value": dict(own="value"),
                     "rank not reduced on the right": dict(reduce_k=False),
                     "strict comparison with the rank": dict(cmp="gt")}.items():
        caught = False
        for seqs in cases:
            N = sum(len(s) for s in seqs)
            for k in range(1, N + 1):
                if _select_variant(seqs, k, **kw) != brute_element(seqs, k):
                    caught = True
                    break
            if caught:
                break
        assert caught, name
