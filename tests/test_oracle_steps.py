"""Pins for the step models of the oracle (CPU only)."""

import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import rng as orng
from oracle import steps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, *outs = [int(x) for x in line.split()]
            assert orng.splitmix64_outputs(seed, len(outs)) == outs


def test_sample_positions_range_and_determinism():
    p1 = orng.sample_positions(9, 1, 3, 12345, 1000, 4096)
    p2 = orng.sample_positions(9, 1, 3, 12345, 1000, 4096)
    assert p1 == p2 and min(p1) >= 0 and max(p1) < 1000
    # roughly uniform: every decile gets 8..12 % of the draws
    counts = np.bincount(np.asarray(p1) // 100, minlength=10)
    assert counts.min() > 0.08 * 4096 and counts.max() < 0.12 * 4096
    assert orng.sample_positions(9, 2, 3, 12345, 1000, 16) != p1[:16]


def test_all_pairs_rank_against_brute_force_and_numpy():
    rng = np.random.default_rng(11)
    for n in range(0, 7):
        for seq in itertools.product([2, 0, 1], repeat=n):
            r = steps.all_pairs_rank(seq)
            bf = oracle.brute_force_perm(oracle.KEY_U64, np.array(seq, dtype=np.uint64)) if n else []
            # rank is the inverse of the sorting permutation
            inv = np.empty(n, dtype=np.int64)
            inv[np.asarray(bf, dtype=np.int64)] = np.arange(n)
            assert np.array_equal(r, inv)
    for n in [1, 64, 300]:
        x = rng.integers(0, 30, size=n).astype(np.uint64)
        r = steps.all_pairs_rank(x)
        inv = np.empty(n, dtype=np.int64)
        inv[np.argsort(x, kind="stable")] = np.arange(n)
        assert np.array_equal(r, inv)
        assert np.array_equal(np.sort(r), np.arange(n))


def test_classify_matches_searchsorted_and_eq_rule():
    rng = np.random.default_rng(12)
    s = np.sort(rng.integers(0, 100, size=15).astype(np.uint64))
    x = rng.integers(0, 101, size=2000).astype(np.uint64)
    ids = steps.classify(x, s, False)
    assert np.array_equal(ids, np.searchsorted(s, x, side="left"))
    eq = steps.classify(x, s, True)
    b = eq // 2
    assert np.array_equal(b, ids)
    is_eq = (eq % 2) == 1
    # equality bucket exactly when the key equals the splitter just above it
    expect = np.array([bi < s.size and xi == s[bi] for xi, bi in zip(x, b)])
    assert np.array_equal(is_eq, expect)
    # ids are monotone in the key
    o = np.argsort(x, kind="stable")
    assert np.all(np.diff(eq[o]) >= 0)
    assert eq.max() <= 2 * s.size


def test_select_splitters_equal_buckets():
    rng = np.random.default_rng(13)
    a, m = 4, 16
    samp = np.sort(rng.choice(10**9, size=a * m, replace=False).astype(np.uint64))
    spl = steps.select_splitters(samp, a, m)
    assert spl.size == m - 1
    ids = steps.classify(samp, spl, False)
    assert np.array_equal(np.bincount(ids, minlength=m), np.full(m, a))


def test_histogram_and_scan():
    rng = np.random.default_rng(14)
    ids = rng.integers(0, 37, size=5000)
    assert np.array_equal(steps.histogram(ids, 37), np.bincount(ids, minlength=37))
    v = rng.integers(0, 100, size=50)
    assert np.array_equal(steps.exclusive_scan(v), np.concatenate([[0], np.cumsum(v)[:-1]]))


def test_pack_optimal_against_exhaustive_enumeration():
    rng = np.random.default_rng(15)
    for trial in range(300):
        nb = int(rng.integers(1, 11))
        r = int(rng.integers(1, 6))
        w = [int(v) for v in rng.integers(0, 20, size=nb)]
        L, starts = steps.pack(w, r)
        assert L == steps.pack_bruteforce(w, r), (w, r)
        assert starts is not None and len(starts) <= r
        W = sum(w)
        assert L >= max(max(w), math.ceil(W / r))
        if L > 0:
            g = steps.greedy_groups(w, L - 1)
            assert g is None or len(g) > r
        ends = starts[1:] + [nb]
        assert max(sum(w[a:b]) for a, b in zip(starts, ends)) <= L


def test_pack_greedy_is_maximal():
    w = [3, 1, 4, 1, 5, 9, 2, 6, 5, 3]
    L, starts = steps.pack(w, 3)
    assert L == steps.pack_bruteforce(w, 3) == 14
    assert starts == [0, 5, 7]


def test_children_properties():
    rng = np.random.default_rng(16)
    for trial in range(200):
        m = int(rng.choice([2, 4, 8, 16]))
        r = int(rng.integers(1, 5))
        eq_on = bool(rng.integers(0, 2))
        nb = steps.num_ids(m, eq_on)
        counts = rng.integers(0, 50, size=nb)
        if eq_on and trial % 3 == 0:
            counts[1] = 10_000  # a dominant equality bucket
        N = int(counts.sum())
        kids = steps.children(counts, eq_on, r)
        if N == 0:
            assert kids == []
            continue
        assert sum(k[2] for k in kids) == N
        assert len(kids) <= 3 * r
        for a, b, size, kind in kids:
            assert size == int(counts[a:b].sum()) and size > 0
            if kind == steps.FINAL:
                assert b == a + 1 and a % 2 == 1 and size >= math.ceil(N / r)
        firsts = [k[0] for k in kids]
        assert firsts == sorted(firsts)
        L, _ = steps.pack([0 if (eq_on and i % 2 and counts[i] >= math.ceil(N / r)) else int(c)
                           for i, c in enumerate(counts)], r)
        assert all(k[2] <= L for k in kids if k[3] == steps.REG)


def test_stable_partition_matches_numpy_stable_argsort():
    rng = np.random.default_rng(17)
    child = rng.integers(0, 9, size=3000)
    sizes = np.bincount(child, minlength=9)
    dst = steps.stable_partition_dest(child, sizes)
    order = np.argsort(child, kind="stable")
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size)
    assert np.array_equal(dst, inv)


def test_level_pass_invariant():
    rng = np.random.default_rng(18)
    x = rng.integers(0, 1 << 40, size=4000).astype(np.uint64)
    x[::7] = x[3]  # plenty of one value
    samp = np.sort(steps.sample(x, 5, 0, 0, 0, 4 * 16))
    spl = steps.select_splitters(samp, 4, 16)
    eq_on = steps.eq_enabled(spl) or True
    ids, hist, kids, out = steps.level_pass(x, spl, eq_on, 4)
    assert np.array_equal(np.sort(out), np.sort(x))
    pos = 0
    prev_max = None
    for a, b, size, kind in kids:
        part = out[pos:pos + size]
        # every key of the child has an id in [a, b)
        assert np.all((steps.classify(part, spl, eq_on) >= a) & (steps.classify(part, spl, eq_on) < b))
        # keys in input order inside the child
        src = x[(ids >= a) & (ids < b)]
        assert np.array_equal(part, src)
        if prev_max is not None:
            # a key value maps to exactly one id, so children never share one
            assert part.min() > prev_max
        if kind == steps.FINAL:
            assert np.all(part == part[0])
        prev_max = part.max()
        pos += size


def test_imbalance_statistical_check_parity_unpinned():
    # Section 6 lemma (probabilistic): uniform keys, b = 16: largest group of
    # the optimal packing within (1 + 2/b) n / r in nearly all seeds.
    ok = 0
    n, r, b, a = 20000, 8, 16, 2
    for seed in range(30):
        rng = np.random.default_rng(100 + seed)
        x = rng.integers(0, 1 << 62, size=n).astype(np.uint64)
        samp = np.sort(steps.sample(x, seed, 0, 0, 0, a * b * r))
        spl = steps.select_splitters(samp, a, b * r)
        h = steps.histogram(steps.classify(x, spl, False), b * r)
        L, _ = steps.pack(h, r)
        ok += steps.imbalance_ok(L, n, r, b)
    assert ok >= 27


def test_pins_catch_planted_oracle_mistakes():
    """Plausible mistakes planted in copies of oracle functions are caught by
    the same pins that the real functions pass."""
    x = np.array([2, 0, 2, 1, 0], dtype=np.uint64)
    inv = np.empty(5, dtype=np.int64)
    inv[np.argsort(x, kind="stable")] = np.arange(5)

    def rank_without_tiebreak(v):  # dropped term
        v = np.asarray(v, dtype=np.uint64)
        return (v[None, :] < v[:, None]).sum(axis=1)

    def rank_wrong_direction(v):  # tie-break on later positions
        v = np.asarray(v, dtype=np.uint64)
        n = v.size
        after = np.triu(np.ones((n, n), dtype=bool), k=1)
        return (v[None, :] < v[:, None]).sum(axis=1) + ((v[None, :] == v[:, None]) & after).sum(axis=1)

    assert np.array_equal(steps.all_pairs_rank(x), inv)
    assert not np.array_equal(rank_without_tiebreak(x), inv)
    assert not np.array_equal(rank_wrong_direction(x), inv)

    def greedy_off_by_one(w, L):  # "<" instead of "<=" when filling a group
        starts, cur = [0], 0
        for j, wj in enumerate(w):
            if wj > L:
                return None
            if cur + wj < L:
                cur += wj
            else:
                starts.append(j)
                cur = wj
        return starts

    w, r = [3, 1, 4, 1, 5, 9, 2, 6, 5, 3], 3
    best = steps.pack_bruteforce(w, r)
    L = best
    assert len(steps.greedy_groups(w, L)) <= r
    assert len(greedy_off_by_one(w, L)) > r

    s = np.array([10, 20, 30], dtype=np.uint64)
    keys = np.array([10, 15, 20, 31], dtype=np.uint64)
    wrong_side = np.searchsorted(s, keys, side="right")  # x <= s counted as above
    assert not np.array_equal(steps.classify(keys, s, False), wrong_side)
