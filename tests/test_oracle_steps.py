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


def test_pack_weights_near_2_to_32():
    # few groups and one heavy bucket: ceil(W/r) + the largest bucket passes
    # 2^32 while W does not; the optimum is worked out by hand
    w = [2 ** 30, 2 ** 31 + 2 ** 20, 2 ** 30 - 2 ** 21]
    L, starts = steps.pack(w, 2)
    assert L == steps.pack_bruteforce(w, 2) == 3 * 2 ** 30 - 2 ** 20
    assert starts == [0, 1]
    w = [2 ** 31, 2 ** 31 - 1]
    assert steps.pack(w, 1) == (2 ** 32 - 1, [0])


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


# ----------------------------------------------------------------------------
# children(): hand-worked golden cases and planted mistakes
# ----------------------------------------------------------------------------

def _golden_children():
    cases = []
    with open(os.path.join(GOLDEN, "children.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            head, counts, kids = [p.strip() for p in line.split("|")]
            r, eq_on = [int(v) for v in head.split()]
            counts = [int(v) for v in counts.split()]
            want = []
            for k in kids.split(";"):
                a, b, size, kind = k.split()
                want.append((int(a), int(b), int(size), steps.FINAL if kind == "F" else steps.REG))
            cases.append((r, bool(eq_on), counts, want))
    return cases


def test_children_golden_cases():
    cases = _golden_children()
    assert len(cases) >= 8
    for r, eq_on, counts, want in cases:
        assert steps.children(counts, eq_on, r) == want, (r, eq_on, counts)
    assert steps.children([0, 0, 0], True, 2) == []


def _children_variant(counts, eq_on, r, *, strict=False, cut=True, drop_empty=True,
                      even_final=False):
    """children() with one planted mistake switched on."""
    c = [int(v) for v in counts]
    N = sum(c)
    if N == 0:
        return []
    tfin = -(-N // r)
    def is_final(i):
        if not eq_on or (i % 2 == 0 and not even_final):
            return False
        return c[i] > tfin if strict else c[i] >= tfin
    final = [is_final(i) for i in range(len(c))]
    w = [0 if final[i] else c[i] for i in range(len(c))]
    _, starts = steps.pack(w, r)
    ends = starts[1:] + [len(c)]
    out = []
    for gs, ge in zip(starts, ends):
        run_start = gs
        for i in range(gs, ge):
            if final[i] and cut:
                size = sum(c[run_start:i])
                if size or not drop_empty:
                    out.append((run_start, i, size, steps.REG))
                out.append((i, i + 1, c[i], steps.FINAL))
                run_start = i + 1
        size = sum(c[run_start:ge])
        if size or not drop_empty:
            out.append((run_start, ge, size, steps.REG))
    return out


def test_children_pins_catch_planted_mistakes():
    cases = _golden_children()
    # the variant with no mistake switched on reproduces every golden case
    for r, eq_on, counts, want in cases:
        assert _children_variant(counts, eq_on, r) == want
    mistakes = {
        "final threshold > instead of >=": dict(strict=True),
        "no cut at a final id": dict(cut=False),
        "empty piece kept": dict(drop_empty=False),
        "final id on a regular (even) bucket": dict(even_final=True),
    }
    for name, kw in mistakes.items():
        caught = any(_children_variant(counts, eq_on, r, **kw) != want
                     for r, eq_on, counts, want in cases)
        assert caught, name


# ----------------------------------------------------------------------------
# eq_enabled(): brute force over small sorted splitter arrays
# ----------------------------------------------------------------------------

def _eq_brute(spl):
    """Some two splitters (any positions) are equal."""
    s = [int(v) for v in spl]
    return any(s[i] == s[j] for i in range(len(s)) for j in range(i + 1, len(s)))


def test_eq_enabled_brute_force():
    seen = 0
    for n in range(0, 7):
        for seq in itertools.combinations_with_replacement(range(4), n):
            spl = np.array(seq, dtype=np.uint64)  # sorted, as splitters are
            assert steps.eq_enabled(spl) == _eq_brute(seq), seq
            seen += 1
    assert seen > 200
    # large ord values (top bit set) compare as unsigned
    big = np.array([1 << 63, (1 << 63) + 1, (1 << 64) - 1], dtype=np.uint64)
    assert not steps.eq_enabled(big)
    assert steps.eq_enabled(np.array([5, (1 << 64) - 1, (1 << 64) - 1], dtype=np.uint64))


def test_eq_enabled_pins_catch_planted_mistakes():
    def skip_one(spl):  # compares s[i] with s[i+2]
        s = np.asarray(spl, dtype=np.uint64)
        return bool(s.size > 2 and np.any(s[2:] == s[:-2]))

    def first_pair_only(spl):  # looks at the first two splitters only
        s = np.asarray(spl, dtype=np.uint64)
        return bool(s.size > 1 and s[0] == s[1])

    def wrong_size_guard(spl):  # needs three splitters before it looks
        s = np.asarray(spl, dtype=np.uint64)
        return bool(s.size > 2 and np.any(s[1:] == s[:-1]))

    for bad in (skip_one, first_pair_only, wrong_size_guard):
        caught = False
        for n in range(0, 7):
            for seq in itertools.combinations_with_replacement(range(4), n):
                if bad(np.array(seq, dtype=np.uint64)) != _eq_brute(seq):
                    caught = True
        assert caught, bad.__name__


# ----------------------------------------------------------------------------
# sample positions: tied to the published SplitMix64 outputs
# ----------------------------------------------------------------------------

def test_stream_state_first_stage_is_published_output():
    # the first fold is SplitMix64's first output at the seed, which the
    # golden file pins (seed 0 -> 16294208416658607535)
    assert orng.mix64(orng.GAMMA) == 16294208416658607535
    assert orng.splitmix64_outputs(1234567, 1)[0] == orng.mix64(1234567 + orng.GAMMA)


def test_sample_positions_are_top_bits_of_the_stream():
    # for n = 2^k, floor(n u / 2^64) is the top k bits of u, and u_i is output
    # i+1 of SplitMix64 started at the subproblem's stream state
    for k in (1, 7, 20, 32):
        st = orng.stream_state(3, 1, 4, 1000)
        outs = orng.splitmix64_outputs(st, 64)
        pos = orng.sample_positions(3, 1, 4, 1000, 1 << k, 64)
        assert pos == [o >> (64 - k) for o in outs]


def test_sample_positions_uniform_chi_square():
    # 65536 draws over 256 cells: chi-square with 255 degrees of freedom
    # stays below 340 with probability > 0.999
    pos = np.asarray(orng.sample_positions(14106754, 0, 0, 0, 256 * 1000, 65536)) // 1000
    cnt = np.bincount(pos, minlength=256)
    e = 65536 / 256
    chi2 = float(((cnt - e) ** 2 / e).sum())
    assert chi2 < 340, chi2


def test_stream_states_are_distinct():
    # every (level, root, offset) key gives its own stream
    states = {orng.stream_state(7, lv, root, off)
              for lv in range(4) for root in range(16) for off in (0, 1, 4096, 1 << 20)}
    assert len(states) == 4 * 16 * 4
