"""Pins for the whole-sort oracle (CPU only).

The oracle is checked against things other than itself: brute force over all
permutations (the output definition of Sections 1 and 2 applied literally),
IEEE totalOrder for float bits, numpy's stable sort where it coincides with
the definition, closed-form special cases, and independent output checkers
that must also reject planted mistakes.
"""

import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import KEY_F32, KEY_U32, KEY_U64, checkers

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_bits():
    out = []
    with open(os.path.join(GOLDEN, "f32_total_order.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                out.append(int(line.split()[0], 16))
    return out


def _keys(key_type, values):
    if key_type == KEY_F32:
        return np.array(values, dtype=np.uint32).view(np.float32)
    return np.array(values, dtype=oracle.key_dtype(key_type))


def _all_routes(key_type, keys):
    c = [int(p) for p in oracle.oracle_sort_perm(key_type, keys)]
    py = oracle.py_mergesort_perm(key_type, keys)
    return c, py


@pytest.mark.parametrize("key_type", [KEY_U32, KEY_U64])
def test_exhaustive_small_ints_match_brute_force(key_type):
    # every sequence over a 3-letter alphabet for n <= 6 (duplicates galore)
    for n in range(0, 7):
        for seq in itertools.product([5, 1, 3], repeat=n):
            keys = _keys(key_type, seq)
            bf = oracle.brute_force_perm(key_type, keys) if n else []
            c, py = _all_routes(key_type, keys)
            assert c == bf and py == bf, seq


def test_n8_random_matches_brute_force():
    rng = np.random.default_rng(1)
    for trial in range(6):
        vals = rng.integers(0, 4, size=8).astype(np.uint64) * np.uint64(0x9000000000000001)
        keys = vals.astype(np.uint64)
        bf = oracle.brute_force_perm(KEY_U64, keys)
        c, py = _all_routes(KEY_U64, keys)
        assert c == bf and py == bf


def test_float_specials_match_brute_force():
    rng = np.random.default_rng(2)
    bits = _golden_bits()
    for trial in range(40):
        n = int(rng.integers(2, 8))
        pick = [bits[int(i)] for i in rng.integers(0, len(bits), size=n)]
        keys = _keys(KEY_F32, pick)
        bf = oracle.brute_force_perm(KEY_F32, keys)
        c, py = _all_routes(KEY_F32, keys)
        assert c == bf and py == bf, [hex(b) for b in pick]


def test_float_total_order_golden():
    bits = np.array(_golden_bits(), dtype=np.uint32)
    rng = np.random.default_rng(3)
    shuffled = bits[rng.permutation(bits.size)]
    out, _ = oracle.oracle_sort(KEY_F32, shuffled.view(np.float32))
    assert np.array_equal(out.view(np.uint32), bits)
    # ord is strictly increasing along the golden list
    o = oracle.ord_keys(KEY_F32, bits.view(np.float32))
    assert np.all(o[1:] > o[:-1])


@pytest.mark.parametrize("key_type", [KEY_U32, KEY_U64])
def test_matches_numpy_stable_argsort_for_ints(key_type):
    # numpy's stable argsort orders ints by value, then position: the definition
    rng = np.random.default_rng(4)
    for n in [1, 2, 17, 1000, 65537]:
        keys = rng.integers(0, 50, size=n).astype(oracle.key_dtype(key_type))
        perm = oracle.oracle_sort_perm(key_type, keys)
        assert np.array_equal(perm.astype(np.int64), np.argsort(keys, kind="stable"))


def test_matches_numpy_for_plain_floats():
    # finite, non-zero, distinct floats: totalOrder coincides with numeric order
    rng = np.random.default_rng(5)
    keys = np.unique(rng.standard_normal(5000).astype(np.float32))
    keys = keys[keys != 0]
    rng.shuffle(keys)
    out, _ = oracle.oracle_sort(KEY_F32, keys)
    assert np.array_equal(out, np.sort(keys))


def test_special_cases():
    n = 1000
    eq = np.full(n, 7, dtype=np.uint64)
    assert np.array_equal(oracle.oracle_sort_perm(KEY_U64, eq).astype(np.int64), np.arange(n))
    inc = np.arange(n, dtype=np.uint64) * np.uint64(3)
    assert np.array_equal(oracle.oracle_sort_perm(KEY_U64, inc).astype(np.int64), np.arange(n))
    dec = inc[::-1].copy()
    assert np.array_equal(oracle.oracle_sort_perm(KEY_U64, dec).astype(np.int64),
                          np.arange(n)[::-1])
    for k in (np.zeros(0, np.uint64), np.array([42], np.uint64)):
        out, _ = oracle.oracle_sort(KEY_U64, k)
        assert np.array_equal(out, k)


def test_payload_follows_key():
    rng = np.random.default_rng(6)
    keys = rng.integers(0, 10, size=3000).astype(np.uint64)
    vals = np.arange(keys.size, dtype=np.uint32)
    ok, ov = oracle.oracle_sort(KEY_U64, keys, vals)
    assert checkers.check_pairs(KEY_U64, keys, ok, ov) is None
    assert checkers.check_keys(KEY_U64, keys, ok) is None


def test_checkers_reject_planted_mistakes():
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 20, size=500).astype(np.uint64)
    vals = np.arange(keys.size, dtype=np.uint32)
    ok, ov = oracle.oracle_sort(KEY_U64, keys, vals)
    # swap two unequal neighbours -> unsorted
    i = int(np.nonzero(ok[1:] != ok[:-1])[0][0])
    bad = ok.copy()
    bad[i], bad[i + 1] = bad[i + 1], bad[i]
    assert checkers.check_keys(KEY_U64, keys, bad) is not None
    # replace one key with a different value that keeps order -> multiset differs
    bad = ok.copy()
    bad[-1] = bad[-1] + np.uint64(1)
    assert checkers.check_keys(KEY_U64, keys, bad) is not None
    # swap payloads of two equal keys -> not stable
    j = int(np.nonzero(ok[1:] == ok[:-1])[0][0])
    badv = ov.copy()
    badv[j], badv[j + 1] = badv[j + 1], badv[j]
    assert checkers.check_pairs(KEY_U64, keys, ok, badv) is not None
    # payload naming the wrong element
    badv = ov.copy()
    badv[0] = badv[-1]
    assert checkers.check_pairs(KEY_U64, keys, ok, badv) is not None


def test_fingerprint_float_bits():
    # -0 and +0 compare equal numerically but are different bit patterns
    a = np.array([0x80000000, 0x00000000], dtype=np.uint32).view(np.float32)
    b = np.array([0x00000000, 0x00000000], dtype=np.uint32).view(np.float32)
    assert checkers.fingerprint(KEY_F32, a) != checkers.fingerprint(KEY_F32, b)


@pytest.mark.parametrize("key_type", [KEY_U32, KEY_U64, KEY_F32])
def test_parallel_mergesort_matches_stable_definition(key_type):
    # the plain parallel form (chunks + pairwise merge tree) must give the same
    # unique permutation: numpy's stable argsort of ord (value, then position)
    rng = np.random.default_rng(6)
    for n in [1, 2, 3, 7, 1000, 65537]:
        if key_type == KEY_F32:
            keys = rng.standard_normal(n).astype(np.float32)
            keys[rng.integers(0, n, size=max(1, n // 4))] = 0.0
        else:
            keys = rng.integers(0, 40, size=n).astype(oracle.key_dtype(key_type))
        want = np.argsort(oracle.ord_keys(key_type, keys), kind="stable")
        for threads in [1, 2, 3, 5, 8, 16]:
            perm = oracle.oracle_sort_perm_parallel(key_type, keys, threads)
            assert np.array_equal(perm.astype(np.int64), want), (n, threads)
