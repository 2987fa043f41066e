"""GPU parity of single steps (through the C ABI step entry points) against
the oracle's step models: splitter selection, one level (classification,
histogram, grouping, children, stable scatter), bucket grouping alone, and
the base case with various cutoffs."""

import math

import numpy as np
import pytest

import oracle
from oracle import rng as orng
from oracle import steps
from gpu_util import gen, log, to_dev, to_host
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu
U32, U64, F32 = W.KEY_U32, W.KEY_U64, W.KEY_F32


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def _oracle_splitters(kt, keys, m, a, seed):
    ords = oracle.ord_keys(kt, keys)
    pos = orng.sample_positions(seed, 0, 0, 0, keys.size, a * m)
    samp = ords[np.asarray(pos, dtype=np.int64)]
    # the sample is sorted by its all-pairs ranks (Section 4.2)
    srt = steps.sort_by_rank(samp) if samp.size <= 2048 else np.sort(samp, kind="stable")
    return steps.select_splitters(srt, a, m)


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("m,a", [(16, 16), (256, 1), (256, 16), (1024, 8), (2048, 4)])
def test_splitters(api, kt, m, a):
    if kt != U64 and a * m > 16384:
        pytest.skip("sample larger than the 32-bit cap")
    if kt == U64 and a * m > 8192:
        pytest.skip("sample larger than the 64-bit cap")
    n = 50000
    keys = gen(kt, n, "few" if m == 16 else "uniform", m + a)
    seed = 1234 + m
    log("splitters kt=%d m=%d a=%d" % (kt, m, a))
    got = to_host(api.step_splitters(to_dev(keys), m, a, seed))
    want = _oracle_splitters(kt, keys, m, a, seed).astype(got.dtype)
    assert np.array_equal(got, want)


def test_sample_rank_pins_numpy_for_large_samples():
    # the large-sample route above sorts with numpy: check it equals the
    # all-pairs ranking on a sample of the same kind
    x = np.random.default_rng(5).integers(0, 1 << 60, size=1500).astype(np.uint64)
    assert np.array_equal(steps.sort_by_rank(x), np.sort(x, kind="stable"))


@pytest.mark.parametrize("stable", [False, True])
@pytest.mark.parametrize("kt", [U64, U32])
@pytest.mark.parametrize("m,r,dist,flags", [
    (16, 4, "uniform", 0), (256, 64, "uniform", 0), (1024, 256, "uniform", 0),
    (64, 16, "few", 0), (64, 16, "few", 1), (32, 8, "equal", 1), (256, 256, "zipf", 1)])
def test_level(api, kt, m, r, dist, flags, stable):
    n = 40000 + 17
    keys = gen(kt, n, dist, m * 7 + r)
    ords = oracle.ord_keys(kt, keys)
    samp = np.sort(steps.sample(ords, 99, 0, 0, 0, 4 * m))
    spl = steps.select_splitters(samp, 4, m)
    eq_on = steps.eq_enabled(spl) or bool(flags & 1)
    log("level kt=%d m=%d r=%d %s eq=%s" % (kt, m, r, dist, eq_on))
    ids, hist, kids, out = steps.level_pass(ords, spl, eq_on, r)
    d_spl = to_dev(spl.astype(keys.dtype if kt != F32 else np.uint32))
    gflags = flags | (2 if stable else 0)  # AMS_FLAG_STABLE_PARTITION
    gout, ghist, gkids = api.step_level(to_dev(keys), d_spl, m, r, gflags)
    gout, ghist, gkids = to_host(gout), to_host(ghist), to_host(gkids)
    nb = steps.num_ids(m, eq_on)
    assert np.array_equal(ghist[:nb].astype(np.int64), hist)
    assert [tuple(int(v) for v in row) for row in gkids] == [tuple(k) for k in kids]
    g = gout.astype(np.uint64)
    if stable:
        # the stable counting partition, element by element
        assert np.array_equal(g, out)
    else:
        # keys-only regroups a tile without keeping order inside a child:
        # what is unique is every child's multiset of keys
        pos = 0
        for a, b, size, kind in kids:
            assert np.array_equal(np.sort(g[pos:pos + size]), np.sort(out[pos:pos + size]))
            pos += size


def test_pack(api):
    import torch
    rng = np.random.default_rng(21)
    cases = []
    for trial in range(60):
        nb = int(rng.integers(1, 4096))
        r = int(rng.choice([1, 2, 3, 7, 64, 256, 1024]))
        w = rng.integers(0, 1000, size=nb).astype(np.uint32)
        if trial % 5 == 0:
            w[rng.integers(0, nb, size=max(1, nb // 3))] = 0
        if trial % 7 == 0:
            w[int(rng.integers(0, nb))] = 100000
        cases.append((w, r))
    cases.append((np.zeros(10, np.uint32), 3))
    cases.append((np.array([5], np.uint32), 1))
    # ceil(W/r) + the largest bucket passes 2^32 while W does not
    cases.append((np.array([2 ** 30, 2 ** 31 + 2 ** 20, 2 ** 30 - 2 ** 21], np.uint32), 2))
    cases.append((np.array([2 ** 31, 2 ** 31 - 1], np.uint32), 1))
    cases.append((np.array([2 ** 20, 2 ** 32 - 2 ** 21, 0, 2 ** 19], np.uint32), 3))
    for w, r in cases:
        L, starts = steps.pack([int(v) for v in w], r)
        out = to_host(api.step_pack(torch.from_numpy(w).cuda(), r))
        g = int(out[1])
        assert int(out[0]) == L, (w.size, r)
        assert [int(v) for v in out[2:2 + g]] == starts


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("cutoff", [2, 16, 64, 1024])
@pytest.mark.parametrize("dist", ["uniform", "few", "equal"])
def test_base_case_cutoffs(api, kt, cutoff, dist):
    n = 7000
    keys = gen(kt, n, dist, cutoff)
    log("base case kt=%d cutoff=%d %s" % (kt, cutoff, dist))
    out = to_host(api.step_base_case(to_dev(keys), cutoff=cutoff))
    want, _ = oracle.oracle_sort(kt, keys)
    assert np.array_equal(out.view(np.uint8), want.view(np.uint8))
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = api.step_base_case(to_dev(keys), to_dev(vals), cutoff=cutoff)
    wk, wv = oracle.oracle_sort(kt, keys, vals)
    assert np.array_equal(to_host(ok).view(np.uint8), wk.view(np.uint8))
    assert np.array_equal(to_host(ov), wv)


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("dist", ["uniform", "sorted", "zipf", "few", "specials"])
@pytest.mark.parametrize("split", ["range", "sampled"])
def test_base_case_split_kinds(api, kt, dist, split):
    # the key-range split (kept when balanced) and the sampled split give the
    # same output; the flag forces the sampled one on every leaf (float32
    # "uniform" keys are normal(0, 1))
    n = 7777
    keys = gen(kt, n, dist, 77)
    flags = 4 if split == "sampled" else 0  # AMS_FLAG_SAMPLED_LEAF_SPLIT
    p = api.make_params(base_cutoff=32, flags=flags)
    log("split kinds kt=%d %s %s" % (kt, dist, split))
    out = to_host(api.sort_keys(to_dev(keys), params=p))
    want, _ = oracle.oracle_sort(kt, keys)
    assert np.array_equal(out.view(np.uint8), want.view(np.uint8))
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = api.sort_pairs(to_dev(keys), to_dev(vals), params=p)
    wk, wv = oracle.oracle_sort(kt, keys, vals)
    assert np.array_equal(to_host(ok).view(np.uint8), wk.view(np.uint8))
    assert np.array_equal(to_host(ov), wv)


def test_all_pairs_rank_definition_on_gpu(api):
    # base case with one bucket (n <= cutoff): the result is the all-pairs
    # rank placement of Section 4.2
    keys = gen(U64, 700, "few", 3)
    out = to_host(api.step_base_case(to_dev(keys), cutoff=1024))
    ranks = steps.all_pairs_rank(keys)
    want = np.empty_like(keys)
    want[ranks] = keys
    assert np.array_equal(out, want)


@pytest.mark.parametrize("spread", [1 << 40, 1 << 33, 1 << 20])
def test_base_case_near_ties(api, spread):
    # uint64 keys that differ only in their low bits inside a wide leaf: the
    # ranking compares the high words of the keys' offsets, so such keys tie
    # there and must still come out in exact order (and equal keys stay equal)
    rng = np.random.default_rng([W.BASE_SEED, 93, spread.bit_length()])
    n = 7500
    centers = rng.integers(0, spread, size=60, dtype=np.uint64)
    keys = centers[rng.integers(0, centers.size, size=n)] + rng.integers(0, 300, size=n, dtype=np.uint64)
    keys[::7] = keys[1::7][: keys[::7].size]  # exact duplicates too
    log("near ties spread=2^%d" % (spread.bit_length() - 1))
    for flags in (0, 4):
        p = api.make_params(base_cutoff=32, flags=flags)
        out = to_host(api.sort_keys(to_dev(keys), params=p))
        want, _ = oracle.oracle_sort(U64, keys)
        assert np.array_equal(out, want), flags
    big = np.concatenate([keys + np.uint64(i) * np.uint64(spread) for i in range(40)])
    rng.shuffle(big)
    p = api.make_params(levels=1, k=64, overpartition_b=2)
    out = to_host(api.sort_keys(to_dev(big), params=p))
    want, _ = oracle.oracle_sort(U64, big)
    assert np.array_equal(out, want)
