"""GPU parity of the batched sort, of deep and forced level plans, and of
oversized groups (partitioned once more, merged only beyond that)."""

import numpy as np
import pytest

import oracle
from gpu_util import gen, log, to_dev, to_host
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu
U32, U64, F32 = W.KEY_U32, W.KEY_U64, W.KEY_F32


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def _segments(rng, count, lo_exp, hi_exp):
    sizes = W.batch_sizes(count, rng, lo_exp, hi_exp)
    sizes[::17] = 0
    sizes[1::19] = 1
    return sizes


@pytest.mark.parametrize("kt", [U64, U32, F32])
def test_batch_keys_match_oracle_per_segment(api, kt):
    rng = np.random.default_rng(31 + kt)
    sizes = _segments(rng, 300, 4, 17)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = gen(kt, int(offs[-1]), "uniform", 40 + kt)
    log("batch kt=%d segments=%d total=%d" % (kt, sizes.size, int(offs[-1])))
    out = to_host(api.sort_batch(to_dev(keys), offs))
    for i in range(sizes.size):
        a, b = int(offs[i]), int(offs[i + 1])
        want, _ = oracle.oracle_sort(kt, keys[a:b])
        assert np.array_equal(out[a:b].view(np.uint8), want.view(np.uint8)), i


def test_batch_pairs_and_alone_equals_in_batch(api):
    rng = np.random.default_rng(33)
    sizes = _segments(rng, 120, 6, 18)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    keys = gen(U64, n, "few", 41)
    vals = np.arange(n, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    ok, ov = api.sort_batch(dk, offs, vals=dv)
    ok, ov = to_host(ok), to_host(ov)
    for i in range(sizes.size):
        a, b = int(offs[i]), int(offs[i + 1])
        wk, wv = oracle.oracle_sort(U64, keys[a:b], vals[a:b])
        assert np.array_equal(ok[a:b], wk) and np.array_equal(ov[a:b], wv), i
        if b - a > 0 and i % 10 == 0:
            ak, av = api.sort_pairs(to_dev(keys[a:b].copy()), to_dev(vals[a:b].copy()))
            assert np.array_equal(to_host(ak), ok[a:b]) and np.array_equal(to_host(av), ov[a:b])


def test_batch_in_place_and_device_offsets(api):
    import torch
    rng = np.random.default_rng(35)
    sizes = _segments(rng, 64, 8, 16)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = gen(U32, int(offs[-1]), "uniform", 43)
    d = to_dev(keys)
    api.sort_batch(d, offs, out_keys=d, d_offsets=torch.from_numpy(offs).cuda())
    out = to_host(d)
    for i in range(sizes.size):
        a, b = int(offs[i]), int(offs[i + 1])
        want, _ = oracle.oracle_sort(U32, keys[a:b])
        assert np.array_equal(out[a:b], want)


# Keys-only scatter paths: per-wavefront scans (at most 768 children, tree
# area a multiple of 16 bytes), the block scan for wider levels (k = 1024),
# the block scan for a uint32 tree of two splitter slots (k * b = 2, an
# 8-byte tree area), and per-wavefront scans for one of four.
@pytest.mark.parametrize("kt,levels,k,b", [(U64, 3, 4, 2), (U64, 2, 16, 4), (U64, 1, 1024, 2),
                                           (U64, 3, 64, 1), (U32, 4, 2, 1), (U32, 3, 4, 1)])
def test_forced_level_plans(api, kt, levels, k, b):
    n = 300000
    keys = gen(kt, n, "uniform", 50 + levels * k)
    p = api.make_params(levels=levels, k=k, overpartition_b=b, samples_per_bucket=4)
    log("kt=%d levels=%d k=%d b=%d" % (kt, levels, k, b))
    out = to_host(api.sort_keys(to_dev(keys), params=p))
    want, _ = oracle.oracle_sort(kt, keys)
    assert np.array_equal(out, want)


def _sort_with_stats(api, kt, keys, p, vals=None, offsets=None):
    """Sort through the C ABI in a workspace of our own; (keys, vals, stats)."""
    n = keys.size
    if offsets is None:
        ws = api.alloc_workspace(api.workspace_bytes(kt, n, vals is not None, p))
        if vals is None:
            return to_host(api.sort_keys(to_dev(keys), params=p, workspace=ws)), None, \
                api.workspace_stats(ws)
        ok, ov = api.sort_pairs(to_dev(keys), to_dev(vals), params=p, workspace=ws)
        return to_host(ok), to_host(ov), api.workspace_stats(ws)
    ws = api.alloc_workspace(api.batch_workspace_bytes(kt, offsets, vals is not None, p))
    if vals is None:
        return to_host(api.sort_batch(to_dev(keys), offsets, params=p, workspace=ws)), None, \
            api.workspace_stats(ws)
    ok, ov = api.sort_batch(to_dev(keys), offsets, vals=to_dev(vals), params=p, workspace=ws)
    return to_host(ok), to_host(ov), api.workspace_stats(ws)


# Oversized groups (more keys than a leaf holds once the planned levels are
# done) are partitioned once more in HBM by their workgroup, into buckets of
# about a quarter of a leaf; only a bucket still larger than a leaf is merged.
@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("dist", ["uniform", "few", "zipf", "sorted"])
def test_oversized_groups_partitioned(api, kt, pairs, dist):
    # one level of 4 groups over 100000 keys with 1024-key leaves: every
    # group holds about 25000 keys, 64 buckets of about 400 each
    n = 100000
    keys = gen(kt, n, dist, 60)
    vals = np.arange(n, dtype=np.uint32) if pairs else None
    p = api.make_params(levels=1, k=4, overpartition_b=1, leaf_capacity=1024)
    log("oversized groups kt=%d pairs=%s %s" % (kt, pairs, dist))
    ok, ov, st = _sort_with_stats(api, kt, keys, p, vals)
    wk, wv = oracle.oracle_sort(kt, keys, vals)
    assert np.array_equal(ok.view(np.uint8), wk.view(np.uint8))
    if pairs:
        assert np.array_equal(ov, wv)
    assert st["device_errors"] == 0
    if dist != "few":  # few distinct keys: the level's equality buckets take them
        assert st["big_leaves"] >= 1 and st["big_keys"] > 0
    if dist == "uniform":
        assert st["merge_ranges"] == 0, st


@pytest.mark.parametrize("kt", [U64, F32])
@pytest.mark.parametrize("pairs", [False, True])
def test_oversized_group_pieces_without_room(api, kt, pairs):
    # the pieces find the leaf list full (test hook): the remainder pass
    # after the base case sorts and copies them instead
    n = 100000
    keys = gen(kt, n, "zipf", 65)
    vals = np.arange(n, dtype=np.uint32) if pairs else None
    p = api.make_params(levels=1, k=4, overpartition_b=1, leaf_capacity=1024, flags=64)
    log("oversized pieces without room kt=%d pairs=%s" % (kt, pairs))
    ok, ov, st = _sort_with_stats(api, kt, keys, p, vals)
    wk, wv = oracle.oracle_sort(kt, keys, vals)
    assert np.array_equal(ok.view(np.uint8), wk.view(np.uint8))
    if pairs:
        assert np.array_equal(ov, wv)
    assert st["big_leaves"] >= 1 and st["device_errors"] == 0, st


@pytest.mark.parametrize("pairs", [False, True])
def test_oversized_groups_partitioned_twice(api, pairs):
    # groups of 2^20 keys with 1024-key leaves: the first partition leaves 64
    # buckets of about 16384 keys, each partitioned once more into pieces
    # that fit a leaf; nothing is merged
    n = 1 << 21
    keys = gen(U64, n, "uniform", 61)
    vals = np.arange(n, dtype=np.uint32) if pairs else None
    p = api.make_params(levels=1, k=2, overpartition_b=1, leaf_capacity=1024)
    log("oversized groups partitioned twice pairs=%s" % pairs)
    ok, ov, st = _sort_with_stats(api, U64, keys, p, vals)
    wk, wv = oracle.oracle_sort(U64, keys, vals)
    assert np.array_equal(ok, wk)
    if pairs:
        assert np.array_equal(ov, wv)
    assert st["big_leaves"] == 2 and st["merge_ranges"] == 0 and st["device_errors"] == 0, st


@pytest.mark.parametrize("pairs", [False, True])
def test_oversized_groups_beyond_two_partitions_merge(api, pairs):
    # groups of 2^23 keys with 1024-key leaves: two partitions of 64 buckets
    # leave pieces of about 2048 keys, which the merge fallback sorts
    n = 1 << 24
    keys = gen(U64, n, "uniform", 64)
    vals = np.arange(n, dtype=np.uint32) if pairs else None
    p = api.make_params(levels=1, k=2, overpartition_b=1, leaf_capacity=1024)
    log("oversized groups beyond two partitions pairs=%s" % pairs)
    ok, ov, st = _sort_with_stats(api, U64, keys, p, vals)
    wk, wv = oracle.oracle_sort(U64, keys, vals)
    assert np.array_equal(ok, wk)
    if pairs:
        assert np.array_equal(ov, wv)
    assert st["big_leaves"] == 2 and st["merge_ranges"] > 64 and st["device_errors"] == 0, st


@pytest.mark.parametrize("pairs", [False, True])
def test_oversized_groups_in_a_skewed_batch(api, pairs):
    # a few large segments among many small ones, 2048-key leaves, one level:
    # the large segments' groups are oversized, the small ones fit a leaf
    rng = np.random.default_rng(62)
    sizes = rng.integers(1, 3000, 200).astype(np.int64)
    sizes[[3, 50, 51, 120]] = [400000, 250000, 123457, 300001]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    keys = gen(U64, n, "zipf", 63)
    vals = np.arange(n, dtype=np.uint32) if pairs else None
    p = api.make_params(levels=1, k=8, leaf_capacity=2048)
    log("skewed batch pairs=%s n=%d" % (pairs, n))
    ok, ov, st = _sort_with_stats(api, U64, keys, p, vals, offsets=offs)
    for i in range(sizes.size):
        a, b = int(offs[i]), int(offs[i + 1])
        wk, wv = oracle.oracle_sort(U64, keys[a:b], None if vals is None else vals[a:b])
        assert np.array_equal(ok[a:b], wk), i
        if pairs:
            assert np.array_equal(ov[a:b], wv), i
    assert st["big_leaves"] >= 4 and st["device_errors"] == 0, st


def test_workspace_given_by_caller(api):
    n = 200000
    keys = gen(F32, n, "uniform", 70)
    wsb = api.workspace_bytes(F32, n)
    ws = api.alloc_workspace(wsb)
    out = to_host(api.sort_keys(to_dev(keys), workspace=ws))
    want, _ = oracle.oracle_sort(F32, keys)
    assert np.array_equal(out.view(np.uint32), want.view(np.uint32))
    from paper_1410_6754_amd import AmsError
    with pytest.raises(AmsError):
        api.sort_keys(to_dev(keys), workspace=api.alloc_workspace(wsb // 2))


@pytest.mark.parametrize("kt", [U64, F32])
def test_stable_partition_flag_same_result(api, kt):
    # keys-only through the stable (ballot-ranked) scatter: same sorted output
    n = 500000
    keys = gen(kt, n, "few", 80)
    p = api.make_params(flags=2, levels=2, k=64)
    out = to_host(api.sort_keys(to_dev(keys), params=p))
    want, _ = oracle.oracle_sort(kt, keys)
    assert np.array_equal(out.view(np.uint8), want.view(np.uint8))


@pytest.mark.parametrize("pay", [False, True])
def test_autotuned_parameters_sort_identically(api, pay):
    # the autotuner's choice (and the remembered choice used by a call with
    # default parameters) must give the oracle's output on every segment
    rng = np.random.default_rng(35 + pay)
    sizes = _segments(rng, 200, 8, 16)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    keys = gen(U64, n, "uniform", 43 + pay)
    vals = np.arange(n, dtype=np.uint32) if pay else None
    dk = to_dev(keys)
    dv = to_dev(vals) if pay else None
    api.autotune_clear()
    log("autotune pay=%s segments=%d total=%d" % (pay, sizes.size, n))
    best, ms = api.autotune(dk, offs, vals=dv, max_trials=6)
    log("tuned %s in %.3f ms" % (api.params_dict(best), ms))
    assert ms > 0
    assert best.k >= 2 and (best.k & (best.k - 1)) == 0
    assert best.k * best.overpartition_b <= 2048
    outs = [api.sort_batch(dk, offs, vals=dv, params=best), api.sort_batch(dk, offs, vals=dv)]
    for out in outs:
        ok = to_host(out[0] if pay else out)
        ov = to_host(out[1]) if pay else None
        for i in range(sizes.size):
            a, b = int(offs[i]), int(offs[i + 1])
            wk, wv = oracle.oracle_sort(U64, keys[a:b], None if vals is None else vals[a:b])
            assert np.array_equal(ok[a:b], wk), i
            if pay:
                assert np.array_equal(ov[a:b], wv), i
    api.autotune_clear()


def test_autotune_rejects_bad_arguments(api):
    from paper_1410_6754_amd._lib import AmsError
    dk = to_dev(gen(U64, 1000, "uniform", 45))
    with pytest.raises(ValueError):
        api.autotune(dk, [0, 10])
    with pytest.raises(AmsError):
        api.autotune(dk, [5, 1000])  # offsets must start at 0


def test_batch_stratified_splitters(api):
    """Batched segments with strata below the first level: each segment
    equals the oracle."""
    import oracle
    rng = np.random.default_rng([W.BASE_SEED, 830])
    sizes = W.batch_sizes(300, rng, 8, 20)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = W.uniform_u64(int(offs[-1]), rng)
    p = api.make_params(levels=2, flags=32)
    out = to_host(api.sort_batch(to_dev(keys), offs, params=p))
    for i in range(sizes.size):
        a, b = int(offs[i]), int(offs[i + 1])
        want, _ = oracle.oracle_sort(W.KEY_U64, keys[a:b])
        assert np.array_equal(out[a:b], want), i
