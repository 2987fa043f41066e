"""GPU parity: the HIP sort, through the C ABI, equals the oracle bit for bit.

Sizes span the base case alone (n <= 8192), one partition level and two
levels, with ragged tails; distributions cover uniform keys, heavy
duplicates, Zipf, all-equal, sorted, reversed and float specials.
"""

import numpy as np
import pytest

from gpu_util import check_sort_keys, check_sort_pairs, gen, log, to_dev, to_host
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu

U32, U64, F32 = W.KEY_U32, W.KEY_U64, W.KEY_F32


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    A.sort_keys  # noqa: B018
    return A


SMALL = [0, 1, 2, 3, 31, 63, 64, 65, 255, 1023, 1024, 1025, 4095, 8191, 8192]
LEVEL = [8193, 20000, 65537, 300001]


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("n", SMALL)
def test_base_case_sizes(api, kt, n):
    log("base case kt=%d n=%d" % (kt, n))
    check_sort_keys(api, kt, gen(kt, n, "uniform", n), what="kt%d n%d" % (kt, n))


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("n", LEVEL)
def test_one_level_sizes(api, kt, n):
    log("one level kt=%d n=%d" % (kt, n))
    check_sort_keys(api, kt, gen(kt, n, "uniform", 100 + n), what="kt%d n%d" % (kt, n))


@pytest.mark.parametrize("dist", ["few", "zipf", "equal", "sorted", "reversed", "specials"])
@pytest.mark.parametrize("n", [5000, 100000])
def test_distributions_u64(api, dist, n):
    log("dist %s n=%d" % (dist, n))
    check_sort_keys(api, U64, gen(U64, n, dist, 7), what=dist)


@pytest.mark.parametrize("dist", ["few", "specials", "equal"])
def test_distributions_f32(api, dist):
    log("f32 dist %s" % dist)
    check_sort_keys(api, F32, gen(F32, 70000, dist, 8), what=dist)


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("distinct", [3, 40, 1000])
def test_keys_only_dense_duplicates(api, kt, distinct):
    """Keys-only leaves where most keys tie with others: equal keys share a
    rank in the first ranking pass, and every bucket with such ties is ranked
    again exactly; also normal float32 keys, whose values repeat once there
    are a few million of them (the serving mix)."""
    log("dense duplicates kt=%d distinct=%d" % (kt, distinct))
    rng = np.random.default_rng([W.BASE_SEED, 900 + distinct + kt])
    n = 300001
    if kt == F32:
        vals = np.round(rng.normal(0.0, 1.0, distinct) * 64.0) / 64.0
        keys = rng.choice(vals.astype(np.float32), n)
    else:
        dt = np.uint64 if kt == U64 else np.uint32
        pool = rng.integers(0, np.iinfo(dt).max, distinct, dtype=dt, endpoint=True)
        keys = rng.choice(pool, n)
    check_sort_keys(api, kt, keys, what="kt%d distinct%d" % (kt, distinct))


@pytest.mark.parametrize("hibits", [12, 20, 28])
@pytest.mark.parametrize("n", [300001, 3000001])
def test_u64_shared_high_words(api, hibits, n):
    """uint64 keys whose high 32-bit words take few values: the partition
    levels classify on high words first and must redo, on the full keys,
    every wavefront holding a key whose high word equals a splitter's."""
    log("shared high words hibits=%d n=%d" % (hibits, n))
    rng = np.random.default_rng([W.BASE_SEED, 950 + hibits])
    # 2^hibits distinct high words spread over the 32-bit range, random low words
    hi = rng.integers(0, 1 << hibits, n, dtype=np.uint64) << np.uint64(64 - hibits)
    keys = hi | rng.integers(0, 1 << 32, n, dtype=np.uint64)
    check_sort_keys(api, U64, keys, what="hibits%d n%d" % (hibits, n))


def test_keys_only_normal_f32_repeats(api):
    log("normal f32 with repeated values")
    keys = gen(F32, 1 << 23, "uniform", 31)  # float32 keys are N(0, 1)
    check_sort_keys(api, F32, keys, what="normal f32 2^23")


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("n", [1, 100, 8192, 50000])
def test_pairs_stable(api, kt, n):
    log("pairs kt=%d n=%d" % (kt, n))
    check_sort_pairs(api, kt, gen(kt, n, "few", 9 + n), what="pairs")


def test_pairs_hard_distributions(api):
    for dist in ["zipf", "equal", "few", "reversed"]:
        log("pairs dist %s" % dist)
        check_sort_pairs(api, U64, gen(U64, 200000, dist, 10), what=dist)


# Forced plans that route pairs through both stable scatters: levels with at
# most 1024 children whose tables fit next to an 8192-pair chunk use the
# 1024-thread kernel; wider ones (k = 512 or 1024, or k * b = 2048 with
# 64-bit keys) the 256-thread one.
@pytest.mark.parametrize("kt", [U64, U32])
@pytest.mark.parametrize("levels,k,b", [(1, 1024, 2), (1, 512, 2), (2, 256, 8), (2, 128, 2), (3, 16, 4)])
def test_pairs_forced_level_plans(api, kt, levels, k, b):
    n = 300001
    log("pairs kt=%d levels=%d k=%d b=%d" % (kt, levels, k, b))
    p = api.make_params(levels=levels, k=k, overpartition_b=b)
    for dist in ["uniform", "few"]:
        check_sort_pairs(api, kt, gen(kt, n, dist, 70 + k + levels), params=p, what=dist)


def test_two_levels(api):
    n = (1 << 22) + 12345
    log("two levels n=%d" % n)
    check_sort_keys(api, U64, gen(U64, n, "uniform", 11), what="2lvl")


# Sorted and reversed input over two levels: at the second level a bucket
# holds a few thousand keys, so the count kernel's rows mostly share a
# bucket (row-wise adds) while the tile tails stay partial.
@pytest.mark.parametrize("kt", [U64, U32])
@pytest.mark.parametrize("dist", ["sorted", "reversed"])
def test_two_levels_ordered_input(api, kt, dist):
    n = (1 << 22) + 12345
    log("two levels kt=%d %s n=%d" % (kt, dist, n))
    check_sort_keys(api, kt, gen(kt, n, dist, 13), what="2lvl " + dist)


def test_in_place(api):
    keys = gen(U64, 100000, "uniform", 12)
    import oracle
    d = to_dev(keys)
    api.sort_keys(d, out=d)
    want, _ = oracle.oracle_sort(U64, keys)
    assert np.array_equal(to_host(d), want)
    vals = np.arange(keys.size, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    api.sort_pairs(dk, dv, out_keys=dk, out_vals=dv)
    wk, wv = oracle.oracle_sort(U64, keys, vals)
    assert np.array_equal(to_host(dk), wk) and np.array_equal(to_host(dv), wv)


def test_determinism(api):
    keys = gen(U64, 300000, "few", 13)
    d = to_dev(keys)
    a = to_host(api.sort_keys(d))
    b = to_host(api.sort_keys(d))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_sampled_leaf_split_full_sort(api, dist):
    # two partition levels with every leaf split by sampled splitters
    n = 1_500_000
    keys = gen(U64, n, dist, 91)
    p = api.make_params(levels=2, k=64, overpartition_b=4, flags=4)  # AMS_FLAG_SAMPLED_LEAF_SPLIT
    log("sampled leaf split %s n=%d" % (dist, n))
    check_sort_keys(api, U64, keys, params=p, what="sampled leaf split")


# Splitters below the first level that follow the parent buckets (the
# overpartitioning exploited in the recursion): same output on every shape.
STRAT = 32  # AMS_FLAG_STRATIFIED


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("dist", ["uniform", "few", "zipf", "sorted", "reversed", "specials"])
def test_stratified_splitters_keys(api, kt, dist):
    n = 1_500_007
    p = api.make_params(levels=2, k=64, overpartition_b=4, flags=STRAT)
    log("stratified kt=%d %s n=%d" % (kt, dist, n))
    check_sort_keys(api, kt, gen(kt, n, dist, 800), params=p, what="stratified " + dist)


@pytest.mark.parametrize("levels,k,b", [(2, 256, 4), (3, 16, 4), (2, 128, 8)])
def test_stratified_splitters_pairs(api, levels, k, b):
    p = api.make_params(levels=levels, k=k, overpartition_b=b, flags=STRAT)
    for dist in ("uniform", "few", "equal"):
        log("stratified pairs levels=%d k=%d b=%d %s" % (levels, k, b, dist))
        check_sort_pairs(api, U64, gen(U64, 2_000_003, dist, 810), params=p,
                         what="stratified pairs " + dist)


def test_stratified_splitters_large_with_stats(api):
    """Two levels of k = 256, b = 4 on 2^24 + odd keys with strata below the
    first level: the output is the oracle's, and every level-1 subproblem's
    grouping still meets its lower bound L* >= ceil(W / r)."""
    n = (1 << 24) + 4321
    keys = gen(U64, n, "uniform", 820)
    p = api.make_params(levels=2, k=256, overpartition_b=4, flags=STRAT)
    ws = api.alloc_workspace(api.workspace_bytes(U64, n, False, p))
    log("stratified 2^24+ with stats")
    out = to_host(api.sort_keys(to_dev(keys), params=p, workspace=ws))
    st = api.workspace_stats(ws)
    import oracle
    want, _ = oracle.oracle_sort(U64, keys)
    assert np.array_equal(out, want)
    assert st["levels"] == 2 and st["keys"][1] == n and st["imbalance_max"][1] >= 1.0


# Final children (equality buckets) of a subproblem read from the output
# buffer (the middle level of three, or any level of an in-place sort) go
# through the temporary buffer and a copy leaf: float keys must be decoded
# exactly once on the way to the output.
@pytest.mark.parametrize("kt", [F32, U64])
@pytest.mark.parametrize("dist", ["few", "zipf", "specials"])
@pytest.mark.parametrize("levels,k,b", [(3, 16, 2), (3, 64, 1)])
def test_final_children_through_temp(api, kt, dist, levels, k, b):
    n = 400_003
    keys = gen(kt, n, dist, 860)
    p = api.make_params(levels=levels, k=k, overpartition_b=b)
    log("final children via temp kt=%d %s levels=%d k=%d b=%d" % (kt, dist, levels, k, b))
    check_sort_keys(api, kt, keys, params=p, what="%s levels %d" % (dist, levels))


@pytest.mark.parametrize("dist", ["few", "zipf", "specials"])
def test_in_place_float_duplicates(api, dist):
    import oracle
    keys = gen(F32, 300_001, dist, 870)
    d = to_dev(keys)
    log("in place f32 %s" % dist)
    api.sort_keys(d, out=d)
    want, _ = oracle.oracle_sort(F32, keys)
    from gpu_util import assert_same_bits
    assert_same_bits(to_host(d), want, "in place f32 " + dist)
    vals = np.arange(keys.size, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    api.sort_pairs(dk, dv, out_keys=dk, out_vals=dv)
    wk, wv = oracle.oracle_sort(F32, keys, vals)
    assert_same_bits(to_host(dk), wk, "in place f32 pairs " + dist)
    assert np.array_equal(to_host(dv), wv)


def test_sorts_on_concurrent_streams(api):
    """Sorts enqueued on two streams at once (keys of three types, then an
    RLM-sort beside a pairs sort), each with its own workspace, run side by
    side on the device and equal the oracle: no state is shared between
    calls beyond the per-device error word."""
    import torch

    import oracle
    from gpu_util import assert_same_bits
    cases = [(U64, gen(U64, (1 << 22) + 3, "uniform", 901)),
             (F32, gen(F32, (1 << 21) + 5, "few", 902)),
             (U32, gen(U32, 300001, "zipf", 903)),
             (U64, gen(U64, 70001, "sorted", 904))]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ins = [to_dev(k) for _, k in cases]
    wss = [api.alloc_workspace(api.workspace_bytes(kt, k.size, False, None)) for kt, k in cases]
    outs = [torch.empty_like(x) for x in ins]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    log("four sorts on two streams, three rounds")
    for _ in range(3):
        for i, x in enumerate(ins):
            s = streams[i % 2]
            with torch.cuda.stream(s):
                api.sort_keys(x, out=outs[i], workspace=wss[i], stream=s)
    # an RLM-sort and a pairs sort join them, one on each stream
    rk = gen(U64, (1 << 20) + 7, "uniform", 905)
    pk = gen(U32, 200003, "few", 906)
    pv = np.arange(pk.size, dtype=np.uint32)
    d_rk, d_pk, d_pv = to_dev(rk), to_dev(pk), to_dev(pv)
    ws_r = api.alloc_workspace(api.rlm_workspace_bytes(U64, rk.size))
    ws_p = api.alloc_workspace(api.workspace_bytes(U32, pk.size, True, None))
    o_r = torch.empty_like(d_rk)
    o_pk, o_pv = torch.empty_like(d_pk), torch.empty_like(d_pv)
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for _ in range(2):
        with torch.cuda.stream(streams[0]):
            api.rlm_sort_keys(d_rk, out=o_r, workspace=ws_r, stream=streams[0])
        with torch.cuda.stream(streams[1]):
            api.sort_pairs(d_pk, d_pv, out_keys=o_pk, out_vals=o_pv, workspace=ws_p,
                           stream=streams[1])
    for s in streams:
        torch.cuda.current_stream().wait_stream(s)
    for (kt, k), o in zip(cases, outs):
        want, _ = oracle.oracle_sort(kt, k)
        assert_same_bits(to_host(o), want, "kt%d n%d" % (kt, k.size))
    assert_same_bits(to_host(o_r), oracle.oracle_sort(U64, rk)[0], "rlm")
    wk, wv = oracle.oracle_sort(U32, pk, pv)
    assert_same_bits(to_host(o_pk), wk, "pairs keys")
    assert_same_bits(to_host(o_pv), wv, "pairs payload")
