"""Full-size parity: the benchmark's own workloads and plans, element by
element against the oracle (its parallel mergesort on the host's cores).

* 2^28 uniform uint64 keys with the benchmark's plan (two levels, k = 256,
  b = 4, 64 Ki-key tiles), and the same keys sorted and reversed: one
  multiset, so the oracle's output is the expected result of all three;
* 2^27 (uint64 key, uint32 index) pairs: 2^10 distinct values, Zipf(1.1)
  and all-equal keys, with the default plan;
* 2^20 uniform uint64 keys with one level, k = 256, b = 1, a = 16 and
  base-case cutoff 1024;
* the batches of 2227 and of 20,000 log-uniform segments (2^28 and about
  2^31.2 keys in all), with the built-in and with the autotuned
  parameters, every segment against the oracle's sort of that segment;
* the serving workload's 1000 requests (mixed uint64, uint32 and float32
  keys, 1.79e9 in all) queued at once into the server, every result
  against the oracle's sort of its request;
* the largest accepted input, AMS_MAX_SEGMENT = 2^32 - 2^20 keys (uint32
  and uint64 keys, the same patterns as float32 under totalOrder, uint32
  pairs, RLM-sort), and a batch of 5.4e9 keys whose
  first segment has that size: each segment a permutation of 0..n-1, so
  the sorted output is known without a host sort (the property holds at
  any size: output[j] = j, and the payload of key j is its input
  position).
Inputs come from the same seeded generators and parameters as bench.py.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import bench
import oracle
from gpu_util import assert_same_bits, log, to_dev
from oracle import checkers
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu


def threads():
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def workload(name):
    n, kt, dist, pay, params, cfg = bench.WORKLOADS[name]
    return n, kt, dist, pay, params, cfg


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def u64_2p28():
    """The default workload's keys and the oracle's sorted output."""
    n, kt, dist, _, _, cfg = workload("uniform_u64_2^28")
    keys = W.keys(kt, n, W.rng_for(cfg), dist)
    log("oracle: 2^28 uint64 keys on %d threads" % threads())
    perm = oracle.oracle_sort_perm_parallel(kt, keys, threads())
    return keys, keys[perm.astype(np.int64)]


def run_keys(api, name, keys):
    n, kt, _, _, params, _ = workload(name)
    p = api.make_params(**params)
    ws = api.alloc_workspace(api.workspace_bytes(kt, n, False, p))
    d = to_dev(keys)
    out = api.sort_keys(d, params=p, workspace=ws)
    st = api.workspace_stats(ws)
    got = host(out)
    del d, out, ws
    return got, st


@pytest.mark.parametrize("name", ["uniform_u64_2^28", "sorted_u64_2^28", "reversed_u64_2^28"])
def test_bench_plan_2p28(api, u64_2p28, name):
    keys, want = u64_2p28
    if name.startswith("sorted"):
        keys = want  # the unique sorted order of the same keys
    elif name.startswith("reversed"):
        keys = want[::-1].copy()
    log("%s on the GPU" % name)
    got, st = run_keys(api, name, keys)
    # the plan the benchmark times: two levels of 1024 buckets, 64 Ki tiles
    assert st["levels"] == 2 and st["device_errors"] == 0
    assert st["tiles"][0] == (1 << 28) // 65536
    assert st["keys"][0] == 1 << 28 and st["keys"][1] == 1 << 28
    assert st["leaf_keys"] + st["copy_keys"] + st["big_keys"] == 1 << 28
    assert_same_bits(got, want, name)
    assert checkers.check_keys(W.KEY_U64, keys, got) is None


@pytest.mark.parametrize("name", ["pairs_few_2^27", "pairs_zipf_2^27", "pairs_equal_2^27"])
def test_bench_plan_pairs_2p27(api, name):
    n, kt, dist, pay, params, cfg = workload(name)
    assert pay
    keys = W.keys(kt, n, W.rng_for(cfg), dist)
    vals = np.arange(n, dtype=np.uint32)
    log("%s: oracle on %d threads" % (name, threads()))
    perm = oracle.oracle_sort_perm_parallel(kt, keys, threads()).astype(np.int64)
    log("%s on the GPU" % name)
    p = api.make_params(**params)
    ws = api.alloc_workspace(api.workspace_bytes(kt, n, True, p))
    ok, ov = api.sort_pairs(to_dev(keys), to_dev(vals), params=p, workspace=ws)
    st = api.workspace_stats(ws)
    gk, gv = host(ok), host(ov)
    assert st["device_errors"] == 0
    assert_same_bits(gk, keys[perm], name + " keys")
    assert_same_bits(gv, perm.astype(np.uint32), name + " payload")
    assert checkers.check_pairs(kt, keys, gk, gv) is None


def test_bench_plan_config1(api):
    name = "uniform_u64_2^20"
    n, kt, dist, _, params, cfg = workload(name)
    assert params == dict(levels=1, k=256, overpartition_b=1, samples_per_bucket=16,
                          base_cutoff=1024)
    keys = W.keys(kt, n, W.rng_for(cfg), dist)
    want, _ = oracle.oracle_sort(kt, keys)
    log("%s on the GPU" % name)
    got, st = run_keys(api, name, keys)
    assert st["levels"] == 1 and st["subproblems"][0] == 1 and st["subproblems"][1] == 0
    assert st["leaf_keys"] + st["big_keys"] == n
    assert_same_bits(got, want, name)


def test_rlm_2p28_matches_oracle(api, u64_2p28):
    """RLM-sort (Section 5) of the default workload's keys: the same unique
    sorted output."""
    keys, want = u64_2p28
    n, kt, dist, pkw, cfg = bench.RLM_WORKLOADS["rlm_uniform_u64_2^28"]
    p = api.rlm_params(**pkw)
    ws = api.alloc_workspace(api.rlm_workspace_bytes(kt, n, p))
    log("rlm_uniform_u64_2^28 on the GPU")
    d = to_dev(keys)
    got = host(api.rlm_sort_keys(d, params=p, workspace=ws))
    assert_same_bits(got, want, "rlm 2^28")


def test_rlm_2p20_matches_oracle(api):
    n, kt, dist, pkw, cfg = bench.RLM_WORKLOADS["rlm_uniform_u64_2^20"]
    keys = W.keys(kt, n, W.rng_for(cfg), dist)
    want, _ = oracle.oracle_sort(kt, keys)
    got = host(api.rlm_sort_keys(to_dev(keys), params=api.rlm_params(**pkw)))
    assert_same_bits(got, want, "rlm 2^20")


@pytest.mark.parametrize("dist", ["zipf", "few", "sorted", "equal"])
def test_rlm_2p24_skewed_matches_oracle(api, dist):
    """RLM-sort of 2^24 + odd uint64 keys at four levels' depth (tiles of 4096,
    r = 16) on skewed inputs: Zipf(1.1), 2^10 distinct values, sorted and
    all equal. The first round's pivots assume tiles of the same mix; here
    they do not, and only the number of selection rounds may change."""
    n = (1 << 24) + 4097
    keys = W.keys(W.KEY_U64, n, W.rng_for(30), dist)
    log("oracle: rlm %s 2^24+ on %d threads" % (dist, threads()))
    perm = oracle.oracle_sort_perm_parallel(W.KEY_U64, keys, threads())
    want = keys[perm.astype(np.int64)]
    log("rlm %s 2^24+ on the GPU" % dist)
    got = host(api.rlm_sort_keys(to_dev(keys)))
    assert_same_bits(got, want, "rlm " + dist)


def test_bench_batch_2p28(api):
    import torch
    # the batch workload exactly as bench.py draws it: 20,000 log-uniform
    # sizes, the leading ones up to 2^28 keys in all, then the keys
    rng = W.rng_for(bench.SPECIAL["batch_2^28"])
    sizes = W.truncate_total(W.batch_sizes(20000, rng, 8, 20), 1 << 28)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(offs[-1])
    keys = W.uniform_u64(total, rng)
    assert sizes.size == 2227 and total > (1 << 28) - (1 << 20)
    log("batch_2^28: oracle over %d segments on %d threads" % (sizes.size, threads()))
    want = np.empty_like(keys)

    def one(i):
        a, b = int(offs[i]), int(offs[i + 1])
        want[a:b] = oracle.oracle_sort(W.KEY_U64, keys[a:b])[0]

    with ThreadPoolExecutor(threads()) as ex:
        list(ex.map(one, range(sizes.size)))
    d_keys = to_dev(keys)
    d_offs = torch.from_numpy(offs.astype(np.int64)).cuda()
    try:
        tuned, _ = api.autotune(d_keys, offs, max_trials=16)
        for label, params in (("built-in", None), ("autotuned", tuned)):
            log("batch_2^28 on the GPU, %s parameters" % label)
            ws = api.alloc_workspace(api.batch_workspace_bytes(W.KEY_U64, offs, params=params))
            out = api.sort_batch(d_keys, offs, d_offsets=d_offs, params=params, workspace=ws)
            st = api.workspace_stats(ws)
            got = host(out)
            del out, ws
            assert st["device_errors"] == 0
            assert_same_bits(got, want, "batch_2^28 " + label)
    finally:
        api.autotune_clear()  # later tests of this process use the built-in choice


def test_bench_batch_20000(api):
    import psutil
    import torch
    # configuration 4 as stated: 20,000 log-uniform segments, about 2^31.2
    # keys (20 GB); the host holds the keys and the sorted output, and the
    # oracle sorts one segment at a time beside the comparison
    if psutil.virtual_memory().available < (64 << 30):
        pytest.skip("needs about 48 GB of free host memory")
    rng = W.rng_for(bench.SPECIAL["batch_20000"])
    sizes = W.batch_sizes(20000, rng, 8, 20)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(offs[-1])
    log("batch_20000: %d keys; generating" % total)
    keys = W.uniform_u64(total, rng)
    d_keys = to_dev(keys)
    d_offs = torch.from_numpy(offs.astype(np.int64)).cuda()
    bad = []

    def check(got, label):
        def one(i):
            a, b = int(offs[i]), int(offs[i + 1])
            want = oracle.oracle_sort(W.KEY_U64, keys[a:b])[0]
            if not np.array_equal(got[a:b], want):
                bad.append((label, i))

        with ThreadPoolExecutor(threads()) as ex:
            list(ex.map(one, range(sizes.size)))

    try:
        tuned, _ = api.autotune(d_keys, offs, max_trials=16)
        for label, params in (("built-in", None), ("autotuned", tuned)):
            log("batch_20000 on the GPU, %s parameters" % label)
            ws = api.alloc_workspace(api.batch_workspace_bytes(W.KEY_U64, offs, params=params))
            out = api.sort_batch(d_keys, offs, d_offsets=d_offs, params=params, workspace=ws)
            st = api.workspace_stats(ws)
            got = host(out)
            del out, ws
            assert st["device_errors"] == 0
            log("batch_20000: oracle over %d segments on %d threads" % (sizes.size, threads()))
            check(got, label)
            del got
            assert not bad, bad[:10]
    finally:
        api.autotune_clear()


def test_bench_serving_requests(api):
    from paper_1410_6754_amd.server import Server
    # the serving workload's requests exactly as bench.py draws them, all
    # queued at once (its closed-loop pass); each result against the oracle
    rng = W.rng_for(bench.SPECIAL["serving"])
    nreq = 1000
    _, sizes, kts = W.serving_stream(nreq, rng, 1.0, 10, 24)
    log("serving: %d requests, %d keys; generating" % (nreq, int(sizes.sum())))
    keys = [W.keys(int(kt), int(n), rng, "uniform") for n, kt in zip(sizes, kts)]
    reqs = [to_dev(k) for k in keys]
    bad = []

    def check(i, got):
        want = oracle.oracle_sort(int(kts[i]), keys[i])[0]
        if not np.array_equal(got.view(np.uint8), want.view(np.uint8)):
            bad.append(i)

    with ThreadPoolExecutor(threads()) as ex, Server(streams=2, max_pending=nreq + 8) as srv:
        tickets = [srv.submit(r) for r in reqs]
        jobs = []
        for i, tk in enumerate(tickets):
            st = srv.wait(tk)
            assert st["status"] == 0, (i, st)
            got = host(srv.result(tk))
            srv.release(tk)
            jobs.append(ex.submit(check, i, got))
        for j in jobs:
            j.result()
    assert not bad, bad[:10]


MAX_SEGMENT = (1 << 32) - (1 << 20)
PERM_A = 0x9E3779B1  # coprime to MAX_SEGMENT = 2^20 * 3^2 * 5 * 7 * 13


def _fill_permutation(out, n, a, wide):
    """out[i] = i * a mod n with gcd(a, n) = 1 (out: an int32 or int64 view of
    n keys): a permutation of 0..n-1, built on the device in chunks."""
    import torch
    step = 1 << 26
    for s0 in range(0, n, step):
        i = torch.arange(s0, min(s0 + step, n), dtype=torch.int64, device=out.device)
        v = _mulmod(i, a, n)
        if not wide:
            v = torch.where(v >= (1 << 31), v - (1 << 32), v).to(torch.int32)
        out[s0:s0 + v.numel()] = v


def _permutation_keys(n, wide):
    import torch
    out = torch.empty(n, dtype=torch.int64 if wide else torch.int32, device="cuda")
    _fill_permutation(out, n, PERM_A, wide)
    return out.view(torch.uint64 if wide else torch.uint32)


def _mulmod(i, a, n):
    """i * a mod n for int64 tensors i < 2^32 and a < 2^32 (no product above 2^49)."""
    return ((i * (a >> 16)) % n * 65536 + i * (a & 0xFFFF)) % n


def _first_not_identity(out, n, wide):
    import torch
    step = 1 << 26
    for s0 in range(0, n, step):
        e = min(s0 + step, n)
        g = out[s0:e].view(torch.int64 if wide else torch.int32).to(torch.int64)
        if not wide:
            g = g & 0xFFFFFFFF
        want = torch.arange(s0, e, dtype=torch.int64, device=out.device)
        if not torch.equal(g, want):
            return s0 + int(torch.nonzero(g != want)[0])
    return None


@pytest.mark.parametrize("inplace", [False, True])
def test_max_segment_float_bits(api, inplace):
    import torch
    # the same permutation of 0..n-1 read as float32 bit patterns: every
    # positive pattern (+0 .. +NaN) and the negative ones from 0x80000000 (-0)
    # to 0xFFEFFFFF (a negative NaN).  IEEE 754 totalOrder puts the negative
    # patterns first, the largest pattern first, then the positive ones.
    n = MAX_SEGMENT
    log("max segment: %d float32 bit patterns; building the permutation" % n)
    keys = _permutation_keys(n, False).view(torch.float32)
    ws = api.alloc_workspace(api.workspace_bytes(W.KEY_F32, n, False, None))
    out = api.sort_keys(keys, out=keys if inplace else None, workspace=ws)
    st = api.workspace_stats(ws)
    assert st["device_errors"] == 0
    del keys, ws
    neg = n - (1 << 31)  # patterns 0x80000000 .. n-1
    step = 1 << 26
    for s0 in range(0, n, step):
        e = min(s0 + step, n)
        j = torch.arange(s0, e, dtype=torch.int64, device="cuda")
        want = torch.where(j < neg, (n - 1) - j, j - neg)
        g = out[s0:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(g, want), "float bits in [%d, %d)" % (s0, e)
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kt,inplace", [(W.KEY_U32, False), (W.KEY_U64, False), (W.KEY_U64, True)])
def test_max_segment(api, kt, inplace):
    import torch
    n = MAX_SEGMENT
    wide = kt == W.KEY_U64
    assert api.workspace_bytes(kt, n + 1, False, None) == 0  # one more is refused
    log("max segment: %d %s keys; building the permutation" % (n, "uint64" if wide else "uint32"))
    keys = _permutation_keys(n, wide)
    probe = keys[:4].view(torch.int64 if wide else torch.int32).cpu().tolist()
    assert probe[0] == 0 and probe[1] != 1  # i * a mod n, not the identity
    ws = api.alloc_workspace(api.workspace_bytes(kt, n, False, None))
    log("max segment: sorting%s" % (" in place" if inplace else ""))
    out = api.sort_keys(keys, out=keys if inplace else None, workspace=ws)
    st = api.workspace_stats(ws)
    log("max segment: levels %d, leaves %d, device errors %d"
        % (st["levels"], st["leaves"], st["device_errors"]))
    assert st["device_errors"] == 0
    del keys, ws
    bad = _first_not_identity(out, n, wide)
    assert bad is None, "output[%d] != %d" % (bad, bad)
    del out
    torch.cuda.empty_cache()


def test_max_segment_pairs(api):
    import torch
    n = MAX_SEGMENT
    log("max segment: %d uint32 pairs; building the permutation" % n)
    keys = _permutation_keys(n, False)
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    step = 1 << 26
    for s0 in range(0, n, step):
        v = torch.arange(s0, min(s0 + step, n), dtype=torch.int64, device="cuda")
        vals[s0:s0 + v.numel()] = torch.where(v >= (1 << 31), v - (1 << 32), v).to(torch.int32)
    vals = vals.view(torch.uint32)
    ws = api.alloc_workspace(api.workspace_bytes(W.KEY_U32, n, True, None))
    log("max segment pairs: sorting")
    ok, ov = api.sort_pairs(keys, vals, workspace=ws)
    st = api.workspace_stats(ws)
    assert st["device_errors"] == 0
    del keys, vals, ws
    bad = _first_not_identity(ok, n, False)
    assert bad is None, "keys: output[%d] != %d" % (bad, bad)
    # key j came from input position j * a^-1 mod n
    ainv = pow(PERM_A, -1, n)
    for s0 in range(0, n, step):
        e = min(s0 + step, n)
        j = torch.arange(s0, e, dtype=torch.int64, device="cuda")
        g = ov[s0:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(g, _mulmod(j, ainv, n)), "payload in [%d, %d)" % (s0, e)
    del ok, ov
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kt", [W.KEY_U32, W.KEY_U64])
def test_max_segment_rlm(api, kt):
    import torch
    n = MAX_SEGMENT
    wide = kt == W.KEY_U64
    assert api.rlm_workspace_bytes(kt, n + 1) == 0
    log("max segment RLM-sort: %d %s keys" % (n, "uint64" if wide else "uint32"))
    keys = _permutation_keys(n, wide)
    ws = api.alloc_workspace(api.rlm_workspace_bytes(kt, n))
    out = api.rlm_sort_keys(keys, workspace=ws)
    torch.cuda.synchronize()
    assert api.device_errors() == 0
    del keys, ws
    bad = _first_not_identity(out, n, wide)
    assert bad is None, "output[%d] != %d" % (bad, bad)
    del out
    torch.cuda.empty_cache()


def test_batch_above_2p32_keys(api):
    import math
    import torch
    # segment sizes: the largest accepted one first, so every later segment
    # starts above 2^32 keys into the batch
    sizes = [MAX_SEGMENT, (1 << 30) + 7, 3, 0, 1, (1 << 20) + 1, 4097]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(offs[-1])
    assert total > (1 << 32) + (1 << 30)
    log("batch of %d uint32 keys in %d segments; building the permutations" % (total, len(sizes)))
    keys = torch.empty(total, dtype=torch.int32, device="cuda")
    for i, n in enumerate(sizes):
        if n:
            a = PERM_A
            while math.gcd(a, n) != 1:
                a += 2
            _fill_permutation(keys[int(offs[i]):int(offs[i + 1])], n, a, False)
    keys = keys.view(torch.uint32)
    ws = api.alloc_workspace(api.batch_workspace_bytes(W.KEY_U32, offs))
    log("batch above 2^32 keys: sorting")
    out = api.sort_batch(keys, offs, workspace=ws)
    st = api.workspace_stats(ws)
    assert st["device_errors"] == 0
    del keys, ws
    for i, n in enumerate(sizes):
        bad = _first_not_identity(out[int(offs[i]):int(offs[i + 1])], n, False)
        assert bad is None, "segment %d: output[%d] != %d" % (i, bad, bad)
    del out
    torch.cuda.empty_cache()
