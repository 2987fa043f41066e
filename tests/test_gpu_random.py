"""Seeded random configurations of every sorting entry point, each checked
element by element against the oracle: sort_keys, stable sort_pairs,
in-place sorts, sort_batch with and without payload, and RLM-sort; random
key type, input distribution, size (log-uniform up to 2^20) and plan
parameters (levels, k, b, stratified splitters; RLM ways and tile size).
Paths that only some plans reach (final children through the temporary
buffer, slices over many empty pieces, mixed group widths) are covered
without naming them."""

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_bits, log, to_dev, to_host
from paper_1410_6754_amd import _lib as L
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu

KTS = [W.KEY_U64, W.KEY_U32, W.KEY_F32]
DISTS = ["uniform", "few", "zipf", "equal", "sorted", "reversed", "specials"]
MODES = ["keys", "pairs", "inplace", "batch", "batchpairs", "rlm"]
PER_SEED = 100


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def oracle_segments(kt, keys, offs, vals=None):
    wk = np.empty_like(keys)
    wv = None if vals is None else np.empty_like(vals)
    for a, b in zip(offs[:-1].astype(np.int64), offs[1:].astype(np.int64)):
        k, v = oracle.oracle_sort(kt, keys[a:b], None if vals is None else vals[a:b])
        wk[a:b] = k
        if vals is not None:
            wv[a:b] = v
    return wk, wv


def run_one(api, rng, idx):
    kt = KTS[rng.integers(0, len(KTS))]
    dist = DISTS[rng.integers(0, len(DISTS))]
    mode = MODES[rng.integers(0, len(MODES))]
    n = int(np.exp(rng.uniform(0, np.log(1 << 20))))
    keys = W.keys(kt, n, np.random.default_rng([W.BASE_SEED, 1000 + idx]), dist)
    vals = rng.integers(0, 1 << 32, n, dtype=np.uint32)
    if mode == "rlm":
        ways = int(rng.choice([2, 3, 4, 8, 16, 16, 32, 64]))
        tile = int(rng.choice([64, 256, 1024, 4096, 4096]))
        p = api.rlm_params(ways=ways, tile_keys=tile, seed=int(rng.integers(1, 1 << 30)))
        what = "#%d rlm ways=%d tile=%d kt=%d %s n=%d" % (idx, ways, tile, kt, dist, n)
        log(what)
        try:
            got = to_host(api.rlm_sort_keys(to_dev(keys), params=p))
        except L.AmsError as e:
            assert e.status == L.AMS_EUNSUPPORTED, what  # more levels than supported
            return
        assert_same_bits(got, oracle.oracle_sort(kt, keys)[0], what)
        return
    levels = int(rng.integers(0, 4))
    kw = {}
    if levels:
        kw = dict(levels=levels, k=int(rng.choice([16, 64, 256])),
                  overpartition_b=int(rng.choice([1, 2, 4])), flags=int(rng.choice([0, 0, 32])),
                  seed=int(rng.integers(1, 1 << 30)))
    p = api.make_params(**kw)
    what = "#%d %s %s kt=%d %s n=%d" % (idx, mode, kw, kt, dist, n)
    log(what)
    if mode == "keys":
        assert_same_bits(to_host(api.sort_keys(to_dev(keys), params=p)),
                         oracle.oracle_sort(kt, keys)[0], what)
    elif mode == "inplace":
        d = to_dev(keys)
        api.sort_keys(d, out=d, params=p)
        assert_same_bits(to_host(d), oracle.oracle_sort(kt, keys)[0], what)
    elif mode == "pairs":
        gk, gv = api.sort_pairs(to_dev(keys), to_dev(vals), params=p)
        wk, wv = oracle.oracle_sort(kt, keys, vals)
        assert_same_bits(to_host(gk), wk, what)
        assert np.array_equal(to_host(gv), wv), what
    else:
        nseg = int(rng.integers(1, 200))
        cuts = np.sort(rng.integers(0, n + 1, nseg - 1))
        offs = np.concatenate([[0], cuts, [n]]).astype(np.uint64)
        if mode == "batch":
            got = api.sort_batch(to_dev(keys), offs, params=p)
            assert_same_bits(to_host(got), oracle_segments(kt, keys, offs)[0], what)
        else:
            gk, gv = api.sort_batch(to_dev(keys), offs, vals=to_dev(vals), params=p)
            wk, wv = oracle_segments(kt, keys, offs, vals)
            assert_same_bits(to_host(gk), wk, what)
            assert np.array_equal(to_host(gv), wv), what


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_configurations(api, seed):
    rng = np.random.default_rng([W.BASE_SEED, 77, seed])
    for j in range(PER_SEED):
        run_one(api, rng, seed * PER_SEED + j)
