"""GPU parity of RLM-sort (recurse-last multiway mergesort, Section 5) and of
its multisequence selection step (Section 4.1), through the C ABI, against
the oracle: bit for bit."""

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_bits, gen, log, to_dev, to_host
from oracle import rlm as orlm
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu

U32, U64, F32 = W.KEY_U32, W.KEY_U64, W.KEY_F32


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def runs_sorted(kt, keys, run_keys):
    """Keys sorted (by the oracle) inside consecutive runs of run_keys."""
    out = keys.copy()
    for a in range(0, keys.size, run_keys):
        out[a:a + run_keys], _ = oracle.oracle_sort(kt, keys[a:a + run_keys])
    return out


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("n,run_keys,parts,dist", [
    (5000, 100, 7, "uniform"), (5000, 100, 7, "few"), (20000, 64, 16, "equal"),
    (30001, 4096, 5, "uniform"), (100000, 300, 33, "zipf"), (70000, 1000, 2, "sorted"),
    (70000, 1000, 9, "reversed"), (3000, 3000, 1, "uniform"), (1000, 10, 1000, "few")])
def test_step_multiselect_matches_oracle(api, kt, n, run_keys, parts, dist):
    keys = gen(kt, n, dist, 700 + parts)
    runs = runs_sorted(kt, keys, run_keys)
    log("multiselect kt=%d n=%d runs of %d, %d parts, %s" % (kt, n, run_keys, parts, dist))
    got = to_host(api.step_multiselect(to_dev(runs), run_keys, parts))
    ords = oracle.ord_keys(kt, runs)
    seqs = [[int(v) for v in ords[a:a + run_keys]] for a in range(0, n, run_keys)]
    want = np.array(orlm.rlm_splits(seqs, parts), dtype=np.uint32)
    assert got.shape == want.shape
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]


def check_rlm(api, kt, keys, params=None, what=""):
    out = to_host(api.rlm_sort_keys(to_dev(keys), params=params))
    want, _ = oracle.oracle_sort(kt, keys)
    assert_same_bits(out, want, what)


@pytest.mark.parametrize("kt", [U64, U32, F32])
@pytest.mark.parametrize("n", [0, 1, 100, 4096, 4097, 65543, 300001, 1 << 20])
def test_rlm_sizes(api, kt, n):
    log("rlm kt=%d n=%d" % (kt, n))
    check_rlm(api, kt, gen(kt, n, "uniform", 710 + n), what="rlm kt%d n%d" % (kt, n))


@pytest.mark.parametrize("dist", ["few", "zipf", "equal", "sorted", "reversed", "specials"])
def test_rlm_distributions(api, dist):
    log("rlm dist %s" % dist)
    check_rlm(api, U64, gen(U64, 500_000, dist, 720), what="rlm " + dist)
    if dist in ("few", "specials", "equal"):
        check_rlm(api, F32, gen(F32, 200_000, dist, 721), what="rlm f32 " + dist)


@pytest.mark.parametrize("ways,tile", [(2, 4096), (4, 1024), (64, 4096), (16, 64), (3, 512)])
def test_rlm_params(api, ways, tile):
    p = api.rlm_params(ways=ways, tile_keys=tile)
    for dist in ("uniform", "few"):
        log("rlm ways=%d tile=%d %s" % (ways, tile, dist))
        check_rlm(api, U64, gen(U64, 200_003, dist, 730 + ways), params=p,
                  what="rlm ways%d tile%d %s" % (ways, tile, dist))


def test_rlm_in_place_and_checked(api):
    from paper_1410_6754_amd import _lib as L
    keys = gen(U64, 1_000_003, "uniform", 740)
    d = to_dev(keys)
    p = api.rlm_params(flags=L.AMS_FLAG_CHECK)
    api.rlm_sort_keys(d, out=d, params=p)
    want, _ = oracle.oracle_sort(U64, keys)
    assert np.array_equal(to_host(d), want)


def test_rlm_two_levels_large(api):
    n = (1 << 22) + 12345
    log("rlm two+ levels n=%d" % n)
    check_rlm(api, U64, gen(U64, n, "uniform", 750), what="rlm 2^22+")


@pytest.mark.parametrize("n,run_keys,parts", [(20000, 100, 9), (200000, 500, 16)])
def test_step_multiselect_unsorted_runs_stay_in_bounds(api, n, run_keys, parts):
    """Runs that are not sorted break the selection's premise: the cuts are
    unspecified, but every window stays inside its run (a window that would
    invert is emptied and the call may report a device error), and a sorted
    call afterwards is exact.  Covers the workgroup path (200 runs) and the
    count/decide path (400 runs)."""
    from paper_1410_6754_amd import _lib as L
    keys = gen(U64, n, "uniform", 760 + parts)  # not sorted within the runs
    log("multiselect over unsorted runs n=%d runs of %d, %d parts" % (n, run_keys, parts))
    try:
        api.step_multiselect(to_dev(keys), run_keys, parts)
    except L.AmsError as e:
        assert e.status == L.AMS_EDEVICE
    runs = runs_sorted(U64, keys, run_keys)
    got = to_host(api.step_multiselect(to_dev(runs), run_keys, parts))
    ords = oracle.ord_keys(U64, runs)
    seqs = [[int(v) for v in ords[a:a + run_keys]] for a in range(0, n, run_keys)]
    want = np.array(orlm.rlm_splits(seqs, parts), dtype=np.uint32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kt", [U64, U32])
def test_rlm_slice_spanning_many_empty_pieces(api, kt):
    """A slice whose pieces lie far apart in sequence order: tiles of 64 keys,
    the smallest keys in tile 0 (one key) and in tiles 100.., none in tiles
    1..99, so the first part's first slice spans 101 pieces of which 99 are
    empty, more pieces than a tile holds keys (the merge then finds the
    pieces in the global piece offsets and compacts their starts by
    ballots)."""
    rng = np.random.default_rng([W.BASE_SEED, 790 + kt])
    dt = np.uint64 if kt == U64 else np.uint32
    T, n = 64, 64 * 200
    keys = rng.integers(1000, 2000, n).astype(dt)       # large keys everywhere
    small = rng.integers(1, 100, n).astype(dt)
    keys[0] = 0                                         # the smallest key, in tile 0
    keys[100 * T:113 * T] = small[100 * T:113 * T]      # tiles 100..112 all small
    p = api.rlm_params(ways=16, tile_keys=T)
    log("rlm slice over 101 pieces kt=%d" % kt)
    check_rlm(api, kt, keys, params=p, what="rlm many empty pieces")
