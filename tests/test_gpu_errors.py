"""Device-side errors reach the caller, run statistics, and the serving loop
keeps serving after a failed batch (GPU)."""

import numpy as np
import pytest

import oracle
from gpu_util import gen, log, to_dev, to_host
from paper_1410_6754_amd import workloads as W
from paper_1410_6754_amd import _lib as L

pytestmark = pytest.mark.gpu

U64 = W.KEY_U64


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def test_tiny_table_raises_device_error(api):
    """A leaf list of one entry cannot hold the leaves of a one-level sort:
    the kernels skip the writes, stay in bounds and raise AMS_DEVERR_TABLE;
    the checked call returns AMS_EDEVICE and the device word keeps the bit
    until cleared."""
    from paper_1410_6754_amd import AmsError
    keys = gen(U64, 100_000, "uniform", 501)
    d = to_dev(keys)
    log("tiny leaf table, checked call")
    assert api.device_errors(clear=True) == 0
    p = api.make_params(flags=L.AMS_FLAG_TEST_TINY_TABLES | L.AMS_FLAG_CHECK)
    with pytest.raises(AmsError) as e:
        api.sort_keys(d, params=p)
    assert e.value.status == L.AMS_EDEVICE
    bits = api.device_errors(clear=True)
    assert bits & L.AMS_DEVERR_TABLE
    # unchecked call with a caller workspace: returns OK, the run's counters
    # and the device word both carry the error
    log("tiny leaf table, unchecked call with workspace")
    p = api.make_params(flags=L.AMS_FLAG_TEST_TINY_TABLES)
    ws = api.alloc_workspace(api.workspace_bytes(U64, keys.size, False, p))
    api.sort_keys(d, params=p, workspace=ws)
    st = api.workspace_stats(ws)
    assert st["device_errors"] & L.AMS_DEVERR_TABLE
    assert api.device_errors(clear=True) & L.AMS_DEVERR_TABLE
    assert api.device_errors(clear=True) == 0
    # the next normal call is unaffected
    p = api.make_params(flags=L.AMS_FLAG_CHECK)
    out = to_host(api.sort_keys(d, params=p))
    want, _ = oracle.oracle_sort(U64, keys)
    assert np.array_equal(out, want)


def test_checked_calls_pass_on_valid_sorts(api):
    p = api.make_params(flags=L.AMS_FLAG_CHECK)
    for kt, n, dist in [(U64, 300_001, "uniform"), (W.KEY_U32, 70_000, "few"),
                        (W.KEY_F32, 20_000, "specials")]:
        keys = gen(kt, n, dist, 502)
        log("checked kt=%d n=%d %s" % (kt, n, dist))
        out = to_host(api.sort_keys(to_dev(keys), params=p))
        want, _ = oracle.oracle_sort(kt, keys)
        assert np.array_equal(out.view(np.uint8), want.view(np.uint8))


def test_run_stats_account_for_every_key(api):
    n = (1 << 22) + 12345
    keys = gen(U64, n, "uniform", 503)
    p = api.make_params(levels=2, k=64, overpartition_b=4)
    ws = api.alloc_workspace(api.workspace_bytes(U64, n, False, p))
    log("stats of a two-level uniform sort n=%d" % n)
    out = to_host(api.sort_keys(to_dev(keys), params=p, workspace=ws))
    st = api.workspace_stats(ws)
    assert st["device_errors"] == 0 and st["levels"] == 2
    assert st["subproblems"][0] == 1 and st["keys"][0] == n
    assert st["keys"][1] <= n and st["subproblems"][1] >= 1
    assert st["final_keys"] == [0, 0, 0, 0]
    assert st["leaf_keys"] + st["copy_keys"] + st["big_keys"] == n
    # L* is at least the average load of the grouping (Section 6)
    assert st["imbalance_max"][0] >= 1.0 and st["imbalance_mean"][0] >= 1.0
    assert st["max_child"][0] >= n // 64
    want, _ = oracle.oracle_sort(U64, keys)
    assert np.array_equal(out, want)


def test_run_stats_all_equal_pairs(api):
    """All keys equal: one final child holds every key after the first level
    (Appendix D), and later passes see none of them."""
    n = 1 << 20
    keys = gen(U64, n, "equal", 504)
    vals = np.arange(n, dtype=np.uint32)
    ws = api.alloc_workspace(api.workspace_bytes(U64, n, True, None))
    log("stats of all-equal pairs n=%d" % n)
    ok, ov = api.sort_pairs(to_dev(keys), to_dev(vals), workspace=ws)
    st = api.workspace_stats(ws)
    assert st["keys"][0] == n and st["final_keys"][0] == n
    assert st["keys"][1] == 0 and st["leaf_keys"] == 0 and st["big_keys"] == 0
    assert np.array_equal(to_host(ok), keys) and np.array_equal(to_host(ov), vals)


def test_server_keeps_serving_after_injected_failure(api):
    from paper_1410_6754_amd import AmsError
    from paper_1410_6754_amd.server import Server
    with Server(streams=1) as srv:
        srv.inject_alloc_failures(1)
        keys = gen(U64, 50_000, "uniform", 505)
        dk = to_dev(keys)
        t1 = srv.submit(dk)
        log("injected failure: waiting for the failed request")
        with pytest.raises(AmsError) as e:
            srv.wait(t1)
        assert e.value.status == L.AMS_ENOMEM
        done, st = srv.poll(t1)
        assert done and st["status"] == L.AMS_ENOMEM
        srv.release(t1)
        t2 = srv.submit(dk)
        st = srv.wait(t2)
        assert st["status"] == 0
        want, _ = oracle.oracle_sort(U64, keys)
        assert np.array_equal(to_host(srv.result(t2)), want)
        srv.release(t2)
