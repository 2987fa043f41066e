"""GPU tests of the serving loop: every result equals the oracle and sorting
the request alone (tolerance 0), admission by the memory budget, queue
limits, poll/wait/release semantics."""

import time

import numpy as np
import pytest

import oracle
from gpu_util import gen, log, to_dev, to_host
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1410_6754_amd import api as A
    return A


def test_mixed_stream_results_match_oracle_and_alone(api):
    from paper_1410_6754_amd.server import Server
    rng = np.random.default_rng(81)
    arrivals, sizes, kts = W.serving_stream(60, rng, rate_per_s=1e4, lo_exp=4, hi_exp=18)
    reqs = []
    with Server(streams=3) as srv:
        for i, (n, kt) in enumerate(zip(sizes, kts)):
            keys = gen(int(kt), int(n), "uniform", 100 + i)
            vals = np.arange(n, dtype=np.uint32) if i % 4 == 0 else None
            dk = to_dev(keys)
            dv = to_dev(vals) if vals is not None else None
            t = srv.submit(dk, dv)
            reqs.append((t, int(kt), keys, vals))
        log("submitted %d requests" % len(reqs))
        batches = set()
        for t, kt, keys, vals in reqs:
            st = srv.wait(t)
            assert st["status"] == 0
            batches.add(st["batch_id"])
            res = srv.result(t)
            if vals is None:
                got = to_host(res)
                want, _ = oracle.oracle_sort(kt, keys)
                assert np.array_equal(got.view(np.uint8), want.view(np.uint8))
                alone = to_host(api.sort_keys(to_dev(keys)))
                assert np.array_equal(got.view(np.uint8), alone.view(np.uint8))
            else:
                gk, gv = to_host(res[0]), to_host(res[1])
                wk, wv = oracle.oracle_sort(kt, keys, vals)
                assert np.array_equal(gk.view(np.uint8), wk.view(np.uint8))
                assert np.array_equal(gv, wv)
            srv.release(t)
        log("ran in %d batches" % len(batches))
        assert len(batches) < len(reqs)  # requests were batched together


def test_admission_and_limits(api):
    from paper_1410_6754_amd import AmsError
    from paper_1410_6754_amd.server import Server
    keys = to_dev(gen(W.KEY_U64, 1 << 20, "uniform", 5))
    with Server(budget=4 << 20, max_pending=2, streams=1) as srv:
        with pytest.raises(AmsError) as e:
            srv.submit(keys)  # needs far more than 4 MiB: can never fit
        assert e.value.status == -2
        small = to_dev(gen(W.KEY_U64, 1000, "uniform", 6))
        t1 = srv.submit(small)
        t2 = srv.submit(small)
        try:
            srv.submit(small)
        except AmsError as err:
            assert err.status == -4  # queue full while both are outstanding
        for t in (t1, t2):
            srv.wait(t)
            done, st = srv.poll(t)
            assert done and st["n"] == 1000
            srv.release(t)
        with pytest.raises(AmsError):
            srv.poll(t1)  # released tickets are forgotten


def test_memory_budget_serialises_but_completes(api):
    from paper_1410_6754_amd.server import Server
    n = 1 << 18
    need = api.workspace_bytes(W.KEY_U64, n) + n * 8
    reqs = []
    with Server(budget=int(need * 1.5), streams=2) as srv:
        for i in range(6):
            keys = gen(W.KEY_U64, n, "uniform", 200 + i)
            reqs.append((srv.submit(to_dev(keys)), keys))
        for t, keys in reqs:
            st = srv.wait(t)
            want, _ = oracle.oracle_sort(W.KEY_U64, keys)
            assert np.array_equal(to_host(srv.result(t)), want)
            srv.release(t)


def test_concurrent_submit_poll_release(api):
    """Several host threads submit, poll, wait and release while the
    scheduler launches batches with its lock released: every result equals
    the oracle, and nothing is lost or answered twice."""
    import threading
    from paper_1410_6754_amd.server import Server
    errors = []

    def client(srv, cid):
        try:
            rng = np.random.default_rng([W.BASE_SEED, 300 + cid])
            mine = []
            for j in range(12):
                n = int(2 ** rng.uniform(6, 16))
                kt = [W.KEY_U64, W.KEY_U32, W.KEY_F32][j % 3]
                keys = gen(kt, n, "uniform", 1000 * cid + j)
                mine.append((srv.submit(to_dev(keys)), kt, keys))
                srv.poll(mine[-1][0])
            for t, kt, keys in mine:
                srv.wait(t)
                want, _ = oracle.oracle_sort(kt, keys)
                got = to_host(srv.result(t))
                if not np.array_equal(got.view(np.uint32) if got.dtype == np.float32 else got,
                                      want.view(np.uint32) if want.dtype == np.float32 else want):
                    errors.append("client %d: wrong result for %d keys" % (cid, keys.size))
                srv.release(t)
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append("client %d: %r" % (cid, e))

    with Server(streams=2) as srv:
        threads = [threading.Thread(target=client, args=(srv, c)) for c in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(120)
        assert not any(th.is_alive() for th in threads), "a client did not finish"
    assert not errors, errors
