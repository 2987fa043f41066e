"""A sort recorded once in a HIP graph (torch.cuda.graph, the caller's
workspace, no allocation or host round trip inside the call) and replayed
with new keys each time: every replay equals the oracle's sort of the keys
it read, with eager work and synchronisations between the replays."""

import time

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_bits, gen, log, to_dev, to_host
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kt,n,pairs", [(W.KEY_U64, 65537, False), (W.KEY_F32, 300001, False),
                                        (W.KEY_U32, 20011, True)])
def test_sort_replayed_from_a_graph(kt, n, pairs):
    import torch
    from paper_1410_6754_amd import api
    keys = to_dev(gen(kt, n, "uniform", 950))
    vals = to_dev(np.arange(n, dtype=np.uint32)) if pairs else None
    ws = api.alloc_workspace(api.workspace_bytes(kt, n, pairs, None))
    out = torch.empty_like(keys)
    ov = torch.empty_like(vals) if pairs else None

    def call():
        if pairs:
            api.sort_pairs(keys, vals, out_keys=out, out_vals=ov, workspace=ws)
        else:
            api.sort_keys(keys, out=out, workspace=ws)

    call()  # eager first call: kernel attributes are set outside the capture
    torch.cuda.synchronize()
    log("capturing kt=%d n=%d pairs=%s" % (kt, n, pairs))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    for r in range(4):
        h = gen(kt, n, ["uniform", "few", "zipf", "reversed"][r], 951 + r)
        keys.copy_(to_dev(h))
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if pairs:
            wk, wv = oracle.oracle_sort(kt, h, np.arange(n, dtype=np.uint32))
            assert_same_bits(to_host(out), wk, "replay %d keys" % r)
            assert_same_bits(to_host(ov), wv, "replay %d payload" % r)
        else:
            assert_same_bits(to_host(out), oracle.oracle_sort(kt, h)[0], "replay %d" % r)
    # launch cost: eager calls against graph replays of the same sort
    reps = 50
    for label, fn in (("eager", call), ("graph", g.replay)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        log("%s: %.1f us per sort" % (label, (time.perf_counter() - t0) / reps * 1e6))
