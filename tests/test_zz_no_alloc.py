"""ams_sort_keys_noalloc: the sort with its workspace in the library's fixed
per-device array, called through the C ABI, equals ams_sort_keys bit for bit
on two calls in a row (the second smaller), and rejects sizes whose
workspace exceeds the array (GPU)."""

import ctypes

import numpy as np
import pytest

from gpu_util import gen, log, to_dev, to_host
from paper_1410_6754_amd import _lib as L
from paper_1410_6754_amd import workloads as W

pytestmark = pytest.mark.gpu


def noalloc(kt, d_in, d_out, params=None):
    import torch
    s = torch.cuda.current_stream().cuda_stream
    return L.lib().ams_sort_keys_noalloc(kt, d_in.data_ptr(), d_out.data_ptr(), d_in.numel(), s,
                                         ctypes.byref(params) if params is not None else None)


def reference(kt, d_in):
    import torch
    from paper_1410_6754_amd import api
    out = torch.empty_like(d_in)
    L.check(L.lib().ams_sort_keys(kt, d_in.data_ptr(), out.data_ptr(), d_in.numel(), None, 0,
                                  torch.cuda.current_stream().cuda_stream, None))
    return out


@pytest.mark.parametrize("kt,sizes", [(W.KEY_U64, [4_000_000, 300_001]),
                                      (W.KEY_U32, [7_000_000, 65_537]),
                                      (W.KEY_F32, [1_000_003, 8_000])])
def test_noalloc_equals_sort_keys_twice(kt, sizes):
    import torch
    for i, n in enumerate(sizes):
        keys = gen(kt, n, "uniform" if i == 0 else "few", 600 + i)
        d = to_dev(keys)
        out = torch.empty_like(d)
        log("noalloc kt=%d n=%d (call %d)" % (kt, n, i + 1))
        L.check(noalloc(kt, d, out))
        want = to_host(reference(kt, d))
        got = to_host(out)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (kt, n)


def test_noalloc_rejects_oversized_input():
    import torch
    from paper_1410_6754_amd import api
    n = 5_000_000  # needs more workspace than the fixed array holds
    assert api.workspace_bytes(W.KEY_U64, n) > L.lib().ams_workspace_bytes(W.KEY_U64, 4_000_000,
                                                                            0, None)
    d = torch.zeros(n, dtype=torch.uint64, device="cuda")
    out = torch.empty_like(d)
    st = noalloc(W.KEY_U64, d, out)
    assert st == L.AMS_EUNSUPPORTED
    assert b"fixed array" in L.lib().ams_last_error()
    # a valid call afterwards still works
    keys = gen(W.KEY_U64, 100_000, "uniform", 610)
    d = to_dev(keys)
    out = torch.empty_like(d)
    L.check(noalloc(W.KEY_U64, d, out))
    assert np.array_equal(to_host(out), np.sort(keys))
