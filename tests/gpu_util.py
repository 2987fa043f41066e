"""Helpers shared by the GPU parity tests: move seeded inputs to the device,
run the library, compare with the oracle bit for bit."""

import sys

import numpy as np

import oracle
from oracle import checkers
from paper_1410_6754_amd import workloads as W


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    return torch


def to_dev(a: np.ndarray):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bits(a: np.ndarray):
    return a.view(np.uint32) if a.dtype == np.float32 else a


def assert_same_bits(got: np.ndarray, want: np.ndarray, what=""):
    g, w = bits(got), bits(want)
    if not np.array_equal(g, w):
        bad = np.nonzero(g != w)[0]
        raise AssertionError("%s: %d of %d differ, first at %d: got %r want %r"
                             % (what, bad.size, g.size, bad[0], g[bad[0]], w[bad[0]]))


def gen(key_type, n, dist, seed):
    rng = np.random.default_rng([W.BASE_SEED, seed])
    return W.keys(key_type, n, rng, dist)


def check_sort_keys(api, key_type, keys, params=None, what=""):
    out = to_host(api.sort_keys(to_dev(keys), params=params))
    want, _ = oracle.oracle_sort(key_type, keys)
    assert_same_bits(out, want, what)
    return out


def check_sort_pairs(api, key_type, keys, params=None, what=""):
    vals = np.arange(keys.size, dtype=np.uint32)
    ok, ov = api.sort_pairs(to_dev(keys), to_dev(vals), params=params)
    ok, ov = to_host(ok), to_host(ov)
    wk, wv = oracle.oracle_sort(key_type, keys, vals)
    assert_same_bits(ok, wk, what + " keys")
    assert_same_bits(ov, wv, what + " payload")
    assert checkers.check_pairs(key_type, keys, ok, ov) is None
