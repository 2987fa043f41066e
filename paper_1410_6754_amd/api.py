"""Torch-facing wrappers of the C ABI: argument marshalling only.

Keys are torch tensors on the GPU with dtype uint64, uint32 or float32; the
payload is uint32.  Every call enqueues on the current torch stream (or the
given one) and returns without synchronising.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import AMS_F32, AMS_U32, AMS_U64, Params, check, lib

_DTYPE_TO_KT = {torch.uint64: AMS_U64, torch.uint32: AMS_U32, torch.float32: AMS_F32}
KT_TO_DTYPE = {AMS_U64: torch.uint64, AMS_U32: torch.uint32, AMS_F32: torch.float32}


def key_type_of(t: torch.Tensor) -> int:
    try:
        return _DTYPE_TO_KT[t.dtype]
    except KeyError:
        raise TypeError("keys must be uint64, uint32 or float32, not %s" % t.dtype) from None


def make_params(**kw) -> Params | None:
    """ams_params from keyword arguments (missing fields = automatic)."""
    if not kw:
        return None
    p = Params()
    for k, v in kw.items():
        if v is None:
            continue
        setattr(p, k, int(v))
    return p


def _pref(p: Params | None):
    return ctypes.byref(p) if p is not None else None


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def workspace_bytes(key_type: int, n: int, with_vals: bool = False, params: Params | None = None) -> int:
    return int(lib().ams_workspace_bytes(key_type, n, int(with_vals), _pref(params)))


def batch_workspace_bytes(key_type: int, offsets, with_vals: bool = False,
                          params: Params | None = None) -> int:
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    return int(lib().ams_batch_workspace_bytes(key_type, offs.ctypes.data, offs.size - 1,
                                               int(with_vals), _pref(params)))


def alloc_workspace(nbytes: int, device=None) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


def sort_keys(keys: torch.Tensor, out: torch.Tensor | None = None, params: Params | None = None,
              workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Sorted copy of ``keys`` (``out`` may be ``keys`` itself: in place)."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    if out is None:
        out = torch.empty_like(keys)
    _dev(out, "out")
    if out.numel() != keys.numel() or out.dtype != keys.dtype:
        raise ValueError("out must match keys")
    ws = workspace.data_ptr() if workspace is not None else None
    wsb = workspace.numel() if workspace is not None else 0
    check(lib().ams_sort_keys(kt, keys.data_ptr(), out.data_ptr(), keys.numel(), ws, wsb,
                              _stream(stream), _pref(params)))
    return out


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, out_keys: torch.Tensor | None = None,
               out_vals: torch.Tensor | None = None, params: Params | None = None,
               workspace: torch.Tensor | None = None, stream=None):
    """Stable sort of (key, uint32 payload) pairs."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    _dev(vals, "vals")
    if vals.dtype != torch.uint32 or vals.numel() != keys.numel():
        raise ValueError("vals must be uint32 with one entry per key")
    out_keys = torch.empty_like(keys) if out_keys is None else out_keys
    out_vals = torch.empty_like(vals) if out_vals is None else out_vals
    _dev(out_keys, "out_keys")
    _dev(out_vals, "out_vals")
    ws = workspace.data_ptr() if workspace is not None else None
    wsb = workspace.numel() if workspace is not None else 0
    check(lib().ams_sort_pairs(kt, keys.data_ptr(), vals.data_ptr(), out_keys.data_ptr(),
                               out_vals.data_ptr(), keys.numel(), ws, wsb, _stream(stream),
                               _pref(params)))
    return out_keys, out_vals


def sort_batch(keys: torch.Tensor, offsets, vals: torch.Tensor | None = None,
               out_keys: torch.Tensor | None = None, out_vals: torch.Tensor | None = None,
               d_offsets: torch.Tensor | None = None, params: Params | None = None,
               workspace: torch.Tensor | None = None, stream=None):
    """Sort every segment [offsets[i], offsets[i+1]) of ``keys`` independently."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if offs.size < 1 or int(offs[-1]) != keys.numel():
        raise ValueError("offsets must have num+1 entries ending at len(keys)")
    out_keys = torch.empty_like(keys) if out_keys is None else out_keys
    vp = ovp = None
    if vals is not None:
        _dev(vals, "vals")
        out_vals = torch.empty_like(vals) if out_vals is None else out_vals
        vp, ovp = vals.data_ptr(), out_vals.data_ptr()
    ws = workspace.data_ptr() if workspace is not None else None
    wsb = workspace.numel() if workspace is not None else 0
    dop = d_offsets.data_ptr() if d_offsets is not None else None
    check(lib().ams_sort_batch(kt, keys.data_ptr(), vp, out_keys.data_ptr(), ovp,
                               offs.ctypes.data, dop, offs.size - 1, ws, wsb, _stream(stream),
                               _pref(params)))
    return (out_keys, out_vals) if vals is not None else out_keys


def autotune(keys: torch.Tensor, offsets=None, vals: torch.Tensor | None = None, stream=None,
             max_trials: int = 0):
    """Time candidate parameter sets for sorting ``keys`` (segments given by
    ``offsets``, one segment when None) and return (best Params, ms per sort).
    The choice is also remembered for this shape class (see ams_autotune)."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    if offsets is None:
        offsets = [0, keys.numel()]
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if offs.size < 2 or int(offs[-1]) != keys.numel():
        raise ValueError("offsets must have num+1 entries ending at len(keys)")
    vp = None
    if vals is not None:
        _dev(vals, "vals")
        vp = vals.data_ptr()
    best = Params()
    ms = ctypes.c_double(0.0)
    check(lib().ams_autotune(kt, keys.data_ptr(), vp, offs.ctypes.data, offs.size - 1,
                             _stream(stream), max_trials, ctypes.byref(best), ctypes.byref(ms)))
    return best, ms.value


def autotune_clear():
    """Forget every autotuned choice of this process."""
    lib().ams_autotune_clear()


def params_dict(p: Params | None) -> dict:
    """The fields of an ams_params as a plain dict."""
    if p is None:
        return {}
    return {name: getattr(p, name) for name, _ in Params._fields_}


# ----------------------------------------------------------------------------
# step entry points (one step of the path on one subproblem)
# ----------------------------------------------------------------------------

def step_splitters(keys: torch.Tensor, m: int, a: int, seed: int, stream=None) -> torch.Tensor:
    """The m-1 splitters (as ord values) drawn for ``keys`` at level 0."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    odt = torch.uint64 if kt == AMS_U64 else torch.uint32
    out = torch.empty(m - 1, dtype=odt, device=keys.device)
    check(lib().ams_step_splitters(kt, keys.data_ptr(), keys.numel(), m, a, seed,
                                   out.data_ptr(), _stream(stream)))
    return out


def step_level(keys: torch.Tensor, splitters: torch.Tensor, m: int, r: int, flags: int = 0,
               stream=None):
    """One level with given splitters: (output, id histogram, children list)."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    _dev(splitters, "splitters")
    out = torch.empty_like(keys)
    hist = torch.zeros(2 * m - 1, dtype=torch.uint32, device=keys.device)
    kids = torch.zeros(4 * 3 * r + 4, dtype=torch.uint32, device=keys.device)
    nk = ctypes.c_uint32(0)
    check(lib().ams_step_level(kt, keys.data_ptr(), out.data_ptr(), keys.numel(),
                               splitters.data_ptr(), m, r, flags, hist.data_ptr(), kids.data_ptr(),
                               ctypes.byref(nk), _stream(stream)))
    n = nk.value
    return out, hist, kids[: 4 * n].view(n, 4) if n else kids[:0].view(0, 4)


def step_pack(weights: torch.Tensor, r: int, stream=None):
    """(L*, group starts) for uint32 weights on the GPU."""
    _dev(weights, "weights")
    if weights.dtype != torch.uint32:
        raise ValueError("weights must be uint32")
    out = torch.zeros(2 + weights.numel() + 1, dtype=torch.uint32, device=weights.device)
    check(lib().ams_step_pack(weights.data_ptr(), weights.numel(), r, out.data_ptr(),
                              _stream(stream)))
    return out


def step_base_case(keys: torch.Tensor, vals: torch.Tensor | None = None, cutoff: int = 0,
                   stream=None):
    kt = key_type_of(keys)
    _dev(keys, "keys")
    ok = torch.empty_like(keys)
    ov = torch.empty_like(vals) if vals is not None else None
    check(lib().ams_step_base_case(kt, keys.data_ptr(), vals.data_ptr() if vals is not None else None,
                                   ok.data_ptr(), ov.data_ptr() if ov is not None else None,
                                   keys.numel(), cutoff, _stream(stream)))
    return (ok, ov) if vals is not None else ok


__all__ = [
    "AMS_U32", "AMS_U64", "AMS_F32", "KT_TO_DTYPE", "key_type_of", "make_params",
    "workspace_bytes", "batch_workspace_bytes", "alloc_workspace", "sort_keys", "sort_pairs",
    "sort_batch", "step_splitters", "step_level", "step_pack", "step_base_case", "_lib",
    "trace_start", "trace_stop", "autotune", "autotune_clear", "params_dict",
    "device_errors", "workspace_stats", "rlm_params", "rlm_workspace_bytes", "rlm_sort_keys",
    "step_multiselect",
]


def trace_start():
    """Start per-kernel event timing for this thread's sort calls."""
    check(lib().ams_trace_start())


def trace_stop() -> list:
    """Stop tracing; [{name, launches, total_ms, max_ms}] per kernel."""
    n = lib().ams_trace_stop(None, 0)
    arr = (_lib.TraceEntry * max(n, 1))()
    n = lib().ams_trace_stop(arr, n)
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches,
             "total_ms": arr[i].total_ms, "max_ms": arr[i].max_ms} for i in range(n)]


def device_errors(clear: bool = True, stream=None) -> int:
    """AMS_DEVERR_* bits raised on the current device since the last clear
    (waits for the stream)."""
    bits = ctypes.c_uint32(0)
    check(lib().ams_device_errors(_stream(stream), ctypes.byref(bits), int(clear)))
    return int(bits.value)


def workspace_stats(workspace: torch.Tensor, stream=None) -> dict:
    """Counters of the last sort that ran in ``workspace`` (waits for the
    stream): per-level subproblems, keys, final keys, largest child and
    imbalance; leaves and their keys."""
    st = _lib.RunStats()
    check(lib().ams_workspace_stats(workspace.data_ptr(), _stream(stream), ctypes.byref(st)))
    return st.as_dict()


def rlm_params(ways: int = 0, tile_keys: int = 0, seed: int = 0, flags: int = 0):
    """ams_rlm_params (0 = automatic)."""
    p = _lib.RlmParams()
    p.ways, p.tile_keys, p.seed, p.flags = int(ways), int(tile_keys), int(seed), int(flags)
    return p


def rlm_workspace_bytes(key_type: int, n: int, params=None) -> int:
    return int(lib().ams_rlm_workspace_bytes(key_type, n, _pref(params)))


def rlm_sort_keys(keys: torch.Tensor, out: torch.Tensor | None = None, params=None,
                  workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Sorted copy of ``keys`` by RLM-sort (recurse-last multiway mergesort)."""
    kt = key_type_of(keys)
    _dev(keys, "keys")
    if out is None:
        out = torch.empty_like(keys)
    _dev(out, "out")
    if out.numel() != keys.numel() or out.dtype != keys.dtype:
        raise ValueError("out must match keys")
    ws = workspace.data_ptr() if workspace is not None else None
    wsb = workspace.numel() if workspace is not None else 0
    check(lib().ams_rlm_sort_keys(kt, keys.data_ptr(), out.data_ptr(), keys.numel(), ws, wsb,
                                  _stream(stream), _pref(params)))
    return out


def step_multiselect(runs: torch.Tensor, run_keys: int, parts: int, seed: int = 0,
                     stream=None) -> torch.Tensor:
    """Cut table (parts+1, number of runs) of one RLM level over keys sorted
    within consecutive runs of run_keys (synchronises)."""
    kt = key_type_of(runs)
    _dev(runs, "runs")
    n = runs.numel()
    S = (n + run_keys - 1) // run_keys
    cuts = torch.empty((parts + 1, S), dtype=torch.uint32, device=runs.device)
    check(lib().ams_step_multiselect(kt, runs.data_ptr(), n, run_keys, parts, seed,
                                     cuts.data_ptr(), _stream(stream)))
    return cuts
