"""Python handle on the C++ serving loop (ams_server_* in the C ABI)."""

from __future__ import annotations

import ctypes

import torch

from ._lib import AMS_OK, ReqStats, check, lib
from .api import KT_TO_DTYPE, _dev, _stream, key_type_of


def _stats(st: ReqStats) -> dict:
    return {f: getattr(st, f) for f, _ in ReqStats._fields_}


class Server:
    """Continuous-batching sort server on one device.

    ``budget`` bytes of device memory (0 = 80% of free) bound the result
    buffers and workspaces of admitted requests; ``streams`` worker streams
    let batches overlap.
    """

    def __init__(self, device: int = 0, budget: int = 0, max_pending: int = 0, streams: int = 0):
        st = ctypes.c_int(0)
        self._h = lib().ams_server_create(device, budget, max_pending, streams, ctypes.byref(st))
        if not self._h:
            check(st.value if st.value else -3)
        self._keep = {}
        self.device = device

    def submit(self, keys: torch.Tensor, vals: torch.Tensor | None = None) -> int:
        kt = key_type_of(keys)
        _dev(keys, "keys")
        vp = None
        if vals is not None:
            _dev(vals, "vals")
            vp = vals.data_ptr()
        t = ctypes.c_uint64(0)
        check(lib().ams_submit(self._h, kt, keys.data_ptr(), vp, keys.numel(), ctypes.byref(t)))
        self._keep[t.value] = (keys, vals)
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int(0)
        st = ReqStats()
        check(lib().ams_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st)))
        return bool(done.value), _stats(st)

    def wait(self, ticket: int) -> dict:
        st = ReqStats()
        rc = lib().ams_wait(self._h, ticket, ctypes.byref(st))
        check(rc)
        return _stats(st)

    def result(self, ticket: int, stream=None):
        """Copies of the sorted keys (and payload) as new tensors."""
        keys, vals = self._keep[ticket]
        ok = torch.empty_like(keys)
        ov = torch.empty_like(vals) if vals is not None else None
        check(lib().ams_result_copy(self._h, ticket, ok.data_ptr(),
                                    ov.data_ptr() if ov is not None else None, _stream(stream)))
        return (ok, ov) if vals is not None else ok

    def result_ptrs(self, ticket: int):
        k = ctypes.c_void_p(0)
        v = ctypes.c_void_p(0)
        check(lib().ams_result(self._h, ticket, ctypes.byref(k), ctypes.byref(v)))
        return k.value, v.value

    def inject_alloc_failures(self, count: int):
        """Test hook: the next ``count`` batches fail as if out of memory."""
        check(lib().ams_server_inject_alloc_failures(self._h, count))

    def release(self, ticket: int):
        # the result may still be read by work queued on the current stream
        # (result() copies there); the library frees in order on its own
        # stream, so let that work finish first
        torch.cuda.current_stream(self.device).synchronize()
        check(lib().ams_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def close(self):
        if self._h:
            lib().ams_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Server", "KT_TO_DTYPE", "AMS_OK"]
