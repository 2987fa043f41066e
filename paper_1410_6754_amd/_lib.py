"""ctypes binding of libams.so.  Argument marshalling only: every step of the
sort runs in the HIP library.  PyTorch supplies device memory and streams.

The library must have been built (``paper_1410_6754_amd.build.build()``);
loading fails loudly otherwise, there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libams.so")

AMS_U32 = 1
AMS_U64 = 2
AMS_F32 = 3

AMS_OK = 0
AMS_EINVAL = -1
AMS_ENOMEM = -2
AMS_EHIP = -3
AMS_EAGAIN = -4
AMS_EUNSUPPORTED = -5
AMS_ENOTFOUND = -6
AMS_EDEVICE = -7

AMS_MAX_SEGMENT = (1 << 32) - (1 << 20)

AMS_FLAG_EQ_ALWAYS = 1
AMS_FLAG_STABLE_PARTITION = 2
AMS_FLAG_SAMPLED_LEAF_SPLIT = 4
AMS_FLAG_CHECK = 8
AMS_FLAG_TEST_TINY_TABLES = 16
AMS_FLAG_STRATIFIED = 32
AMS_FLAG_TEST_NO_PIECE_ROOM = 64

AMS_DEVERR_TABLE = 1
AMS_DEVERR_ACTIVE = 2
AMS_DEVERR_TILES = 4
AMS_DEVERR_GROUPS = 8
AMS_DEVERR_RANGE = 16
AMS_DEVERR_LEAF = 32

_STATUS = {0: "AMS_OK", -1: "AMS_EINVAL", -2: "AMS_ENOMEM", -3: "AMS_EHIP",
           -4: "AMS_EAGAIN", -5: "AMS_EUNSUPPORTED", -6: "AMS_ENOTFOUND", -7: "AMS_EDEVICE"}


class AmsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class Params(ctypes.Structure):
    """Mirror of ams_params (0 = automatic)."""
    _fields_ = [
        ("levels", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("overpartition_b", ctypes.c_uint32),
        ("samples_per_bucket", ctypes.c_uint32),
        ("tile_keys", ctypes.c_uint32),
        ("base_cutoff", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("leaf_capacity", ctypes.c_uint32),
    ]


class ReqStats(ctypes.Structure):
    """Mirror of ams_req_stats."""
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("key_type", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("batch_id", ctypes.c_uint64),
        ("batch_size", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("t_submit_us", ctypes.c_double),
        ("t_admit_us", ctypes.c_double),
        ("t_launch_us", ctypes.c_double),
        ("t_done_us", ctypes.c_double),
        ("gpu_ms", ctypes.c_double),
    ]


class TraceEntry(ctypes.Structure):
    """Mirror of ams_trace_entry."""
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("total_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double),
    ]


class RunStats(ctypes.Structure):
    """Mirror of ams_run_stats."""
    _fields_ = [
        ("device_errors", ctypes.c_uint32),
        ("levels", ctypes.c_uint32),
        ("subproblems", ctypes.c_uint32 * 4),
        ("keys", ctypes.c_uint64 * 4),
        ("final_keys", ctypes.c_uint64 * 4),
        ("max_child", ctypes.c_uint32 * 4),
        ("tiles", ctypes.c_uint32 * 4),
        ("imbalance_max", ctypes.c_double * 4),
        ("imbalance_mean", ctypes.c_double * 4),
        ("leaves", ctypes.c_uint32),
        ("big_leaves", ctypes.c_uint32),
        ("leaf_keys", ctypes.c_uint64),
        ("copy_keys", ctypes.c_uint64),
        ("big_keys", ctypes.c_uint64),
        ("merge_ranges", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("merge_keys", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class RlmParams(ctypes.Structure):
    """Mirror of ams_rlm_params (0 = automatic)."""
    _fields_ = [
        ("ways", ctypes.c_uint32),
        ("tile_keys", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


# (name, restype, argtypes) of every exported symbol declared in include/ams.h
_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_I = ctypes.c_int
EXPORTS = [
    ("ams_workspace_bytes", _SZ, [_I, _SZ, _I, _P]),
    ("ams_batch_workspace_bytes", _SZ, [_I, _P, _SZ, _I, _P]),
    ("ams_sort_keys", _I, [_I, _P, _P, _SZ, _P, _SZ, _P, _P]),
    ("ams_sort_pairs", _I, [_I, _P, _P, _P, _P, _SZ, _P, _SZ, _P, _P]),
    ("ams_sort_batch", _I, [_I, _P, _P, _P, _P, _P, _P, _SZ, _P, _SZ, _P, _P]),
    ("ams_last_error", ctypes.c_char_p, []),
    ("ams_version", ctypes.c_char_p, []),
    ("ams_trace_start", _I, []),
    ("ams_trace_stop", _I, [_P, _I]),
    ("ams_server_create", _P, [_I, _SZ, _U32, _U32, _P]),
    ("ams_submit", _I, [_P, _I, _P, _P, _SZ, _P]),
    ("ams_poll", _I, [_P, _U64, _P, _P]),
    ("ams_wait", _I, [_P, _U64, _P]),
    ("ams_result", _I, [_P, _U64, _P, _P]),
    ("ams_result_copy", _I, [_P, _U64, _P, _P, _P]),
    ("ams_release", _I, [_P, _U64]),
    ("ams_server_destroy", None, [_P]),
    ("ams_step_splitters", _I, [_I, _P, _SZ, _U32, _U32, _U64, _P, _P]),
    ("ams_step_level", _I, [_I, _P, _P, _SZ, _P, _U32, _U32, _U32, _P, _P, _P, _P]),
    ("ams_step_pack", _I, [_P, _U32, _U32, _P, _P]),
    ("ams_step_base_case", _I, [_I, _P, _P, _P, _P, _SZ, _U32, _P]),
    ("ams_autotune", _I, [_I, _P, _P, _P, _SZ, _P, _U32, _P, _P]),
    ("ams_autotune_clear", None, []),
    ("ams_device_errors", _I, [_P, _P, _I]),
    ("ams_workspace_stats", _I, [_P, _P, _P]),
    ("ams_server_inject_alloc_failures", _I, [_P, _U32]),
    ("ams_device_copy", _I, [_P, _P, _SZ, _P]),
    ("ams_rlm_workspace_bytes", _SZ, [_I, _SZ, _P]),
    ("ams_rlm_sort_keys", _I, [_I, _P, _P, _SZ, _P, _SZ, _P, _P]),
    ("ams_step_multiselect", _I, [_I, _P, _SZ, _U32, _U32, _U64, _P, _P]),
    ("ams_sort_keys_noalloc", _I, [_I, _P, _P, _SZ, _P, _P]),
]

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libams.so is not built; run paper_1410_6754_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in EXPORTS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != AMS_OK:
        msg = lib().ams_last_error()
        raise AmsError(status, msg.decode() if msg else "")
