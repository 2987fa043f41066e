"""The C ABI library loads and exports every symbol include/ams.h declares;
host-only calls behave (CPU only: no kernel is launched)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ams.h")


def _lib():
    from paper_1410_6754_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1410_6754_amd import _lib as L
    return L.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ams_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = _lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1410_6754_amd import _lib as L
    assert sorted(n for n, _, _ in L.EXPORTS) == _declared()


def test_version_and_error_string():
    lib = _lib()
    assert b"gfx950" in lib.ams_version()
    assert lib.ams_last_error() is not None


def test_invalid_arguments_rejected_without_gpu():
    lib = _lib()
    from paper_1410_6754_amd import _lib as L
    # unknown key type
    assert lib.ams_sort_keys(7, None, None, 10, None, 0, None, None) == L.AMS_EINVAL
    # NULL pointers with n > 0
    assert lib.ams_sort_keys(L.AMS_U64, None, None, 10, None, 0, None, None) == L.AMS_EINVAL
    # n = 0 is a no-op
    assert lib.ams_sort_keys(L.AMS_U64, None, None, 0, None, 0, None, None) == L.AMS_OK
    # sizes of 2^32 or more are unsupported
    assert lib.ams_workspace_bytes(L.AMS_U64, 1 << 32, 0, None) == 0
    # bad tuning parameters
    p = L.Params()
    p.k = 3
    assert lib.ams_sort_keys(L.AMS_U64, 8, 8, 100000, None, 0, None, ctypes.byref(p)) == L.AMS_EINVAL
    assert b"power of two" in lib.ams_last_error()


def test_workspace_grows_with_n_and_payload():
    lib = _lib()
    from paper_1410_6754_amd import _lib as L
    small = lib.ams_workspace_bytes(L.AMS_U64, 1000, 0, None)
    big = lib.ams_workspace_bytes(L.AMS_U64, 1 << 20, 0, None)
    pairs = lib.ams_workspace_bytes(L.AMS_U64, 1 << 20, 1, None)
    assert 0 < small < big < pairs
    # the level buffers hold at least one copy of the keys
    assert big >= (1 << 20) * 8
    offs = (ctypes.c_uint64 * 4)(0, 100, 100, 70000)
    assert lib.ams_batch_workspace_bytes(L.AMS_U32, offs, 3, 0, None) > 0


@pytest.mark.parametrize("n", [1 << 20, 1 << 28])
def test_plan_capacities_cover_the_level_bounds(n):
    # workspace for a one-root sort holds the keys once more plus the tables;
    # far below four copies of the data for large n
    lib = _lib()
    from paper_1410_6754_amd import _lib as L
    ws = lib.ams_workspace_bytes(L.AMS_U64, n, 0, None)
    assert n * 8 <= ws < 4 * n * 8
