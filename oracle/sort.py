"""Whole-sort oracle.  TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition followed (problem statement, Section 1; tie-breaking by input
position, Section 2 and Appendix D): the output is the unique permutation pi
of 0..n-1 for which (ord(K[pi(i)]), pi(i)) strictly increases in i.  Keys are
returned bit for bit (K'[i] = K[pi(i)]) and the payload follows
(V'[i] = V[pi(i)]).

ord is the identity for unsigned integers.  Float32 keys are ordered by IEEE
754-2008 totalOrder on their bit patterns (-NaN < -inf < ... < -0 < +0 < ...
< +inf < +NaN), which the paper does not cover (it sorts 64-bit integers).

Three independent routes compute pi:
  * ``oracle_sort_perm``  textbook top-down mergesort in C (``mergesort.c``);
    ``oracle_sort_perm_parallel`` is the same mergesort on several threads
    (chunks, then a pairwise merge tree), used to time the oracle on all
    host cores;
  * ``py_mergesort_perm`` the same textbook algorithm in pure Python, for
    tiny inputs;
  * ``brute_force_perm``  enumeration of all n! permutations, keeping the one
    that satisfies the definition (n <= 8).
"""

from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

KEY_U32 = 1
KEY_U64 = 2
KEY_F32 = 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_liboracle.so")
_SRC = os.path.join(_HERE, "mergesort.c")
_lib = None


def key_dtype(key_type: int):
    """numpy dtype holding the raw key bits of a key type."""
    return {KEY_U32: np.uint32, KEY_U64: np.uint64, KEY_F32: np.float32}[key_type]


def build_oracle(force: bool = False) -> str:
    """Compile ``mergesort.c`` with gcc into ``_liboracle.so`` (plain C)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-pthread", "-shared", "-fPIC", _SRC,
                               "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_oracle())
        lib.oracle_sort_perm.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_void_p]
        lib.oracle_sort_perm.restype = ctypes.c_int
        lib.oracle_sort.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_sort.restype = ctypes.c_int
        lib.oracle_sort_perm_parallel.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                                  ctypes.c_void_p, ctypes.c_int]
        lib.oracle_sort_perm_parallel.restype = ctypes.c_int
        _lib = lib
    return _lib


# ----------------------------------------------------------------------------
# ord
# ----------------------------------------------------------------------------

def ord_bits(key_type: int, bits: int) -> int:
    """ord of one key given as its raw bit pattern (Python int)."""
    if key_type in (KEY_U32, KEY_U64):
        return bits
    if bits & 0x80000000:
        return (~bits) & 0xFFFFFFFF
    return bits | 0x80000000


def ord_keys(key_type: int, keys: np.ndarray) -> np.ndarray:
    """ord of every key, as uint64 (vectorised form of ``ord_bits``)."""
    if key_type == KEY_U32:
        return keys.astype(np.uint64)
    if key_type == KEY_U64:
        return keys.astype(np.uint64, copy=True)
    u = keys.view(np.uint32).astype(np.uint64)
    neg = (u & np.uint64(0x80000000)) != 0
    return np.where(neg, (~u) & np.uint64(0xFFFFFFFF), u | np.uint64(0x80000000))


def raw_bits(key_type: int, keys: np.ndarray) -> list:
    """Raw bit patterns as Python ints."""
    if key_type == KEY_F32:
        return [int(x) for x in keys.view(np.uint32)]
    return [int(x) for x in keys]


# ----------------------------------------------------------------------------
# C mergesort
# ----------------------------------------------------------------------------

def oracle_sort_perm(key_type: int, keys: np.ndarray) -> np.ndarray:
    """pi as a uint64 array, from the C textbook mergesort."""
    keys = np.ascontiguousarray(keys, dtype=key_dtype(key_type))
    n = keys.size
    perm = np.empty(n, dtype=np.uint64)
    if n:
        rc = _load().oracle_sort_perm(key_type, keys.ctypes.data, n, perm.ctypes.data)
        if rc:
            raise MemoryError("oracle_sort_perm failed (%d)" % rc)
    return perm


def oracle_sort_perm_parallel(key_type: int, keys: np.ndarray, threads: int) -> np.ndarray:
    """pi from the plain parallel mergesort (one chunk per thread, then a
    pairwise merge tree); the same permutation as ``oracle_sort_perm``."""
    keys = np.ascontiguousarray(keys, dtype=key_dtype(key_type))
    n = keys.size
    perm = np.empty(n, dtype=np.uint64)
    if n:
        rc = _load().oracle_sort_perm_parallel(key_type, keys.ctypes.data, n, perm.ctypes.data,
                                               int(threads))
        if rc:
            raise ValueError("oracle_sort_perm_parallel failed (%d)" % rc)
    return perm


def oracle_sort(key_type: int, keys: np.ndarray, vals: np.ndarray | None = None):
    """Sorted keys (bit for bit) and, when given, the payload that follows them."""
    keys = np.ascontiguousarray(keys, dtype=key_dtype(key_type))
    n = keys.size
    out_k = np.empty_like(keys)
    out_v = None
    vp = None
    ovp = None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        if vals.size != n:
            raise ValueError("payload length differs from key length")
        out_v = np.empty_like(vals)
        vp = vals.ctypes.data
        ovp = out_v.ctypes.data
    if n:
        rc = _load().oracle_sort(key_type, keys.ctypes.data, vp, n, out_k.ctypes.data, ovp)
        if rc:
            raise MemoryError("oracle_sort failed (%d)" % rc)
    return out_k, out_v


# ----------------------------------------------------------------------------
# Pure-Python twin and brute force (tiny inputs)
# ----------------------------------------------------------------------------

def py_mergesort_perm(key_type: int, keys) -> list:
    """Textbook top-down mergesort of positions by ord; ties take the left run."""
    ords = [ord_bits(key_type, b) for b in raw_bits(key_type, np.asarray(keys, dtype=key_dtype(key_type)))]

    def msort(idx):
        if len(idx) < 2:
            return idx
        mid = len(idx) // 2
        left, right = msort(idx[:mid]), msort(idx[mid:])
        out = []
        i = j = 0
        while i < len(left) and j < len(right):
            if ords[right[j]] < ords[left[i]]:
                out.append(right[j])
                j += 1
            else:
                out.append(left[i])
                i += 1
        out.extend(left[i:])
        out.extend(right[j:])
        return out

    return msort(list(range(len(ords))))


def brute_force_perm(key_type: int, keys) -> list:
    """The permutation satisfying the output definition, found by trying all n!.

    Asserts that exactly one permutation qualifies (uniqueness of the result).
    """
    ords = [ord_bits(key_type, b) for b in raw_bits(key_type, np.asarray(keys, dtype=key_dtype(key_type)))]
    n = len(ords)
    if n > 8:
        raise ValueError("brute force is for n <= 8")
    found = []
    for p in itertools.permutations(range(n)):
        if all((ords[p[i]], p[i]) < (ords[p[i + 1]], p[i + 1]) for i in range(n - 1)):
            found.append(list(p))
    assert len(found) == 1, "output definition must single out one permutation"
    return found[0]
