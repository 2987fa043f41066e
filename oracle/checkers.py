"""Independent checks on a sort's output.  TEST INFRASTRUCTURE ONLY.

Together these properties characterise the unique result of the problem
statement (Section 1) with position tie-breaking (Section 2):
  * keys-only: the output is non-decreasing in ord and holds the same multiset
    of bit patterns as the input (count, wrapping sum and xor of a 64-bit
    mix of every key; ord is a bijection, so equal ord means equal bits);
  * pairs with payload V = 0..n-1: V' is a permutation of 0..n-1, every
    output key is the input key its payload names (K'[i] == K[V'[i]] bit for
    bit), the keys are non-decreasing in ord, and equal keys carry strictly
    increasing payloads (stability).
They run vectorised over arrays of any size, so they also cover full-size
outputs that the mergesort would take too long to produce.
"""

from __future__ import annotations

import numpy as np

from .sort import KEY_F32, KEY_U32, KEY_U64, ord_keys  # noqa: F401


def _bits64(key_type: int, keys: np.ndarray) -> np.ndarray:
    if key_type == KEY_F32:
        return keys.view(np.uint32).astype(np.uint64)
    return keys.astype(np.uint64)


def mix64_np(z: np.ndarray) -> np.ndarray:
    """SplitMix64's output function, vectorised (wrapping uint64 arithmetic)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def fingerprint(key_type: int, keys: np.ndarray, chunk: int = 1 << 24):
    """(count, sum of mix64(bits) mod 2^64, xor of mix64(bits))."""
    n = keys.size
    s = np.uint64(0)
    x = np.uint64(0)
    with np.errstate(over="ignore"):
        for i in range(0, n, chunk):
            h = mix64_np(_bits64(key_type, keys[i:i + chunk]))
            s = np.uint64(s + np.add.reduce(h, dtype=np.uint64))
            x = np.uint64(x ^ np.bitwise_xor.reduce(h))
    return int(n), int(s), int(x)


def is_sorted(key_type: int, keys: np.ndarray, chunk: int = 1 << 24) -> bool:
    """ord non-decreasing over the whole array."""
    n = keys.size
    prev = None
    for i in range(0, n, chunk):
        o = ord_keys(key_type, keys[i:i + chunk])
        if o.size and prev is not None and o[0] < prev:
            return False
        if o.size > 1 and np.any(o[1:] < o[:-1]):
            return False
        if o.size:
            prev = o[-1]
    return True


def check_keys(key_type: int, keys_in: np.ndarray, keys_out: np.ndarray) -> str | None:
    """None when keys_out is the sorted permutation of keys_in, else a reason."""
    if keys_in.size != keys_out.size:
        return "length differs"
    if not is_sorted(key_type, keys_out):
        return "output not sorted"
    if fingerprint(key_type, keys_in) != fingerprint(key_type, keys_out):
        return "multiset of keys differs"
    return None


def check_pairs(key_type: int, keys_in: np.ndarray, keys_out: np.ndarray,
                vals_out: np.ndarray) -> str | None:
    """None when (keys_out, vals_out) is the stable sort of keys_in with the
    payload 0..n-1, else a reason."""
    n = keys_in.size
    if keys_out.size != n or vals_out.size != n:
        return "length differs"
    if n == 0:
        return None
    v = vals_out.astype(np.int64)
    if v.min() < 0 or v.max() >= n:
        return "payload out of range"
    if np.bincount(v, minlength=n).max() != 1:
        return "payload is not a permutation"
    if not np.array_equal(_bits64(key_type, keys_in)[v], _bits64(key_type, keys_out)):
        return "key does not match the element its payload names"
    o = ord_keys(key_type, keys_out)
    if np.any(o[1:] < o[:-1]):
        return "output not sorted"
    ties = o[1:] == o[:-1]
    if np.any(ties & (v[1:] <= v[:-1])):
        return "equal keys out of input order (not stable)"
    return None
