"""Seeded synthetic inputs shaped like the paper's workloads and the named
sort configurations.

This module holds no part of the sort: it only draws keys.  Both the GPU path
and the oracle are fed from it.  The paper sorts uniformly random 64-bit
integers (Section 7, experimental setup); the other shapes (heavy duplicates,
Zipf, all-equal, float32 normals, uneven batches, Poisson request streams)
follow the workload descriptions of the benchmark configurations.

Base seed 14106754; workload c uses seed 14106754 + c.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 14106754

KEY_U32 = 1
KEY_U64 = 2
KEY_F32 = 3


def dtype_of(key_type: int):
    return {KEY_U32: np.uint32, KEY_U64: np.uint64, KEY_F32: np.float32}[key_type]


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng([BASE_SEED + config, salt])


def uniform_u64(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform over [0, 2^64)."""
    return rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)


def uniform_u32(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.integers(0, np.iinfo(np.uint32).max, size=n, dtype=np.uint32, endpoint=True)


def normal_f32(n: int, rng: np.random.Generator) -> np.ndarray:
    """float32 drawn from N(0, 1)."""
    return rng.standard_normal(n, dtype=np.float32)


def few_distinct_u64(n: int, rng: np.random.Generator, distinct: int = 1 << 10) -> np.ndarray:
    """Keys drawn from ``distinct`` uniform u64 values (heavy duplicates)."""
    values = uniform_u64(distinct, rng)
    return values[rng.integers(0, distinct, size=n)]


def zipf_u64(n: int, rng: np.random.Generator, s: float = 1.1, support: int = 1 << 32) -> np.ndarray:
    """Zipf(s) ranks truncated to [1, support] by redrawing; key = rank - 1."""
    out = np.empty(n, dtype=np.uint64)
    filled = 0
    while filled < n:
        draw = rng.zipf(s, size=max(1024, int((n - filled) * 1.15)))
        draw = draw[draw <= support]
        take = min(draw.size, n - filled)
        out[filled:filled + take] = (draw[:take] - 1).astype(np.uint64)
        filled += take
    return out


def all_equal_u64(n: int, value: int = 0x0123456789ABCDEF) -> np.ndarray:
    return np.full(n, value, dtype=np.uint64)


def float_specials() -> np.ndarray:
    """float32 bit patterns covering the edge cases of totalOrder."""
    bits = [
        0x00000000, 0x80000000,              # +0, -0
        0x7F800000, 0xFF800000,              # +inf, -inf
        0x7FC00000, 0xFFC00000,              # quiet NaNs
        0x7F800001, 0xFF800001,              # signalling NaNs
        0x7FFFFFFF, 0xFFFFFFFF,              # NaNs with full payload
        0x00000001, 0x80000001,              # smallest subnormals
        0x007FFFFF, 0x807FFFFF,              # largest subnormals
        0x00800000, 0x80800000,              # smallest normals
        0x3F800000, 0xBF800000,              # +1, -1
        0x7F7FFFFF, 0xFF7FFFFF,              # largest finite
    ]
    return np.array(bits, dtype=np.uint32).view(np.float32)


def keys(key_type: int, n: int, rng: np.random.Generator, dist: str = "uniform") -> np.ndarray:
    """Keys of one type and distribution."""
    if dist == "uniform":
        if key_type == KEY_U64:
            return uniform_u64(n, rng)
        if key_type == KEY_U32:
            return uniform_u32(n, rng)
        return normal_f32(n, rng)
    if dist == "few":
        k = few_distinct_u64(n, rng)
    elif dist == "zipf":
        k = zipf_u64(n, rng)
    elif dist == "equal":
        k = all_equal_u64(n)
    elif dist == "sorted":
        k = np.sort(keys(key_type, n, rng, "uniform"))
        return k
    elif dist == "reversed":
        return np.sort(keys(key_type, n, rng, "uniform"))[::-1].copy()
    elif dist == "specials":
        base = float_specials().view(np.uint32)
        pick = base[rng.integers(0, base.size, size=n)]
        if key_type == KEY_F32:
            return pick.view(np.float32)
        k = pick.astype(np.uint64)
    else:
        raise ValueError(dist)
    if key_type == KEY_U64:
        return k
    if key_type == KEY_U32:
        return (k & np.uint64(0xFFFFFFFF)).astype(np.uint32) if dist != "equal" else k.astype(np.uint32)
    return (k & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


def batch_sizes(count: int, rng: np.random.Generator, lo_exp: float = 8.0, hi_exp: float = 20.0) -> np.ndarray:
    """Segment sizes floor(2^U), U ~ Uniform(lo_exp, hi_exp) (log-uniform)."""
    return np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)


def truncate_total(sizes: np.ndarray, total: int) -> np.ndarray:
    """Leading segments whose cumulative size stays within ``total``."""
    c = np.cumsum(sizes)
    return sizes[: int(np.searchsorted(c, total, side="right"))]


def serving_stream(count: int, rng: np.random.Generator, rate_per_s: float,
                   lo_exp: float = 10.0, hi_exp: float = 24.0):
    """Poisson arrivals (exponential gaps), log-uniform sizes, key types mixed
    50% u64 / 25% u32 / 25% f32.  Returns (arrival_s, sizes, key_types)."""
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = batch_sizes(count, rng, lo_exp, hi_exp)
    u = rng.uniform(size=count)
    kt = np.where(u < 0.5, KEY_U64, np.where(u < 0.75, KEY_U32, KEY_F32)).astype(np.int64)
    return arrivals, sizes, kt
