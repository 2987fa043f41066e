// Device-side building blocks of the sample sort: key encodings, the
// SplitMix64 sampling stream, wavefront primitives and the splitter-tree
// descent.  gfx950 only (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AMS_DEV __device__ __forceinline__
#define AMS_HD __host__ __device__ __forceinline__

namespace ams {

enum : int { KT_U32 = 1, KT_U64 = 2, KT_F32 = 3 };

// Where a subproblem's elements currently live.
enum : uint32_t { BUF_IN = 0, BUF_TMP = 1, BUF_OUT = 2 };
// Leaf kinds for the base-case kernel.
enum : uint32_t { LEAF_REG = 0, LEAF_COPY = 1, LEAF_BIG = 2 };
// Child kinds (bucket grouping output).
enum : uint32_t { CHILD_REG = 0, CHILD_FINAL = 1 };

constexpr uint32_t WAVE = 64;
constexpr uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;

// ---------------------------------------------------------------------------
// Keys.  T is the stored word; enc maps raw bits to an unsigned value whose
// integer order is the key order (identity for integers, IEEE totalOrder for
// float32: set the sign bit of non-negative values, invert negative ones).
// ---------------------------------------------------------------------------
template <int KT> struct Key;
template <> struct Key<KT_U32> {
  typedef uint32_t T;
  static AMS_DEV T enc(T x) { return x; }
  static AMS_DEV T dec(T x) { return x; }
};
template <> struct Key<KT_U64> {
  typedef uint64_t T;
  static AMS_DEV T enc(T x) { return x; }
  static AMS_DEV T dec(T x) { return x; }
};
template <> struct Key<KT_F32> {
  typedef uint32_t T;
  static AMS_DEV T enc(T x) { return (x & 0x80000000u) ? ~x : (x | 0x80000000u); }
  static AMS_DEV T dec(T x) { return (x & 0x80000000u) ? (x & 0x7FFFFFFFu) : ~x; }
};

// ---------------------------------------------------------------------------
// Subproblems.  A root is one independent input; a segment is a contiguous
// range of a root in one of its three buffers.
// ---------------------------------------------------------------------------
struct Root {
  const void *kin;
  const uint32_t *vin;
  void *kout;
  uint32_t *vout;
  uint64_t n;
  uint64_t tmp_off;  // element offset of this root inside the TMP buffers
};

struct Seg {
  uint32_t off;   // element offset inside the root
  uint32_t size;  // elements
  uint32_t root;
  uint32_t meta;  // buf | kind << 4 | dst << 8
};

AMS_HD uint32_t seg_meta(uint32_t buf, uint32_t kind, uint32_t dst) {
  return buf | (kind << 4) | (dst << 8);
}
AMS_DEV uint32_t seg_buf(uint32_t meta) { return meta & 15u; }
AMS_DEV uint32_t seg_kind(uint32_t meta) { return (meta >> 4) & 15u; }
AMS_DEV uint32_t seg_dst(uint32_t meta) { return (meta >> 8) & 15u; }

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): output i of a generator at state s is
// mix64(s + i * gamma).  Sample positions are floor(n * u / 2^64).
// ---------------------------------------------------------------------------
AMS_DEV uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

AMS_DEV uint64_t stream_state(uint64_t seed, uint32_t level, uint32_t root, uint64_t off) {
  uint64_t s = mix64(seed + GOLDEN_GAMMA);
  s = mix64(s ^ (uint64_t)(level + 1));
  s = mix64(s ^ (uint64_t)root);
  return mix64(s ^ off);
}

AMS_DEV uint32_t draw_pos(uint64_t state, uint32_t i, uint32_t n) {
  uint64_t u = mix64(state + (uint64_t)(i + 1) * GOLDEN_GAMMA);
  return (uint32_t)__umul64hi(u, (uint64_t)n);
}

// ---------------------------------------------------------------------------
// Raw buffer access.  A buffer resource covers [base, base + bytes); loads
// outside it return zero instead of faulting, which lets ragged tails load
// with full-width instructions.  The resource and the byte offsets are
// wave-uniform (scalar registers); each lane adds its own offset.
// ---------------------------------------------------------------------------
// An object in global memory.  Accesses through GMem<T> pointers compile to
// global_* instructions, which count only in vmcnt; flat ones (what generic
// pointers loaded from memory become) also count in lgkmcnt, so a wait for
// an LDS result would also wait for every flat access in flight.
template <typename T> using GMem = __attribute__((address_space(1))) T;

// A 64-bit word that may alias narrower data: rows of 16-bit LDS entries are
// written or cleared four entries at a time through it and read back entry
// by entry, which type-based alias analysis would otherwise let the compiler
// reorder.
typedef uint64_t __attribute__((__may_alias__)) u64_alias;

typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t Rsrc;

AMS_DEV Rsrc make_rsrc(const void *base, uint32_t bytes) {
  // word 3: raw (untyped) access with 32-bit data format, as gfx9 expects
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// 16 bytes per lane: 2 uint64 or 4 uint32 keys.
template <typename K> struct Vec16;
template <> struct Vec16<uint64_t> {
  static constexpr uint32_t N = 2;
  static AMS_DEV void get(v4u32 v, uint64_t *x) {
    x[0] = ((uint64_t)v.y << 32) | v.x;
    x[1] = ((uint64_t)v.w << 32) | v.z;
  }
};
template <> struct Vec16<uint32_t> {
  static constexpr uint32_t N = 4;
  static AMS_DEV void get(v4u32 v, uint32_t *x) {
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  }
};

// One element (4 or 8 bytes) through a buffer resource at byte offset off
// (the whole offset in the range-checked vector operand): past the
// resource's range it reads as zero, so a load needs no branch.
template <typename T> AMS_DEV T buf_load(Rsrc rs, uint32_t off);
template <> AMS_DEV uint32_t buf_load<uint32_t>(Rsrc rs, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
}
template <> AMS_DEV uint64_t buf_load<uint64_t>(Rsrc rs, uint32_t off) {
  const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
  return ((uint64_t)v.y << 32) | v.x;
}

// Wave-uniform copy of a pointer (scalar registers).
template <typename T> AMS_DEV T *uniform_ptr(T *p) {
  const uint64_t a = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return (T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Wavefront primitives (wave64).
// ---------------------------------------------------------------------------
AMS_DEV uint32_t lane_id() { return __lane_id(); }
AMS_DEV uint64_t ballot(bool p) { return __ballot(p ? 1 : 0); }
// number of set bits of mask below this lane
AMS_DEV uint32_t bits_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Lanes (among `valid`) that hold the same value c, found with one ballot per
// bit of c (nbits bits are compared).
AMS_DEV uint64_t match_lanes(uint32_t c, bool valid, uint32_t nbits) {
  uint64_t m = ballot(valid);
  for (uint32_t b = 0; b < nbits; ++b) {
    bool bit = (c >> b) & 1u;
    uint64_t bm = ballot(bit);
    m &= bit ? bm : ~bm;
  }
  return m;
}

// Add 1 to counter ctr[c] for every active lane and return the lane's old
// value (its slot).  When every active lane of the wavefront names the same
// counter (sorted or heavily skewed input) one lane adds for all of them, so
// the LDS atomics do not serialise on one address.  Call from uniform
// control flow.
AMS_DEV uint32_t wave_slot_add(uint32_t *ctr, uint32_t c, bool active) {
  const uint64_t act = ballot(active);
  if (act == 0) return 0;
  const uint32_t lead = (uint32_t)__builtin_ctzll(act);
  const uint32_t c0 = __builtin_amdgcn_readlane(c, lead);
  if (ballot(active && c == c0) == act) {
    uint32_t base = 0;
    if (lane_id() == lead) base = atomicAdd(&ctr[c0], (uint32_t)__popcll(act));
    base = __builtin_amdgcn_readlane(base, lead);
    return base + bits_below(act);
  }
  return active ? atomicAdd(&ctr[c], 1u) : 0u;
}

// Add 1 to ctr[c] for every active lane (no slots returned), aggregated the
// same way.
AMS_DEV void wave_count_add(uint32_t *ctr, uint32_t c, bool active) {
  uint64_t act = ballot(active);
  // up to four runs of equal values (a row of sorted keys crosses a bucket
  // boundary now and then): one add per value, then one per lane
  for (int round = 0; round < 4 && act; ++round) {
    const uint32_t lead = (uint32_t)__builtin_ctzll(act);
    const uint32_t c0 = __builtin_amdgcn_readlane(c, lead);
    const uint64_t same = ballot(active && c == c0) & act;
    if (lane_id() == lead) atomicAdd(&ctr[c0], (uint32_t)__popcll(same));
    act &= ~same;
    active = active && c != c0;
  }
  if (act && active) atomicAdd(&ctr[c], 1u);
}

template <typename T> AMS_DEV T wave_sum(T v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
template <typename T> AMS_DEV T wave_max(T v) {
  for (int d = 32; d >= 1; d >>= 1) {
    T o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}
template <typename T> AMS_DEV T wave_min(T v) {
  for (int d = 32; d >= 1; d >>= 1) {
    T o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Splitter tree.  tree[1..m-1] holds the m-1 sorted splitters in Eytzinger
// (breadth-first) order; descending with "x > node -> right child" for log2 m
// steps ends at m + #{splitters < x}.  The splitter of sorted index j-1
// (j = 1..m-1, in-order rank j) sits at node (m + j) >> (ctz(j) + 1).
// ---------------------------------------------------------------------------
AMS_DEV uint32_t eytzinger_slot(uint32_t j, uint32_t m) { return (m + j) >> (__builtin_ctz(j) + 1); }

// Bucket ids of U keys at once: the descents advance level by level, so each
// level issues U independent LDS reads.  With equality buckets, the splitter
// just above bucket b (in-order rank b + 1) is read from the tree itself
// (eytzinger_slot), so classification touches no memory but the tree.
template <typename K, int U>
AMS_DEV void classify_batch(const K (&x)[U], uint32_t (&id)[U], const K *tree, uint32_t logm,
                            bool eq) {
  uint32_t i[U];
#pragma unroll
  for (int u = 0; u < U; ++u) i[u] = 1;
  for (uint32_t l = 0; l < logm; ++l) {
    K t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = tree[i[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) i[u] = 2 * i[u] + (x[u] > t[u] ? 1u : 0u);
  }
  const uint32_t m = 1u << logm;
  if (!eq) {
#pragma unroll
    for (int u = 0; u < U; ++u) id[u] = i[u] - m;
    return;
  }
  K up[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t b = i[u] - m;
    up[u] = tree[b < m - 1 ? eytzinger_slot(b + 1, m) : 1u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t b = i[u] - m;
    id[u] = 2 * b + ((b < m - 1 && x[u] == up[u]) ? 1u : 0u);
  }
}

// Number of elements < x (strict) or <= x in a sorted array of n = 2^k.
template <typename K> AMS_DEV uint32_t count_less(const K *a, uint32_t n, K x) {
  uint32_t base = 0;
  while (n > 1) {
    uint32_t half = n >> 1;
    base = (a[base + half - 1] < x) ? base + half : base;
    n -= half;
  }
  return base + (a[base] < x ? 1u : 0u);
}
template <typename K> AMS_DEV uint32_t count_less_eq(const K *a, uint32_t n, K x) {
  uint32_t base = 0;
  while (n > 1) {
    uint32_t half = n >> 1;
    base = (a[base + half - 1] <= x) ? base + half : base;
    n -= half;
  }
  return base + (a[base] <= x ? 1u : 0u);
}

// ---------------------------------------------------------------------------
// Item distribution for persistent grids.  Workgroups are dispatched
// round-robin over the 8 XCDs, so block b runs on XCD b % 8; each XCD gets a
// contiguous range of items so that neighbouring tiles share one L2.
// ---------------------------------------------------------------------------
struct ItemRange {
  uint32_t first, step, end;
};
AMS_DEV ItemRange xcd_items(uint32_t total) {
  uint32_t G = gridDim.x, b = blockIdx.x;
  ItemRange r;
  if ((G & 7u) != 0 || total < G) {
    r.first = b;
    r.step = G;
    r.end = total;
    return r;
  }
  uint32_t x = b & 7u, j = b >> 3, G8 = G >> 3;
  uint32_t chunk = (total + 7u) >> 3;
  uint32_t lo = x * chunk;
  uint32_t hi = lo + chunk < total ? lo + chunk : total;
  r.first = lo + j;
  r.step = G8;
  r.end = hi;
  return r;
}

// One item per workgroup, for grids of 8 * ceil(total / 8) or more
// workgroups: workgroup b takes item j = b / 8 of the contiguous eighth of
// the items that XCD x = b mod 8 owns (an empty range past the items).  The
// hardware hands the workgroups out as earlier ones finish, which balances
// items of unequal sizes.
AMS_DEV ItemRange xcd_item(uint32_t total) {
  const uint32_t b = blockIdx.x, x = b & 7u, j = b >> 3;
  const uint32_t chunk = (total + 7u) >> 3;
  const uint32_t g = x * chunk + j;
  ItemRange r;
  r.first = g;
  r.step = 1;
  r.end = (j < chunk && g < total) ? g + 1 : g;
  return r;
}

// Largest i in [0, n) with prefix[i] <= g (prefix non-decreasing, prefix[0] = 0).
AMS_DEV uint32_t find_owner(const uint32_t *prefix, uint32_t n, uint32_t g) {
  uint32_t lo = 0, hi = n;  // answer in [lo, hi)
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
AMS_DEV uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += y;
  }
  return v;
}

// In-place exclusive scan of a[0..n) by a block of NT threads; tmp holds at
// least NT/64 words of LDS.  Every thread scans a contiguous run, runs are
// combined by a wavefront scan and one exchange of per-wave totals.  Returns
// the total.  Ends with a barrier.
template <int NT> AMS_DEV uint32_t block_exscan(uint32_t *a, uint32_t n, uint32_t *tmp) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  constexpr uint32_t NW = NT / 64;
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t lo = tid * per < n ? tid * per : n;
  const uint32_t hi = lo + per < n ? lo + per : n;
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += a[i];
  const uint32_t incl = wave_incl_scan(s);
  if (lane == 63) tmp[wave] = incl;
  __syncthreads();
  uint32_t off = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < NW; ++w) {
    const uint32_t t = tmp[w];
    off += w < wave ? t : 0u;
    total += t;
  }
  uint32_t run = off + incl - s;
  for (uint32_t i = lo; i < hi; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

}  // namespace ams
