// Adaptive multi-level sample sort (Section 6) on gfx950: level kernels, the
// base-case kernel, planning and launch.
//
// One level runs over every active subproblem at once:
//   k_plan           tile / sample-block prefix sums over the active list
//   k_sample_blocks  random sample (with replacement), blocks of 256 ranked by
//                    comparing all pairs (Section 4.2)
//   k_sample_rank    rank across the sorted blocks by binary search (the merge
//                    step of Section 4.2); the elements of rank j*a-1 become the
//                    splitters, stored sorted and as an Eytzinger tree
//   k_count          classify every key against the tree held in LDS (with the
//                    equality buckets of Appendix D when splitters repeat) and
//                    count per tile with per-wavefront LDS histograms
//   k_block_reduce   histograms summed over blocks of tiles
//   k_pack           bucket totals; optimal grouping of buckets into at most r
//                    groups (Section 6 and its lemma; Appendix C search);
//                    children in key order; per-block child offsets
//   k_tile_scan      per-tile start offset of every child (child-major,
//                    tile-minor exclusive scan: Section 4.3 prefix sums)
//   k_scatter        stable scatter of every key into its child through LDS
// and the leaves are finished by k_finish: in-LDS split with a small sampled
// splitter set, then all-pairs ranking inside every small bucket.
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ams_engine.h"

namespace ams {

// ---------------------------------------------------------------------------
// device state
// ---------------------------------------------------------------------------
struct Ctr {
  uint32_t nact[MAXLEV + 1];
  uint32_t nleaf;
  uint32_t P, ntile, nblk, nsblk;
  uint32_t overflow;  // AMS_DEVERR_* bits raised by this run
  uint32_t nbig;      // oversized leaves (merge fallback)
  uint32_t L;         // partition levels of the plan
  // statistics of the run, per level (ams_workspace_stats)
  uint32_t lv_sub[MAXLEV];       // subproblems partitioned
  uint32_t lv_maxchild[MAXLEV];  // largest regular child produced
  uint32_t lv_imb_max[MAXLEV];   // max of L* / ceil(W / r), 16.16 fixed point
  uint32_t lv_tiles[MAXLEV];     // tiles of the level pass
  uint32_t nmerge;               // ranges the merge fallback sorted
  uint32_t nbl;                  // entries of the oversized-leaf list
  uint32_t nrest;                // entries of the remainder list (k_big_rest)
  uint32_t finNext;              // leaves k_finish handed out after the first gridDim.x
  uint32_t pad0;
  unsigned long long lv_keys[MAXLEV];     // keys in the partitioned subproblems
  unsigned long long lv_final[MAXLEV];    // keys placed in final children
  unsigned long long lv_imb_sum[MAXLEV];  // sum of the ratio over subproblems
  unsigned long long leaf_keys[3];        // keys in leaves, by leaf kind
  unsigned long long merge_keys;          // keys the merge fallback sorted
};
static_assert(sizeof(Ctr) % 8 == 0 && offsetof(Ctr, lv_keys) % 8 == 0, "Ctr layout");

// Every device error any run on this device has raised since the host last
// cleared it (ams_device_errors): sort calls on caller streams return before
// their kernels run, so a table bound exceeded on the device is recorded
// here as well as in the run's own counters.
__device__ uint32_t g_dev_errors;

AMS_DEV void raise_error(Ctr *c, uint32_t bits) {
  atomicOr(&c->overflow, bits);
  atomicOr(&g_dev_errors, bits);
}

// The buckets a group of one level brings to the next level (the paper's
// overpartitioning, Section 6: a group holds about b consecutive buckets of
// known size).  Up to STRATA_MAX strata of consecutive buckets, each with
// its exact key count; stratum j holds the keys x with thr[j-1] < x <=
// thr[j] (ord values; the last stratum is unbounded above).
constexpr uint32_t STRATA_MAX = 16;
struct Strata {
  uint64_t thr[STRATA_MAX];
  uint32_t cnt[STRATA_MAX];
  uint32_t k;  // strata (0: none recorded)
  uint32_t pad;
};

struct Ws {
  Root *roots;
  uint32_t nroots;
  void *tmpK;
  uint32_t *tmpV;
  Ctr *ctr;
  Seg *act[MAXLEV + 1];
  uint32_t capAct[MAXLEV + 1];
  Seg *leaves;
  uint32_t capLeaf;
  Seg *bigLeaves;  // capBig oversized leaves (k_big_part), then 2 capBig remainder entries
  uint32_t capBig;
  uint32_t *tileStart, *blkStart, *sampStart;
  void *samp, *spl, *tree;
  uint8_t *eqOn;
  uint32_t *hist, *blkHist, *totals, *tileOff;
  uint16_t *i2c, *cfirst;
  uint32_t *cstart;
  uint8_t *cdst;
  uint32_t *nch;
  Strata *strata;  // per active subproblem of the next level: its parent buckets
  uint32_t capTile, capBlk, capSBlk;
  uint32_t *dbgHist, *dbgChildren, *dbgNChild;
  uint64_t *sink;  // SINK_WORDS words that stores of empty slots go to (never read)
};

struct Lev {
  uint32_t level, L, last, shrink;
  uint32_t rmax, b, a, mmax, Smax, TC, TB, HS, CH, rankG;
  uint32_t C, flags, Scap;
  uint32_t strata;      // this level's splitters follow the strata its subproblems carry
  uint32_t strataNext;  // the grouping records strata for the next level
  uint32_t kw;          // key bytes
  uint32_t capTile, capBlk, capSBlk;  // the level's table capacities
  uint64_t seed;
};

struct LevTable {
  Lev l[MAXLEV];
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
AMS_HD uint32_t ilog2c(uint32_t x) {  // ceil(log2 x), x >= 1
  uint32_t l = 0;
  while ((1u << l) < x) ++l;
  return l;
}

// Shape of one subproblem of N keys: r groups (the paper's r), m = b*r buckets
// and a sample of S = a*m keys (whole blocks of 256, at most Scap).  With
// `shrink`, the number of groups is cut to what the base case needs (about
// C/2 keys per group), so small subproblems are not over-partitioned.
AMS_HD void seg_shape(uint32_t N, uint32_t C, bool shrink, uint32_t rmax,
                                       uint32_t b, uint32_t a, uint32_t Scap, uint32_t &logr,
                                       uint32_t &logm, uint32_t &S) {
  uint32_t r = rmax;
  if (shrink) {
    uint64_t need = (2ull * N + C - 1) / C;
    r = 2;
    while (r < need && r < rmax) r <<= 1;
    if (r > rmax) r = rmax;
  }
  uint32_t m = r * b;
  if (m > 2048) m = 2048;
  if (m < 2) m = 2;
  logr = ilog2c(r);
  logm = ilog2c(m);
  uint64_t s = (uint64_t)a * m;
  s = (s + 255) & ~255ull;
  if (s > Scap) s = Scap;
  S = (uint32_t)s;
}

AMS_DEV uint32_t meta_logm(uint32_t meta) { return (meta >> 12) & 15u; }
AMS_DEV uint32_t meta_logr(uint32_t meta) { return (meta >> 16) & 15u; }
AMS_HD uint32_t make_meta(uint32_t buf, uint32_t kind, uint32_t dst,
                                          uint32_t logm, uint32_t logr) {
  return buf | (kind << 4) | (dst << 8) | (logm << 12) | (logr << 16);
}

// Buffer the children of a subproblem go to.  Read from the caller's input,
// the first level writes the output buffer when an odd number of levels
// remain (so the last level lands in the output) and input and output do not
// alias; later levels alternate between TMP and OUT.
AMS_HD uint32_t dst_for(uint32_t buf, bool inplace, uint32_t L, uint32_t lv) {
  if (buf == BUF_IN) return (((L - lv) & 1u) && !inplace) ? BUF_OUT : BUF_TMP;
  return buf == BUF_TMP ? BUF_OUT : BUF_TMP;
}

AMS_DEV bool root_inplace(const Root &R) {
  return R.kin == (const void *)R.kout || (R.vin != nullptr && R.vin == R.vout);
}

template <typename K> AMS_DEV K *kptr(const Ws &w, const Root &R, uint32_t buf) {
  if (buf == BUF_IN) return (K *)R.kin;
  if (buf == BUF_OUT) return (K *)R.kout;
  return (K *)w.tmpK + R.tmp_off;
}
AMS_DEV uint32_t *vptr(const Ws &w, const Root &R, uint32_t buf) {
  if (buf == BUF_IN) return (uint32_t *)R.vin;
  if (buf == BUF_OUT) return R.vout;
  return w.tmpV + R.tmp_off;
}

// Leaf counts of one thread, summed per wavefront before they reach the
// run's counters (flush_place_stats), so that tens of thousands of leaves
// do not serialise on a few atomics.
struct PlaceStats {
  unsigned long long leafKeys[3];  // by leaf kind
  uint32_t big;
};

AMS_DEV PlaceStats no_place_stats() { return PlaceStats{{0, 0, 0}, 0}; }

// Call from uniform control flow (every lane of the wavefront).
AMS_DEV void flush_place_stats(const Ws &w, const PlaceStats &ps) {
  unsigned long long k[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) k[i] = wave_sum(ps.leafKeys[i]);
  const uint32_t big = wave_sum(ps.big);
  if (lane_id() == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (k[i]) atomicAdd(&w.ctr->leaf_keys[i], k[i]);
    if (big) atomicAdd(&w.ctr->nbig, big);
  }
}

AMS_DEV void push_leaf(const Ws &w, Seg s, PlaceStats &ps) {
  const uint32_t kind = seg_kind(s.meta);
  if (kind == LEAF_BIG) {
    const uint32_t slot = atomicAdd(&w.ctr->nbl, 1u);
    if (slot < w.capBig) w.bigLeaves[slot] = s; else raise_error(w.ctr, 1u);
  } else {
    const uint32_t slot = atomicAdd(&w.ctr->nleaf, 1u);
    if (slot < w.capLeaf) w.leaves[slot] = s; else raise_error(w.ctr, 1u);
  }
  ps.leafKeys[kind < 3 ? kind : 0] += s.size;
  ps.big += kind == LEAF_BIG ? 1u : 0u;
}

// A root or child of N keys entering level lv: a leaf when it fits the base
// case, an oversized leaf when no partition level is left, otherwise an
// active subproblem of level lv.
// Returns the subproblem's slot in the level's active list, or 0xFFFFFFFF
// when it became a leaf.
AMS_DEV uint32_t place_subproblem(const Ws &w, const LevTable &lt, uint32_t L, uint32_t lv,
                                  uint32_t off, uint32_t N, uint32_t root, uint32_t buf,
                                  bool inplace, uint32_t C, PlaceStats &ps) {
  if (N == 0) return 0xFFFFFFFFu;
  if (N <= C) {
    push_leaf(w, Seg{off, N, root, make_meta(buf, LEAF_REG, 0, 0, 0)}, ps);
    return 0xFFFFFFFFu;
  }
  if (lv >= L) {
    push_leaf(w, Seg{off, N, root, make_meta(buf, LEAF_BIG, 0, 0, 0)}, ps);
    return 0xFFFFFFFFu;
  }
  const Lev &l = lt.l[lv];
  uint32_t logr, logm, S;
  seg_shape(N, C, l.shrink != 0, l.rmax, l.b, l.a, l.Scap, logr, logm, S);
  uint32_t slot = atomicAdd(&w.ctr->nact[lv], 1u);
  Seg s{off, N, root, make_meta(buf, 0, dst_for(buf, inplace, L, lv), logm, logr)};
  if (slot < w.capAct[lv]) {
    w.act[lv][slot] = s;
    return slot;
  }
  raise_error(w.ctr, 1u);
  return 0xFFFFFFFFu;
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
__global__ void k_reset(Ws w) {
  uint32_t *p = (uint32_t *)w.ctr;
  for (uint32_t i = threadIdx.x; i < sizeof(Ctr) / 4; i += blockDim.x) p[i] = 0;
}

// mode 0: one root given by value; 1: contiguous segments of base arrays at
// device offsets; 2: root table already in the workspace.
__global__ void k_init_roots(Ws w, LevTable lt, uint32_t L, uint32_t C, int mode, Root single,
                             const char *kin, const uint32_t *vin, char *kout, uint32_t *vout,
                             const uint64_t *offs, uint32_t kw) {
  PlaceStats ps = no_place_stats();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < w.nroots;
       i += gridDim.x * blockDim.x) {
    Root R;
    if (mode == 0) {
      R = single;
    } else if (mode == 1) {
      uint64_t o = offs[i], e = offs[i + 1];
      R.kin = kin + o * kw;
      R.vin = vin ? vin + o : nullptr;
      R.kout = kout + o * kw;
      R.vout = vout ? vout + o : nullptr;
      R.n = e - o;
      R.tmp_off = o;
    } else {
      R = w.roots[i];
    }
    if (mode != 2) w.roots[i] = R;
    place_subproblem(w, lt, L, 0, 0, (uint32_t)R.n, i, BUF_IN, root_inplace(R), C, ps);
  }
  flush_place_stats(w, ps);
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctr->L = L;
}

// Prefix sums over the active list of a level: tiles, tile blocks, sample blocks.
__global__ void __launch_bounds__(1024) k_plan(Ws w, Lev lv) {
  __shared__ uint32_t tmp[1024];
  const uint32_t tid = threadIdx.x;
  uint32_t n = w.ctr->nact[lv.level];
  if (n > w.capAct[lv.level]) {
    if (tid == 0) raise_error(w.ctr, 2u);
    n = w.capAct[lv.level];
  }
  const Seg *act = w.act[lv.level];
  unsigned long long keys = 0;
  for (uint32_t i = tid; i < n; i += 1024) {
    Seg s = act[i];
    keys += s.size;
    uint32_t tiles = (s.size + lv.TC - 1) / lv.TC;
    w.tileStart[i] = tiles;
    w.blkStart[i] = (tiles + lv.TB - 1) / lv.TB;
    uint32_t logr, logm, S;
    seg_shape(s.size, lv.C, lv.shrink != 0, lv.rmax, lv.b, lv.a, lv.Scap, logr, logm, S);
    w.sampStart[i] = S / 256;
  }
  keys = wave_sum(keys);
  if ((tid & 63u) == 0 && keys) atomicAdd(&w.ctr->lv_keys[lv.level], keys);
  if (tid == 0) w.ctr->lv_sub[lv.level] = n;
  __syncthreads();
  uint32_t tt = block_exscan<1024>(w.tileStart, n, tmp);
  uint32_t tb = block_exscan<1024>(w.blkStart, n, tmp);
  uint32_t ts = block_exscan<1024>(w.sampStart, n, tmp);
  if (tid == 0) {
    w.tileStart[n] = tt;
    w.blkStart[n] = tb;
    w.sampStart[n] = ts;
    // capacities are upper bounds by construction; if one were exceeded the
    // level processes nothing (and the overflow flag is raised) rather than
    // index past its tables
    const bool over = tt > lv.capTile || tb > lv.capBlk || ts > lv.capSBlk;
    if (over) raise_error(w.ctr, 4u);
    w.ctr->lv_tiles[lv.level] = tt;
    w.ctr->P = over ? 0 : n;
    w.ctr->ntile = over ? 0 : tt;
    w.ctr->nblk = over ? 0 : tb;
    w.ctr->nsblk = over ? 0 : ts;
  }
}

// ---------------------------------------------------------------------------
// Sample (Section 6: a random sample of a*b*r keys), ranked inside blocks of
// 256 by comparing all pairs (Section 4.2), ties broken by sample index.
// ---------------------------------------------------------------------------
template <int KT> __global__ void __launch_bounds__(256) k_sample_blocks(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  __shared__ K sh[256];
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P, total = w.ctr->nsblk;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    uint32_t i = find_owner(w.sampStart, P, item);
    uint32_t j = item - w.sampStart[i];
    Seg s = w.act[lv.level][i];
    Root R = w.roots[s.root];
    uint32_t buf = seg_buf(s.meta);
    const K *src = kptr<K>(w, R, buf) + s.off;
    uint64_t st = stream_state(lv.seed, lv.level, s.root, s.off);
    K x = ((const GMem<K> *)src)[draw_pos(st, j * 256 + tid, s.size)];
    if (buf == BUF_IN) x = Key<KT>::enc(x);
    sh[tid] = x;
    __syncthreads();
    uint32_t rank = 0;
    for (uint32_t q = 0; q < 256; ++q) {
      K y = sh[q];
      rank += (uint32_t)(y < x) | ((uint32_t)(y == x) & (uint32_t)(q < tid));
    }
    ((K *)w.samp)[(size_t)i * lv.Smax + j * 256 + rank] = x;
    __syncthreads();
  }
}

// Rank every sample element across the sorted blocks (binary search: the
// merge step of Section 4.2; equal keys ordered by block, i.e. by sample
// index) and write the element of rank j*a-1 as splitter j (j = 1..m-1)
// into the sorted array and the Eytzinger tree.  Item = (subproblem, group
// of rankG blocks); unused item slots exit at once.
template <int KT> __global__ void __launch_bounds__(256) k_sample_rank(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  K *sh = (K *)smem_raw;
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P;
  const uint32_t G = lv.rankG;
  const uint32_t ngMax = (lv.Smax / 256 + G - 1) / G;
  const uint32_t total = P * ngMax;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    uint32_t i = item / ngMax, g = item - i * ngMax;
    uint32_t nb = w.sampStart[i + 1] - w.sampStart[i];
    if (g * G >= nb) continue;
    Seg s = w.act[lv.level][i];
    const uint32_t S = nb * 256;
    const uint32_t m = 1u << meta_logm(s.meta);
    const uint32_t a = S / m;
    const K *src = (const K *)w.samp + (size_t)i * lv.Smax;
    for (uint32_t q = tid; q < S; q += 256) sh[q] = src[q];
    __syncthreads();
    K *spl = (K *)w.spl + (size_t)i * lv.mmax;
    K *tree = (K *)w.tree + (size_t)i * lv.mmax;
    uint32_t jEnd = (g + 1) * G < nb ? (g + 1) * G : nb;
    for (uint32_t j = g * G; j < jEnd; ++j) {
      K x = sh[j * 256 + tid];
      uint32_t rank = tid;
      for (uint32_t jb = 0; jb < nb; ++jb) {
        if (jb == j) continue;
        const K *blk = sh + jb * 256;
        rank += (jb < j) ? count_less_eq(blk, 256u, x) : count_less(blk, 256u, x);
      }
      if ((rank + 1) % a == 0) {
        uint32_t sp = (rank + 1) / a;
        if (sp >= 1 && sp <= m - 1) {
          spl[sp - 1] = x;
          tree[eytzinger_slot(sp, m)] = x;
        }
      }
    }
    __syncthreads();
  }
}

// Splitters of a subproblem that carries strata from the level above
// (exploiting the overpartitioning in the recursion, Section 6): the sample
// is sorted whole, the m buckets are shared among the strata in proportion
// to their exact key counts, every stratum boundary becomes a splitter, and
// each stratum's own buckets take equidistant ranks of the sample keys that
// fall into it.  Without strata this is the plain rule (rank j*a - 1).  One
// workgroup per subproblem.
template <int KT> __global__ void __launch_bounds__(256) k_sample_strata(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ uint32_t sR[STRATA_MAX + 1], sM[STRATA_MAX + 1];
  __shared__ K sT[STRATA_MAX];
  __shared__ uint32_t sk;
  K *sh = (K *)smem_raw;
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P;
  for (uint32_t i = blockIdx.x; i < P; i += gridDim.x) {
    const uint32_t nb = w.sampStart[i + 1] - w.sampStart[i];
    const Seg s = w.act[lv.level][i];
    const uint32_t S = nb * 256;
    const uint32_t m = 1u << meta_logm(s.meta);
    K *srt = sh + lv.Smax;
    const K *src = (const K *)w.samp + (size_t)i * lv.Smax;
    for (uint32_t q = tid; q < S; q += 256) sh[q] = src[q];
    __syncthreads();
    // the whole sample sorted: rank across the sorted blocks (equal keys by
    // block, then by position), each element written at its rank
    for (uint32_t q = tid; q < S; q += 256) {
      const uint32_t j = q >> 8;
      const K x = sh[q];
      uint32_t rank = q & 255u;
      for (uint32_t jb = 0; jb < nb; ++jb) {
        if (jb == j) continue;
        const K *blk = sh + jb * 256;
        rank += (jb < j) ? count_less_eq(blk, 256u, x) : count_less(blk, 256u, x);
      }
      srt[rank] = x;
    }
    // strata: thresholds, sample keys below each, buckets per stratum
    if (tid == 0) {
      const Strata *st = w.strata + i;
      uint32_t k = lv.strata ? st->k : 0u;
      if (k == 0) k = 1;
      uint64_t cum = 0;
      const uint64_t N = s.size;
      sM[0] = 0;
      for (uint32_t b = 0; b < k; ++b) {
        const uint32_t c = k == 1 ? s.size : st->cnt[b];
        cum += c;
        sM[b + 1] = b + 1 == k ? m : (uint32_t)((cum * m) / N);
        if (b + 1 < k) sT[b] = (K)st->thr[b];
      }
      // every stratum keeps at least one bucket (its upper boundary)
      for (uint32_t b = 1; b <= k; ++b)
        if (sM[b] <= sM[b - 1]) sM[b] = sM[b - 1] + 1;
      if (sM[k] > m) k = 1, sM[1] = m;  // cannot happen with the strata's sizes
      sk = k;
    }
    __syncthreads();
    const uint32_t k = sk;
    // sample keys in strata below b: those <= thr[b-1]
    for (uint32_t b = tid; b <= k; b += 256) {
      if (b == 0) sR[0] = 0;
      else if (b == k) sR[k] = S;
      else {
        uint32_t lo = 0, hi = S;  // first rank with srt > thr
        const K t = sT[b - 1];
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (srt[mid] <= t) lo = mid + 1; else hi = mid;
        }
        sR[b] = lo;
      }
    }
    __syncthreads();
    K *spl = (K *)w.spl + (size_t)i * lv.mmax;
    K *tree = (K *)w.tree + (size_t)i * lv.mmax;
    for (uint32_t sp = 1 + tid; sp < m; sp += 256) {
      uint32_t b = 0;  // stratum owning slot sp: sM[b] < sp <= sM[b+1]
      while (b + 1 < k && sM[b + 1] < sp) ++b;
      K x;
      if (sp == sM[b + 1] && b + 1 < k) {
        x = sT[b];  // the stratum's upper boundary
      } else {
        const uint32_t mb = sM[b + 1] - sM[b], sb = sR[b + 1] - sR[b];
        const uint32_t ii = sp - sM[b];  // 1 .. mb-1
        if (sb) {
          const uint32_t r = (uint32_t)(((uint64_t)ii * sb + mb - 1) / mb);  // ceil(ii sb / mb)
          x = srt[sR[b] + (r ? r - 1 : 0)];
        } else {
          x = b + 1 < k ? sT[b] : (b ? sT[b - 1] : srt[S - 1]);
        }
      }
      spl[sp - 1] = x;
      tree[eytzinger_slot(sp, m)] = x;
    }
    __syncthreads();
  }
}

// Splitters given by the caller (step entry point): sorted ord values.
template <int KT> __global__ void k_set_splitters(Ws w, Lev lv, const void *given) {
  typedef typename Key<KT>::T K;
  if (w.ctr->P == 0) return;
  Seg s = w.act[0][0];
  uint32_t m = 1u << meta_logm(s.meta);
  const K *g = (const K *)given;
  K *spl = (K *)w.spl;
  K *tree = (K *)w.tree;
  for (uint32_t j = threadIdx.x; j + 1 < m; j += blockDim.x) {
    spl[j] = g[j];
    tree[eytzinger_slot(j + 1, m)] = g[j];
  }
}

// ---------------------------------------------------------------------------
// Classification and per-tile histograms (Section 6: partition into b*r
// buckets; Appendix D: equality buckets when splitters repeat).
// ---------------------------------------------------------------------------
template <typename K>
AMS_DEV bool load_tree(const Ws &w, const Lev &lv, uint32_t i, uint32_t m, K *sTree, K *sSpl) {
  const K *gt = (const K *)w.tree + (size_t)i * lv.mmax;
  const K *gs = (const K *)w.spl + (size_t)i * lv.mmax;
  bool dup = false;
  for (uint32_t j = threadIdx.x; j < m; j += blockDim.x) {
    if (j >= 1) sTree[j] = gt[j];
    if (j + 1 < m) {
      K v = gs[j];
      if (sSpl) sSpl[j] = v;
      if (j + 2 < m && v == gs[j + 1]) dup = true;
    }
  }
  return __syncthreads_or(dup ? 1 : 0) || (lv.flags & AMS_FLAG_EQ_ALWAYS);
}

// Per-tile bucket counts.  One LDS histogram per workgroup (LDS atomics);
// every thread keeps CU keys in flight so that enough loads are outstanding to
// cover HBM latency.
template <int KT> __global__ void __launch_bounds__(256) k_count(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  constexpr int CU = 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  K *sTree = (K *)smem_raw;
  uint32_t *sH = (uint32_t *)(sTree + lv.mmax);  // NB
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P;
  const uint32_t ntile = w.ctr->ntile;
  ItemRange ir = xcd_item(ntile);  // one tile per workgroup
  // the grid covers every tile (the plan bounds the count); else flagged
  if (blockIdx.x == 0 && tid == 0 && 8u * ((ntile + 7u) / 8u) > gridDim.x) raise_error(w.ctr, 4u);
  uint32_t cur = 0xFFFFFFFFu;
  bool eq = false;
  uint32_t logm = 0, m = 0;
  for (uint32_t g = ir.first; g < ir.end; g += ir.step) {
    uint32_t i = find_owner(w.tileStart, P, g);
    uint32_t t = g - w.tileStart[i];
    Seg s = w.act[lv.level][i];
    if (i != cur) {
      __syncthreads();
      logm = meta_logm(s.meta);
      m = 1u << logm;
      eq = load_tree<K>(w, lv, i, m, sTree, nullptr);
      cur = i;
    }
    const uint32_t NB = eq ? 2 * m - 1 : m;
    for (uint32_t q = tid; q < NB; q += 256) sH[q] = 0;
    __syncthreads();
    Root R = w.roots[s.root];
    uint32_t buf = seg_buf(s.meta);
    const K *src = kptr<K>(w, R, buf) + s.off;
    const bool enc = buf == BUF_IN;
    uint32_t lo = t * lv.TC;
    uint32_t hi = lo + lv.TC < s.size ? lo + lv.TC : s.size;
    // the tile through a buffer resource: 16-byte loads, zeros past its end
    const Rsrc rs = make_rsrc(uniform_ptr(src + lo), (hi - lo) * (uint32_t)sizeof(K));
    constexpr uint32_t V = Vec16<K>::N;
    for (uint32_t base = lo; base < hi; base += 256 * CU) {
      K xs[CU];
#pragma unroll
      for (uint32_t k = 0; k < CU / V; ++k) {
        // whole offset in the vector operand, which the range check covers
        const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(
            rs, tid * 16u + (base - lo) * (uint32_t)sizeof(K) + k * (256u * 16u), 0, 0);
        Vec16<K>::get(v, &xs[k * V]);
      }
      if (enc) {
#pragma unroll
        for (int u = 0; u < CU; ++u) xs[u] = Key<KT>::enc(xs[u]);
      }
      uint32_t ids[CU];
      classify_batch<K, CU>(xs, ids, sTree, logm, eq);
      // one add for the whole wavefront when all its keys share a bucket
      // (sorted or skewed input), else one LDS atomic per key
      const uint32_t ntv = base + 256u * CU <= hi ? 256u * CU : hi - base;  // valid keys
      const uint64_t lanes = ballot(true);
      const uint32_t c0 = __builtin_amdgcn_readlane(ids[0], (uint32_t)__builtin_ctzll(lanes));
      bool same = true;
#pragma unroll
      for (uint32_t u = 0; u < CU; ++u) {
        const uint32_t p = base + (u / V) * (V * 256u) + V * tid + (u % V);
        same = same && (p >= hi || ids[u] == c0);
      }
      if (ballot(same) == lanes && ntv == 256u * CU) {
        if (tid % 64 == 0) atomicAdd(&sH[c0], 64u * CU);
      } else if (__popcll(ballot(ids[0] == __builtin_amdgcn_readfirstlane(ids[0]))) >= 32) {
        // clustered input (sorted runs): most lanes of a row share a bucket,
        // so each row adds once per bucket instead of once per key
#pragma unroll
        for (uint32_t u = 0; u < CU; ++u) {
          const uint32_t p = base + (u / V) * (V * 256u) + V * tid + (u % V);
          wave_count_add(sH, ids[u], p < hi);
        }
      } else {
#pragma unroll
        for (uint32_t u = 0; u < CU; ++u) {
          const uint32_t p = base + (u / V) * (V * 256u) + V * tid + (u % V);
          if (p < hi) atomicAdd(&sH[ids[u]], 1u);
        }
      }
    }
    __syncthreads();
    uint32_t *gh = w.hist + (size_t)g * lv.HS;
    for (uint32_t id = tid; id < NB; id += 256) gh[id] = sH[id];
    if (t == 0 && tid == 0) w.eqOn[i] = eq ? 1 : 0;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_block_reduce(Ws w, Lev lv) {
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P;
  // item = (tile block, 256 bucket ids)
  const uint32_t chunks = (lv.HS + 255) / 256, total = w.ctr->nblk * chunks;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    const uint32_t B = item / chunks, ch = item - B * chunks;
    uint32_t i = find_owner(w.blkStart, P, B);
    uint32_t bb = B - w.blkStart[i];
    uint32_t t0 = w.tileStart[i] + bb * lv.TB;
    uint32_t t1 = t0 + lv.TB < w.tileStart[i + 1] ? t0 + lv.TB : w.tileStart[i + 1];
    Seg s = w.act[lv.level][i];
    uint32_t m = 1u << meta_logm(s.meta);
    uint32_t NB = w.eqOn[i] ? 2 * m - 1 : m;
    const uint32_t id = ch * 256 + tid;
    if (id < NB) {
      // 16 tile rows in flight at a time
      uint32_t sum = 0;
      const uint32_t *h = w.hist + (size_t)t0 * lv.HS + id;
      uint32_t t = t0;
      for (; t + 16 <= t1; t += 16, h += 16 * (size_t)lv.HS) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = h[(size_t)u * lv.HS];
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += v[u];
      }
      for (; t < t1; ++t, h += lv.HS) sum += *h;
      w.blkHist[(size_t)B * lv.HS + id] = sum;
    }
  }
}

// Per subproblem and bucket id: exclusive prefix over its tile blocks (in
// place in blkHist) and the total (bucket size).  Item = (subproblem, 256 ids).
__global__ void __launch_bounds__(256) k_block_scan(Ws w, Lev lv) {
  const uint32_t P = w.ctr->P;
  const uint32_t chunks = (lv.HS + 255) / 256;
  const uint32_t total = P * chunks;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    const uint32_t i = item / chunks;
    const uint32_t id = (item - i * chunks) * 256 + threadIdx.x;
    const uint32_t m = 1u << meta_logm(w.act[lv.level][i].meta);
    const uint32_t NB = w.eqOn[i] ? 2 * m - 1 : m;
    if (id >= NB) continue;
    const uint32_t b0 = w.blkStart[i], nbk = w.blkStart[i + 1] - b0;
    uint32_t *col = w.blkHist + (size_t)b0 * lv.HS + id;
    uint32_t run = 0;
    uint32_t bb = 0;
    for (; bb + 8 <= nbk; bb += 8) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[(size_t)(bb + u) * lv.HS];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        col[(size_t)(bb + u) * lv.HS] = run;
        run += v[u];
      }
    }
    for (; bb < nbk; ++bb) {
      uint32_t v = col[(size_t)bb * lv.HS];
      col[(size_t)bb * lv.HS] = run;
      run += v;
    }
    w.totals[(size_t)i * lv.HS + id] = run;
  }
}

// ---------------------------------------------------------------------------
// Bucket grouping (Section 6: scan the bucket sizes, open the next group
// when the load would exceed L; smallest feasible L by search, optimal by the
// section's lemma.  Appendix C: many candidates per round, the bounds moved to
// the largest group of a feasible scan and to the smallest overflowing group
// of an infeasible one).
// ---------------------------------------------------------------------------
struct Greedy {
  bool feasible;
  uint32_t maxG, zmin;
};

// wgt is 16-byte aligned and padded with zeros to a multiple of 8 entries;
// eight weights are fetched per step so the scan is not bound by LDS latency
// (zero weights never open a group).
AMS_DEV Greedy greedy_scan(const uint32_t *wgt, uint32_t nb, uint32_t L, uint32_t r) {
  uint32_t cur = 0, groups = 1, maxG = 0, zmin = 0xFFFFFFFFu;
  const uint4 *w4 = (const uint4 *)wgt;
  const uint32_t n8 = (nb + 7) / 8;
  for (uint32_t j = 0; j < n8; ++j) {
    const uint4 a = w4[2 * j], b = w4[2 * j + 1];
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int u = 0; u < 8; ++u) {  // branch-free: selects only
      const uint32_t t = cur + v[u];
      const bool o = t > L;
      zmin = o ? min(zmin, t) : zmin;
      maxG = o ? max(maxG, cur) : maxG;
      groups += o ? 1u : 0u;
      cur = o ? v[u] : t;
    }
  }
  maxG = max(maxG, cur);
  return Greedy{groups <= r, maxG, zmin};
}

// L* for weights wgt[0..nb) and at most r groups, by a block of NT threads.
// red: 2*NT/64 words of LDS.
template <int NT>
AMS_DEV uint32_t optimal_load(const uint32_t *wgt, uint32_t nb, uint32_t r, uint32_t *red,
                              uint32_t *Wout = nullptr) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr uint32_t NW = NT / 64;
  uint32_t W = 0, mx = 0;
  for (uint32_t j = tid; j < nb; j += NT) {
    W += wgt[j];
    mx = max(mx, wgt[j]);
  }
  W = wave_sum(W);
  mx = wave_max(mx);
  if (lane == 0) {
    red[wave] = W;
    red[NW + wave] = mx;
  }
  __syncthreads();
  W = 0;
  mx = 0;
  for (uint32_t q = 0; q < NW; ++q) {
    W += red[q];
    mx = max(mx, red[NW + q]);
  }
  __syncthreads();
  if (Wout) *Wout = W;
  uint32_t avg = (uint32_t)(((uint64_t)W + r - 1) / r);
  // L* <= avg + mx (under that load every group the greedy closes holds more
  // than avg, so there are at most r) and L* <= W (one group holds all); the
  // sum is formed in 64 bits: with few groups and one heavy bucket it can
  // pass 2^32 while W cannot
  uint32_t lo = max(mx, avg);
  uint32_t hi = (uint32_t)min((uint64_t)avg + mx, (uint64_t)W);
  while (lo < hi) {
    uint32_t span = hi - lo;
    bool active;
    uint32_t cand;
    if (span <= NT) {
      active = tid < span;
      cand = lo + tid;
    } else {
      active = true;
      cand = lo + (uint32_t)(((uint64_t)span * (tid + 1)) / (NT + 1));
    }
    uint32_t newHi = 0xFFFFFFFFu, newLo = 0;
    if (active) {
      Greedy gr = greedy_scan(wgt, nb, cand, r);
      if (gr.feasible) newHi = gr.maxG; else newLo = gr.zmin;
    }
    newHi = wave_min(newHi);
    newLo = wave_max(newLo);
    if (lane == 0) {
      red[wave] = newHi;
      red[NW + wave] = newLo;
    }
    __syncthreads();
    for (uint32_t q = 0; q < NW; ++q) {
      hi = min(hi, red[q]);
      lo = max(lo, red[NW + q]);
    }
    __syncthreads();
  }
  return lo;
}

struct PackSmem {
  uint32_t *tot, *wgt, *sz, *start, *tmp, *red;
  uint16_t *first, *end;
  uint8_t *fin, *kind;
  uint32_t *aux;  // HS + 1 words of scan space
  uint16_t *pst;  // HS + 1 piece starts
  uint8_t *gs;    // HS + 8 flags: the greedy opens a group at this id
  uint32_t *nzr;  // 2 (CH + 1) words: per child, first and end of its nonempty ids
};

AMS_HD size_t pack_al16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS layout of k_pack (byte offsets rounded to 16); returns the total size
AMS_HD size_t pack_layout(uint32_t HS, uint32_t CH, size_t *o) {
  size_t b = 0;
  o[0] = b; b = pack_al16(b + (size_t)HS * 4);            // tot
  o[1] = b; b = pack_al16(b + ((size_t)HS + 8) * 4);      // wgt, zero-padded to 8
  o[2] = b; b = pack_al16(b + ((size_t)CH + 1) * 4);      // sz
  o[3] = b; b = pack_al16(b + ((size_t)CH + 1) * 4);      // start
  o[4] = b; b = pack_al16(b + 256 * 4);                   // tmp
  o[5] = b; b = pack_al16(b + 16 * 4);                    // red
  o[6] = b; b = pack_al16(b + ((size_t)CH + 1) * 2);      // first
  o[7] = b; b = pack_al16(b + ((size_t)CH + 1) * 2);      // end
  o[8] = b; b = pack_al16(b + ((size_t)HS + 1) * 4);      // aux
  o[9] = b; b = pack_al16(b + ((size_t)HS + 1) * 2);      // pst
  o[10] = b; b = pack_al16(b + HS);                       // fin
  o[11] = b; b = pack_al16(b + CH);                       // kind
  o[12] = b; b = pack_al16(b + (size_t)HS + 8);           // gs
  o[13] = b; b = pack_al16(b + 2 * ((size_t)CH + 1) * 4); // nzr
  return b;
}

AMS_DEV PackSmem pack_smem(unsigned char *base, uint32_t HS, uint32_t CH) {
  size_t o[14];
  pack_layout(HS, CH, o);
  PackSmem p;
  p.tot = (uint32_t *)(base + o[0]);
  p.wgt = (uint32_t *)(base + o[1]);
  p.sz = (uint32_t *)(base + o[2]);
  p.start = (uint32_t *)(base + o[3]);
  p.tmp = (uint32_t *)(base + o[4]);
  p.red = (uint32_t *)(base + o[5]);
  p.first = (uint16_t *)(base + o[6]);
  p.end = (uint16_t *)(base + o[7]);
  p.aux = (uint32_t *)(base + o[8]);
  p.pst = (uint16_t *)(base + o[9]);
  p.fin = base + o[10];
  p.kind = base + o[11];
  p.gs = base + o[12];
  p.nzr = (uint32_t *)(base + o[13]);
  return p;
}

// Children of one subproblem from its id totals (p.tot), weights (p.wgt)
// and final flags (p.fin), by the whole block of NT threads:
//  1. one lane runs the greedy under L and flags the ids that open a group
//     (final ids weigh 0 and never open one);
//  2. pieces start at id 0, at group starts, at every final id and right
//     after it; a final id is a child of its own (CHILD_FINAL), any other
//     piece is a CHILD_REG child if it holds keys and is dropped otherwise
//     (its ids then fall to the child before it).
// Returns the number of children; p.aux[NB] holds the total key count.
template <int NT>
AMS_DEV uint32_t build_children(const PackSmem &p, uint32_t NB, uint32_t L, uint32_t CH) {
  const uint32_t tid = threadIdx.x;
  if (tid == 0) {
    uint32_t cur = 0;
    const uint4 *w4 = (const uint4 *)p.wgt;
    for (uint32_t j0 = 0; j0 < NB; j0 += 8) {
      const uint4 a = w4[j0 / 4], b = w4[j0 / 4 + 1];
      const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      uint32_t bits = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t t = cur + v[u];
        const bool o = t > L;
        cur = o ? v[u] : t;
        bits |= (o ? 1u : 0u) << (8 * (u & 3));
        if (u == 3 || u == 7) {
          *(uint32_t *)(p.gs + j0 + (u & 4)) = bits;  // gs is 4-byte aligned
          bits = 0;
        }
      }
    }
  }
  __syncthreads();
  // piece starts, numbered by a scan
  for (uint32_t j = tid; j < NB; j += NT)
    p.aux[j] = (j == 0 || p.gs[j] || p.fin[j] || p.fin[j - 1]) ? 1u : 0u;
  __syncthreads();
  const uint32_t np = block_exscan<NT>(p.aux, NB, p.tmp);
  for (uint32_t j = tid; j < NB; j += NT)
    if (j == 0 || p.gs[j] || p.fin[j] || p.fin[j - 1]) p.pst[p.aux[j]] = (uint16_t)j;
  if (tid == 0) p.pst[np] = (uint16_t)NB;
  // key counts before every id
  for (uint32_t j = tid; j < NB; j += NT) p.aux[j] = p.tot[j];
  __syncthreads();
  const uint32_t total = block_exscan<NT>(p.aux, NB, p.tmp);
  if (tid == 0) p.aux[NB] = total;
  __syncthreads();
  // kept pieces, numbered by a scan over the pieces (p.start as space)
  for (uint32_t q = tid; q < np; q += NT) {
    const uint32_t a = p.pst[q], b = p.pst[q + 1];
    p.start[q] = (p.fin[a] || p.aux[b] > p.aux[a]) ? 1u : 0u;
  }
  __syncthreads();
  // pieces number at most 3r = CH: r groups, r final ids (each holds at
  // least N/r keys), and the pieces right after final ids
  const uint32_t nch = block_exscan<NT>(p.start, np < CH ? np : CH, p.tmp);
  for (uint32_t q = tid; q < np && q < CH; q += NT) {
    const uint32_t a = p.pst[q], b = p.pst[q + 1];
    const bool fin = p.fin[a] != 0;
    if (fin || p.aux[b] > p.aux[a]) {
      const uint32_t c = p.start[q];
      p.first[c] = (uint16_t)a;
      p.end[c] = (uint16_t)b;
      p.sz[c] = p.aux[b] - p.aux[a];
      p.kind[c] = fin ? CHILD_FINAL : CHILD_REG;
    }
  }
  __syncthreads();
  return np <= CH ? nch : CH + 1;  // CH + 1: cannot happen, reported as an overflow
}

// Strata of one group for the next level: its consecutive bucket ids
// [f, e) cut greedily into at most STRATA_MAX runs of about size /
// STRATA_MAX keys each (a short last run joins the one before).  The cut
// before id j is a key threshold: without equality buckets id j holds
// s_j < x <= s_{j+1}, so ids below j hold x <= s_j; with them, ids below
// 2b+1 hold x < s_{b+1} and ids below 2b+2 hold x <= s_{b+1}.
template <typename K>
AMS_DEV void record_strata_t(const Ws &w, const Lev &lv, uint32_t i, uint32_t m, bool eq,
                             const uint32_t *tot, uint32_t f, uint32_t e, uint32_t size,
                             uint32_t slot) {
  const K *spl = (const K *)w.spl + (size_t)i * lv.mmax;
  Strata *st = w.strata + slot;
  const uint32_t target = (size + STRATA_MAX - 1) / STRATA_MAX;
  uint32_t k = 0, acc = 0;
  for (uint32_t id = f; id < e; ++id) {
    acc += tot[id];
    if (acc >= target && k + 1 < STRATA_MAX && id + 1 < e) {
      // threshold before id + 1
      const uint32_t j = id + 1;
      bool ok = true;
      uint64_t thr;
      if (!eq) {
        thr = (uint64_t)spl[j - 1];
      } else if (j & 1u) {  // j = 2b+1: ids below hold x < s_{b+1}
        const K v = spl[j >> 1];
        ok = v != 0;
        thr = (uint64_t)v - 1;
      } else {  // j = 2b+2: ids below hold x <= s_{b+1}
        thr = (uint64_t)spl[(j >> 1) - 1];
      }
      if (ok) {
        st->thr[k] = thr;
        st->cnt[k] = acc;
        ++k;
        acc = 0;
      }
    }
  }
  st->cnt[k] = acc;
  ++k;
  // a last stratum of less than half the target joins the one before
  if (k >= 2 && st->cnt[k - 1] < target / 2) {
    st->cnt[k - 2] += st->cnt[k - 1];
    --k;
  }
  st->k = k;
  (void)m;
}

AMS_DEV void record_strata(const Ws &w, const Lev &lv, uint32_t i, uint32_t m, bool eq,
                           const uint32_t *tot, uint32_t f, uint32_t e, uint32_t size,
                           uint32_t slot) {
  if (lv.kw == 8) record_strata_t<uint64_t>(w, lv, i, m, eq, tot, f, e, size, slot);
  else record_strata_t<uint32_t>(w, lv, i, m, eq, tot, f, e, size, slot);
}

__global__ void __launch_bounds__(256) k_pack(Ws w, Lev lv, LevTable lt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t HS = lv.HS, CH = lv.CH;
  PackSmem p = pack_smem(smem_raw, HS, CH);
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P;
  for (uint32_t i = blockIdx.x; i < P; i += gridDim.x) {
    Seg s = w.act[lv.level][i];
    Root R = w.roots[s.root];
    const uint32_t m = 1u << meta_logm(s.meta);
    const uint32_t r = 1u << meta_logr(s.meta);
    const bool eq = w.eqOn[i] != 0;
    const uint32_t NB = eq ? 2 * m - 1 : m;
    for (uint32_t id = tid; id < NB; id += 256) p.tot[id] = w.totals[(size_t)i * HS + id];
    __syncthreads();
    const uint32_t N = s.size;
    const uint32_t tfin = (N + r - 1) / r;
    for (uint32_t id = tid; id < ((NB + 7) & ~7u); id += 256) {
      bool fin = id < NB && eq && (id & 1u) && p.tot[id] >= tfin;
      if (id < NB) p.fin[id] = fin ? 1 : 0;
      p.wgt[id] = (fin || id >= NB) ? 0u : p.tot[id];
    }
    __syncthreads();
    uint32_t Wreg = 0;  // keys outside final children
    const uint32_t L = optimal_load<256>(p.wgt, NB, r, p.red, &Wreg);
    uint32_t nch = build_children<256>(p, NB, L, CH);
    if (nch > CH || p.aux[NB] != N) {  // cannot happen: at most 3r = CH children
      if (tid == 0) raise_error(w.ctr, 8u);
      nch = 0;
    }
    if (w.dbgHist && lv.level == 0 && i == 0) {
      for (uint32_t id = tid; id < NB; id += 256) w.dbgHist[id] = p.tot[id];
      for (uint32_t c = tid; c < nch; c += 256) {
        w.dbgChildren[4 * c] = p.first[c];
        w.dbgChildren[4 * c + 1] = p.end[c];
        w.dbgChildren[4 * c + 2] = p.sz[c];
        w.dbgChildren[4 * c + 3] = p.kind[c];
      }
      if (tid == 0) *w.dbgNChild = nch;
    }
    for (uint32_t c = tid; c < nch; c += 256) p.start[c] = p.sz[c];
    __syncthreads();
    block_exscan<256>(p.start, nch, p.tmp);
    // table ranges: child c owns ids [first_c, first_{c+1}); ids of dropped
    // empty pieces fall to the child before them (they hold no keys)
    if (tid == 0) {
      p.first[0] = 0;
      p.first[nch] = (uint16_t)NB;
    }
    __syncthreads();
    uint16_t *gF = w.cfirst + (size_t)i * 2 * (CH + 1);
    uint32_t *gS = w.cstart + (size_t)i * (CH + 1);
    uint8_t *gD = w.cdst + (size_t)i * CH;
    uint16_t *gI = w.i2c + (size_t)i * HS;
    const bool inplace = root_inplace(R);
    const uint32_t srcbuf = seg_buf(s.meta), dst = seg_dst(s.meta);
    const bool finToOut = srcbuf == BUF_TMP || (srcbuf == BUF_IN && !inplace);
    // id -> child map, and per child the range of ids that hold keys
    // (gF[2c], gF[2c+1]): a child can span many empty ids (all-equal or
    // heavily duplicated keys), which the tile scan then skips
    uint32_t *nzr = p.nzr;
    for (uint32_t c = tid; c < nch; c += 256) {
      nzr[2 * c] = 0xFFFFu;
      nzr[2 * c + 1] = 0;
    }
    __syncthreads();
    for (uint32_t id = tid; id < NB; id += 256) {
      uint32_t c = 0;  // the last child whose first id is <= id
      for (uint32_t span = 1u << ilog2c(nch + 1); span; span >>= 1)
        if (c + span < nch && p.first[c + span] <= id) c += span;
      gI[id] = (uint16_t)c;
      if (p.tot[id]) {
        atomicMin(&nzr[2 * c], id);
        atomicMax(&nzr[2 * c + 1], id + 1);
      }
    }
    __syncthreads();
    for (uint32_t c = tid; c < nch; c += 256) {
      const uint32_t a = nzr[2 * c], b = nzr[2 * c + 1];
      gF[2 * c] = (uint16_t)(a < b ? a : p.first[c]);
      gF[2 * c + 1] = (uint16_t)(a < b ? b : p.first[c]);
      gS[c] = p.start[c];
    }
    PlaceStats ps = no_place_stats();
    uint32_t maxChild = 0;
    for (uint32_t c = tid; c < nch; c += 256) {
      const uint32_t off = s.off + p.start[c], size = p.sz[c];
      uint32_t cd;
      if (p.kind[c] == CHILD_REG) {
        cd = dst;
        maxChild = size > maxChild ? size : maxChild;
        const uint32_t slot =
            place_subproblem(w, lt, lv.L, lv.level + 1, off, size, s.root, cd, inplace, lv.C, ps);
        if (lv.strataNext && slot != 0xFFFFFFFFu)
          record_strata(w, lv, i, m, eq, p.tot, p.first[c], p.end[c], size, slot);
      } else {
        cd = finToOut ? BUF_OUT : dst;
        if (cd != BUF_OUT) {
          uint32_t nc = (size + lv.C - 1) / lv.C;
          uint32_t slot = atomicAdd(&w.ctr->nleaf, nc);
          for (uint32_t q = 0; q < nc; ++q) {
            uint32_t o = q * lv.C;
            uint32_t sz = size - o < lv.C ? size - o : lv.C;
            if (slot + q < w.capLeaf)
              w.leaves[slot + q] = Seg{off + o, sz, s.root, make_meta(cd, LEAF_COPY, 0, 0, 0)};
            else
              raise_error(w.ctr, 1u);
          }
          ps.leafKeys[LEAF_COPY] += size;
        }
      }
      // high bits: decode on the way out, for final children written to the
      // output only (keys in TMP stay encoded; their copy leaf decodes them)
      gD[c] = (uint8_t)(cd | ((p.kind[c] != CHILD_REG && cd == BUF_OUT) ? (1u << 4) : 0u));
    }
    // statistics: leaves, the largest regular child, keys in final children
    // and the imbalance L* / ceil(W / r) of the grouping (Section 6, lemma on
    // the largest group)
    flush_place_stats(w, ps);
    maxChild = wave_max(maxChild);
    if ((tid & 63u) == 0 && maxChild) atomicMax(&w.ctr->lv_maxchild[lv.level], maxChild);
    if (tid == 0) {
      w.nch[i] = nch;
      if (N > Wreg) atomicAdd(&w.ctr->lv_final[lv.level], (unsigned long long)(N - Wreg));
      if (Wreg) {
        const uint32_t avg = (Wreg + r - 1) / r;
        const uint32_t q = (uint32_t)(((uint64_t)L << 16) / avg);
        atomicMax(&w.ctr->lv_imb_max[lv.level], q);
        atomicAdd(&w.ctr->lv_imb_sum[lv.level], (unsigned long long)q);
      }
    }
    __syncthreads();
  }
}

// Grouping alone (step entry point): out[0] = L*, out[1] = groups,
// out[2..] = group starts.
__global__ void __launch_bounds__(256) k_pack_only(const uint32_t *wgt, uint32_t nb, uint32_t r,
                                                   uint32_t *out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint32_t *sW = (uint32_t *)smem_raw;
  __shared__ uint32_t red[16];
  for (uint32_t j = threadIdx.x; j < ((nb + 7) & ~7u); j += 256) sW[j] = j < nb ? wgt[j] : 0u;
  __syncthreads();
  uint32_t L = optimal_load<256>(sW, nb, r, red);
  if (threadIdx.x == 0) {
    uint32_t cur = 0, g = 0;
    out[2 + g++] = 0;
    for (uint32_t j = 0; j < nb; ++j) {
      if (cur + sW[j] > L) {
        out[2 + g++] = j;
        cur = 0;
      }
      cur += sW[j];
    }
    out[0] = L;
    out[1] = g;
  }
}

__global__ void __launch_bounds__(256) k_tile_scan(Ws w, Lev lv) {
  const uint32_t tid = threadIdx.x;
  const uint32_t P = w.ctr->P;
  // item = (tile block, 256 children)
  const uint32_t chunks = (lv.CH + 255) / 256, total = w.ctr->nblk * chunks;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    const uint32_t B = item / chunks, ch = item - B * chunks;
    uint32_t i = find_owner(w.blkStart, P, B);
    uint32_t bb = B - w.blkStart[i];
    uint32_t t0 = w.tileStart[i] + bb * lv.TB;
    uint32_t t1 = t0 + lv.TB < w.tileStart[i + 1] ? t0 + lv.TB : w.tileStart[i + 1];
    uint32_t nch = w.nch[i];
    const uint16_t *tf = w.cfirst + (size_t)i * 2 * (lv.CH + 1);
    const uint32_t *cs = w.cstart + (size_t)i * (lv.CH + 1);
    const uint32_t *pre = w.blkHist + (size_t)B * lv.HS;  // prefix over earlier blocks
    const uint32_t c = ch * 256 + tid;
    if (c < nch) {
      const uint32_t f = tf[2 * c], e = tf[2 * c + 1];  // the child's nonempty ids
      uint32_t run = cs[c];
      for (uint32_t id = f; id < e; ++id) run += pre[id];
      // the child's count in 8 tiles at a time (independent loads), then
      // the running offsets
      uint32_t t = t0;
      for (; t + 8 <= t1; t += 8) {
        uint32_t cnt[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t *h = w.hist + (size_t)(t + u) * lv.HS;
          uint32_t x = 0;
          for (uint32_t id = f; id < e; ++id) x += h[id];
          cnt[u] = x;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          w.tileOff[(size_t)(t + u) * lv.CH + c] = run;
          run += cnt[u];
        }
      }
      for (; t < t1; ++t) {
        w.tileOff[(size_t)t * lv.CH + c] = run;
        const uint32_t *h = w.hist + (size_t)t * lv.HS;
        for (uint32_t id = f; id < e; ++id) run += h[id];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stable scatter (Section 6 data delivery to groups, here into HBM ranges;
// the prefix sums of Section 4.3 give every tile's start in every child).
// A tile is processed in chunks of 256*KPT keys: every wavefront takes a
// contiguous quarter of the chunk, ranks its keys among equal children with
// ballots (input order kept), the chunk is regrouped by child in LDS and
// written out in runs.  Pairs use it for levels too wide for
// k_scatter_pairs; keys-only sorts use it when a stable partition is asked
// for.
// ---------------------------------------------------------------------------
template <int KT, bool PAY, int KPT>
__global__ void __launch_bounds__(256) k_scatter(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  constexpr uint32_t CHK = 256 * KPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t CH = lv.CH;
  K *sTree = (K *)smem_raw;                                  // mmax
  K *stK = sTree + lv.mmax;                                  // CHK
  uint32_t *stV = (uint32_t *)(stK + CHK);                   // CHK if PAY
  uint16_t *stC = (uint16_t *)(stV + (PAY ? CHK : 0));       // CHK
  uint16_t *sI2C = stC + CHK;                                // HS
  uint32_t *sBase = (uint32_t *)(sI2C + lv.HS);              // CH
  uint32_t *sL = sBase + CH;                                 // CH + 1
  uint32_t *sTot = sL + CH + 1;                              // CH
  uint32_t *sCnt = sTot + CH;                                // 4 * CH
  uint32_t *sTmp = sCnt + 4 * CH;                            // 256
  uint8_t *sCd = (uint8_t *)(sTmp + 256);                    // CH
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t P = w.ctr->P;
  ItemRange ir = xcd_items(w.ctr->ntile);
  uint32_t cur = 0xFFFFFFFFu, logm = 0, nch = 0, nbits = 0;
  bool eq = false;
  for (uint32_t g = ir.first; g < ir.end; g += ir.step) {
    uint32_t i = find_owner(w.tileStart, P, g);
    uint32_t t = g - w.tileStart[i];
    Seg s = w.act[lv.level][i];
    if (i != cur) {
      __syncthreads();
      logm = meta_logm(s.meta);
      const uint32_t m = 1u << logm;
      const K *gt = (const K *)w.tree + (size_t)i * lv.mmax;
      for (uint32_t j = tid + 1; j < m; j += 256) sTree[j] = gt[j];
      eq = w.eqOn[i] != 0;
      nch = w.nch[i];
      nbits = ilog2c(nch);
      const uint32_t NB = eq ? 2 * m - 1 : m;
      const uint16_t *gi = w.i2c + (size_t)i * lv.HS;
      for (uint32_t j = tid; j < NB; j += 256) sI2C[j] = gi[j];
      const uint8_t *gd = w.cdst + (size_t)i * CH;
      for (uint32_t c = tid; c < nch; c += 256) sCd[c] = gd[c];
      cur = i;
    }
    for (uint32_t c = tid; c < nch; c += 256) sBase[c] = w.tileOff[(size_t)g * CH + c];
    Root R = w.roots[s.root];
    const uint32_t buf = seg_buf(s.meta);
    const GMem<K> *src = (const GMem<K> *)(kptr<K>(w, R, buf) + s.off);
    const GMem<uint32_t> *vsrc = PAY ? (const GMem<uint32_t> *)(vptr(w, R, buf) + s.off) : nullptr;
    const bool enc = buf == BUF_IN;
    const uint32_t lo = t * lv.TC;
    const uint32_t hi = lo + lv.TC < s.size ? lo + lv.TC : s.size;
    // chunk keys (and payloads) at cb into registers; the next chunk of the
    // tile is requested before the current one is classified
    auto load_chunk = [&](uint32_t cb, K (&xk)[KPT], uint32_t (&xv)[KPT]) {
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t p = cb + wave * (CHK / 4) + k * 64 + lane;
        const bool valid = p < hi;
        xk[k] = valid ? src[p] : (K)0;
        xv[k] = PAY && valid ? vsrc[p] : 0u;
      }
    };
    K xk[KPT];
    uint32_t xv[KPT];
    load_chunk(lo, xk, xv);
    for (uint32_t cb = lo; cb < hi; cb += CHK) {
      K nk[KPT];
      uint32_t nv[KPT];
      if (cb + CHK < hi) load_chunk(cb + CHK, nk, nv);
      for (uint32_t q = tid; q < 4 * CH; q += 256) sCnt[q] = 0;
      __syncthreads();
      if (enc) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) xk[k] = Key<KT>::enc(xk[k]);
      }
      uint32_t xcr[KPT];  // child << 16 | rank inside (wave, child)
      classify_batch<K, KPT>(xk, xcr, sTree, logm, eq);
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t p = cb + wave * (CHK / 4) + k * 64 + lane;
        const bool valid = p < hi;
        const K x = xk[k];
        const uint32_t v = xv[k];
        uint32_t c = valid ? sI2C[xcr[k]] : 0u;
        uint64_t peers = match_lanes(c, valid, nbits);
        uint32_t below = bits_below(peers);
        uint32_t r = 0;
        if (valid) {
          uint32_t *cnt = sCnt + wave * CH + c;
          r = *cnt + below;
          if (below == 0) *cnt = r + (uint32_t)__popcll(peers);
        }
        xk[k] = x;
        xv[k] = v;
        xcr[k] = (c << 16) | r;
      }
      __syncthreads();
      for (uint32_t c = tid; c < nch; c += 256) {
        uint32_t tot = sCnt[c] + sCnt[CH + c] + sCnt[2 * CH + c] + sCnt[3 * CH + c];
        sTot[c] = tot;
        sL[c] = tot;
      }
      __syncthreads();
      block_exscan<256>(sL, nch, sTmp);
      for (uint32_t c = tid; c < nch; c += 256) {
        uint32_t run = sL[c];
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
          uint32_t v = sCnt[ww * CH + c];
          sCnt[ww * CH + c] = run;
          run += v;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t p = cb + wave * (CHK / 4) + k * 64 + lane;
        if (p < hi) {
          const uint32_t c = xcr[k] >> 16;
          const uint32_t q = sCnt[wave * CH + c] + (xcr[k] & 0xFFFFu);
          stK[q] = xk[k];
          stC[q] = (uint16_t)c;
          if (PAY) stV[q] = xv[k];
        }
      }
      __syncthreads();
      const uint32_t cnt = hi - cb < CHK ? hi - cb : CHK;
      for (uint32_t q = tid; q < cnt; q += 256) {
        const uint32_t c = stC[q];
        const uint32_t rel = sBase[c] + (q - sL[c]);
        if (rel >= s.size) {  // defensive: tables inconsistent; never write outside
          raise_error(w.ctr, 16u);
          continue;
        }
        const uint32_t d = s.off + rel;
        const uint32_t cd = sCd[c];
        const uint32_t db = cd & 15u;
        K x = stK[q];
        if (cd >> 4) x = Key<KT>::dec(x);
        ((GMem<K> *)kptr<K>(w, R, db))[d] = x;
        if (PAY) ((GMem<uint32_t> *)vptr(w, R, db))[d] = stV[q];
      }
      __syncthreads();
      for (uint32_t c = tid; c < nch; c += 256) sBase[c] += sTot[c];
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        xk[k] = nk[k];
        xv[k] = nv[k];
      }
    }
  }
}

// Keys-only scatter.  Without a payload, equal keys are equal bit patterns, so
// their order inside a child is immaterial and a chunk is regrouped with LDS
// atomics instead of ballot ranks.  The next chunk's keys are loaded into
// registers while the current one is classified, regrouped and written.
constexpr uint32_t SCK_THREADS = 1024;
// Stores of a chunk's empty slots (past the tile's end, or of a child that
// would overrun its subproblem) go to a sink in the workspace instead of
// being skipped: every store of the write-out is then unconditional, and the
// compiler's count of outstanding memory operations stays exact, so the
// next chunk's keys are waited for without waiting for the stores.
constexpr uint32_t SINK_WORDS = SCK_THREADS * 8;

// Chunk keys of a tile: the tile's keys are read through a buffer resource
// over [tile start, tile end), 16 bytes per lane and load; chunk offset coff
// is in bytes from the tile start.  Key u of a thread sits at chunk position
// sck_pos(u) (positions past the tile end read as zero).
template <typename K, int KPT> AMS_DEV uint32_t sck_pos(uint32_t u) {
  constexpr uint32_t V = Vec16<K>::N;
  return (u / V) * (V * SCK_THREADS) + V * threadIdx.x + (u % V);
}

template <int KT, int KPT>
AMS_DEV void sck_load(Rsrc rs, uint32_t coff, typename Key<KT>::T (&x)[KPT]) {
  typedef typename Key<KT>::T K;
  constexpr uint32_t V = Vec16<K>::N;
  static_assert(KPT % V == 0, "whole 16-byte loads per thread");
#pragma unroll
  for (uint32_t k = 0; k < KPT / V; ++k) {
    // whole offset in the vector operand, which the range check covers
    const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(
        rs, threadIdx.x * 16u + coff + k * (SCK_THREADS * 16u), 0, 0);
    Vec16<K>::get(v, &x[k * V]);
  }
}

// Out-of-place exclusive scan of in[0..n) into out by a block of NT threads
// (tmp: NT/64 words of LDS); same scheme as block_exscan.
template <int NT>
AMS_DEV void block_exscan_to(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *tmp) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  constexpr uint32_t NW = NT / 64;
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t lo = tid * per < n ? tid * per : n;
  const uint32_t hi = lo + per < n ? lo + per : n;
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += in[i];
  const uint32_t incl = wave_incl_scan(s);
  if (lane == 63) tmp[wave] = incl;
  __syncthreads();
  uint32_t off = 0;
#pragma unroll
  for (uint32_t w = 0; w < NW; ++w) off += w < wave ? tmp[w] : 0u;
  uint32_t run = off + incl - s;
  for (uint32_t i = lo; i < hi; ++i) {
    out[i] = run;
    run += in[i];
  }
  __syncthreads();
}

// Buffer resource over the keys of tile g of a level (wave-uniform).
template <typename K>
AMS_DEV Rsrc tile_rsrc(const Ws &w, const Lev &lv, uint32_t P, uint32_t g) {
  const uint32_t i = find_owner(w.tileStart, P, g);
  const uint32_t t = g - w.tileStart[i];
  const Seg s = w.act[lv.level][i];
  const Root R = w.roots[s.root];
  const uint32_t lo = t * lv.TC;
  const uint32_t hi = lo + lv.TC < s.size ? lo + lv.TC : s.size;
  const K *src = kptr<K>(w, R, seg_buf(s.meta)) + s.off + lo;
  return make_rsrc(uniform_ptr(src), __builtin_amdgcn_readfirstlane((hi - lo) * (uint32_t)sizeof(K)));
}

// With PRIV (levels of at most SCK_PCH children) every wavefront scans the
// chunk's child counts itself into a row of 16-bit offsets of its own, and
// the counters alternate between two banks from chunk to chunk: a chunk then
// needs two barriers instead of four.
constexpr uint32_t SCK_PCH = 768;  // 12 children per lane

template <int KT, int KPT, bool PRIV>
__global__ void __launch_bounds__(SCK_THREADS, 1) k_scatter_keys(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  constexpr uint32_t CHK = SCK_THREADS * KPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t CH = lv.CH;
  K *sTree = (K *)smem_raw;                       // mmax
  K *stK = sTree + lv.mmax;                       // CHK
  // CH + 2: output address of chunk slot 0, per child; entry CH: the sink
  // (the second extra entry keeps the next arrays 16-byte aligned)
  uint64_t *sDst = (uint64_t *)(stK + CHK);
  // PRIV: two banks of SCK_PCH counters and 16 rows of SCK_PCH offsets
  uint32_t *sCnt2 = (uint32_t *)(sDst + CH + 2);
  uint16_t *sRows = (uint16_t *)(sCnt2 + (PRIV ? 2 * SCK_PCH : 0));
  uint16_t *stC = sRows + (PRIV ? (SCK_THREADS / 64) * SCK_PCH : 0);  // CHK
  uint16_t *sI2C = stC + CHK;                     // HS
  uint32_t *sBase = (uint32_t *)(sI2C + lv.HS);   // CH
  uint32_t *sL = sBase + CH;                      // CH (not PRIV)
  uint32_t *sCnt = sL + (PRIV ? 0 : CH);          // CH (not PRIV)
  uint32_t *sTmp = sCnt + (PRIV ? 0 : CH);        // SCK_THREADS / 64
  uint8_t *sCd = (uint8_t *)(sTmp + SCK_THREADS / 64);  // CH
  const uint32_t tid = threadIdx.x;
  uint16_t *myRow = sRows + (tid >> 6) * SCK_PCH;
  uint32_t par = 0;  // PRIV: counter bank of the current chunk
  const uint32_t P = w.ctr->P;
  ItemRange ir = xcd_items(w.ctr->ntile);
  uint32_t cur = 0xFFFFFFFFu, logm = 0, nch = 0;
  bool eq = false;
  if (PRIV) {
    for (uint32_t c = tid; c < 2 * SCK_PCH; c += SCK_THREADS) sCnt2[c] = 0;
  } else {
    for (uint32_t c = tid; c < CH; c += SCK_THREADS) sCnt[c] = 0;
  }
  if (tid == 0) sDst[CH] = (uint64_t)(uintptr_t)w.sink;  // slots past the chunk's end
  if (ir.first >= ir.end) return;
  // The keys of the first chunk of a tile are loaded while the previous
  // tile's last chunk is processed, so no tile starts on an empty pipeline.
  K xa[KPT];
  sck_load<KT, KPT>(tile_rsrc<K>(w, lv, P, ir.first), 0u, xa);
  for (uint32_t g = ir.first; g < ir.end; g += ir.step) {
    const uint32_t i = find_owner(w.tileStart, P, g);
    const uint32_t t = g - w.tileStart[i];
    const Seg s = w.act[lv.level][i];
    const Root R = w.roots[s.root];
    const uint32_t buf = seg_buf(s.meta);
    const K *src = kptr<K>(w, R, buf) + s.off;
    const bool enc = buf == BUF_IN;
    const uint32_t lo = t * lv.TC;
    const uint32_t hi = lo + lv.TC < s.size ? lo + lv.TC : s.size;
    const bool more = g + ir.step < ir.end;
    const Rsrc rs = make_rsrc(uniform_ptr(src + lo), (hi - lo) * (uint32_t)sizeof(K));
    const Rsrc rsn = more ? tile_rsrc<K>(w, lv, P, g + ir.step) : rs;
    if (i != cur) {
      __syncthreads();
      logm = meta_logm(s.meta);
      const uint32_t m = 1u << logm;
      const K *gt = (const K *)w.tree + (size_t)i * lv.mmax;
      for (uint32_t j = tid + 1; j < m; j += SCK_THREADS) sTree[j] = gt[j];
      eq = w.eqOn[i] != 0;
      nch = w.nch[i];
      const uint32_t NB = eq ? 2 * m - 1 : m;
      const uint16_t *gi = w.i2c + (size_t)i * lv.HS;
      for (uint32_t j = tid; j < NB; j += SCK_THREADS) sI2C[j] = gi[j];
      const uint8_t *gd = w.cdst + (size_t)i * CH;
      for (uint32_t c = tid; c < nch; c += SCK_THREADS) sCd[c] = gd[c];
      cur = i;
      __syncthreads();  // the subproblem's tables are in LDS
    }
    // sBase[c]: this tile's next output offset of child c (read and
    // advanced only by thread c % SCK_THREADS, so no barrier is needed)
    for (uint32_t c = tid; c < nch; c += SCK_THREADS) sBase[c] = w.tileOff[(size_t)g * CH + c];
    for (uint32_t cb = lo; cb < hi; cb += CHK) {
      // the next chunk: of this tile, else the first of the next tile, else
      // an offset past the range (zeros); always issued, see SINK_WORDS
      K xb[KPT];
      const bool inTile = cb + CHK < hi;
      sck_load<KT, KPT>(inTile ? rs : rsn,
                        inTile ? (cb + CHK - lo) * (uint32_t)sizeof(K) : (more ? 0u : 0x80000000u),
                        xb);
      if (enc) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) xa[k] = Key<KT>::enc(xa[k]);
      }
      uint32_t xcs[KPT];  // child << 16 | slot
      classify_batch<K, KPT>(xa, xcs, sTree, logm, eq);
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t p = cb + sck_pos<K, KPT>(k);
        const uint32_t c = p < hi ? (uint32_t)sI2C[xcs[k]] : 0u;
        const uint32_t slot = wave_slot_add(PRIV ? sCnt2 + par * SCK_PCH : sCnt, c, p < hi);
        xcs[k] = (c << 16) | slot;
      }
      __syncthreads();
      const uint32_t *ccnt = PRIV ? sCnt2 + par * SCK_PCH : sCnt;  // this chunk's counts
      const uint16_t *off16 = myRow;  // PRIV: this wavefront's offsets
      if (PRIV) {
        // the whole exclusive scan of the counts in every wavefront: lane
        // l takes children [12 l, 12 l + 12) (counts past nch are zero)
        const uint32_t lane = tid & 63u;
        const uint4 *c4 = (const uint4 *)(ccnt + 12 * lane);
        const uint4 a0 = c4[0], a1 = c4[1], a2 = c4[2];
        const uint32_t v[12] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x, a2.y, a2.z, a2.w};
        uint32_t tot = 0;
#pragma unroll
        for (int j = 0; j < 12; ++j) tot += v[j];
        uint32_t run = wave_incl_scan(tot) - tot;
        uint64_t o[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 12; ++j) {
          o[j / 4] |= (uint64_t)(run & 0xFFFFu) << (16 * (j % 4));
          run += v[j];
        }
        u64_alias *r8 = (u64_alias *)(myRow + 12 * lane);
        r8[0] = o[0];
        r8[1] = o[1];
        r8[2] = o[2];
      } else {
        block_exscan_to<SCK_THREADS>(sCnt, sL, nch, sTmp);
      }
      // per child: the output address of chunk slot 0 (low bit: decode the
      // key on the way out; a child that would overrun its subproblem has
      // its keys sent to the sink, flagged as an overflow); then advance sBase
      for (uint32_t c = tid; c < nch; c += SCK_THREADS) {
        const uint32_t cd = sCd[c];
        const uint32_t nc = ccnt[c];
        const uint32_t lc = PRIV ? (uint32_t)off16[c] : sL[c];
        uint64_t d;
        if ((uint64_t)sBase[c] + nc <= s.size) {
          const K *base = kptr<K>(w, R, cd & 15u) + s.off + sBase[c];
          d = ((uint64_t)(uintptr_t)base - (uint64_t)lc * sizeof(K)) | (uint64_t)(cd >> 4);
        } else {
          raise_error(w.ctr, 16u);
          d = (uint64_t)(uintptr_t)w.sink - (uint64_t)lc * sizeof(K);
        }
        sDst[c] = d;
        sBase[c] += nc;
        if (!PRIV) sCnt[c] = 0;  // its last use in this chunk: ready for the next one
      }
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t p = cb + sck_pos<K, KPT>(k);
        if (p < hi) {
          const uint32_t c = xcs[k] >> 16;
          const uint32_t q = (PRIV ? (uint32_t)off16[c] : sL[c]) + (xcs[k] & 0xFFFFu);
          stK[q] = xa[k];
          stC[q] = (uint16_t)c;
        }
      }
      __syncthreads();
      // write out: consecutive slots of a child go to consecutive addresses
      const uint32_t cnt = hi - cb < CHK ? hi - cb : CHK;
      uint32_t cc[KPT];
      K xo[KPT];
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t q = tid + SCK_THREADS * k;
        cc[k] = q < cnt ? stC[q] : CH;  // past the chunk's end: the sink
        xo[k] = stK[q];
      }
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        const uint32_t q = tid + SCK_THREADS * k;
        const uint64_t d = sDst[cc[k]];
        const K x = (d & 1u) ? Key<KT>::dec(xo[k]) : xo[k];
        *(GMem<K> *)((d & ~(uint64_t)1) + (uint64_t)q * sizeof(K)) = x;
      }
      // no barrier here: every wavefront finishes this write-out before it
      // reaches the next chunk's first barrier, and the staging area is
      // only written after that barrier
      if (PRIV) {
        // this bank was last read before the barrier above; it is counted
        // into again two chunks on, after two more barriers
        for (uint32_t c = tid; c < nch; c += SCK_THREADS) sCnt2[par * SCK_PCH + c] = 0;
        par ^= 1u;
      }
#pragma unroll
      for (int k = 0; k < KPT; ++k) xa[k] = xb[k];
    }
  }
}

// Pairs scatter with 1024 threads and chunks of 8192 pairs, so a child's run
// in a chunk is four times longer than with k_scatter's 2048-pair chunks.
// Wavefront v ranks the v-th sixteenth of the chunk in input order: ballots
// rank lanes with equal children, and a row of 16-bit counters of its own
// carries the rank from one row of keys to the next.  After the per-child
// totals and offsets are formed, each wavefront clears its own row once it
// has staged its keys, so the reset needs no barrier of its own.  The next
// chunk of the tile is requested before the current one is classified.
constexpr uint32_t SCP_KPT = 8;

template <int KT>
__global__ void __launch_bounds__(SCK_THREADS, 1) k_scatter_pairs(Ws w, Lev lv) {
  typedef typename Key<KT>::T K;
  constexpr uint32_t KPT = SCP_KPT, CHK = SCK_THREADS * KPT, NW = SCK_THREADS / 64;
  constexpr uint32_t PW = CHK / NW;  // pairs per wavefront and chunk
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t CH = lv.CH, CHP = (CH + 3) & ~3u;
  K *sTree = (K *)smem_raw;                                  // mmax
  K *stK = sTree + lv.mmax;                                  // CHK
  uint32_t *stV = (uint32_t *)(stK + CHK);                   // CHK
  uint16_t *stC = (uint16_t *)(stV + CHK);                   // CHK
  uint16_t *sRow = stC + CHK;                                // NW rows of CHP counters
  uint16_t *sI2C = sRow + NW * CHP;                          // HS (rounded up to even)
  uint32_t *sBase = (uint32_t *)(sI2C + ((lv.HS + 1) & ~1u)); // CH
  uint32_t *sL = sBase + CH;                                 // CH
  uint32_t *sRel = sL + CH;                                  // CH: output index of slot 0
  uint32_t *sTmp = sRel + CH;                                // NW
  uint8_t *sCd = (uint8_t *)(sTmp + NW);                     // CH
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t P = w.ctr->P;
  ItemRange ir = xcd_items(w.ctr->ntile);
  uint32_t cur = 0xFFFFFFFFu, logm = 0, nch = 0, nbits = 0;
  bool eq = false;
  for (uint32_t q = tid; q < NW * CHP; q += SCK_THREADS) sRow[q] = 0;
  uint16_t *row = sRow + wave * CHP;
  for (uint32_t g = ir.first; g < ir.end; g += ir.step) {
    const uint32_t i = find_owner(w.tileStart, P, g);
    const uint32_t t = g - w.tileStart[i];
    const Seg s = w.act[lv.level][i];
    const Root R = w.roots[s.root];
    if (i != cur) {
      __syncthreads();
      logm = meta_logm(s.meta);
      const uint32_t m = 1u << logm;
      const K *gt = (const K *)w.tree + (size_t)i * lv.mmax;
      for (uint32_t j = tid + 1; j < m; j += SCK_THREADS) sTree[j] = gt[j];
      eq = w.eqOn[i] != 0;
      nch = w.nch[i];
      nbits = ilog2c(nch);
      const uint32_t NB = eq ? 2 * m - 1 : m;
      const uint16_t *gi = w.i2c + (size_t)i * lv.HS;
      for (uint32_t j = tid; j < NB; j += SCK_THREADS) sI2C[j] = gi[j];
      const uint8_t *gd = w.cdst + (size_t)i * CH;
      for (uint32_t c = tid; c < nch; c += SCK_THREADS) sCd[c] = gd[c];
      cur = i;
      __syncthreads();  // the subproblem's tables are in LDS
    }
    // sBase[c]: this tile's next output offset of child c (thread c only;
    // nch <= CH <= 1024, so thread c owns child c)
    if (tid < nch) sBase[tid] = w.tileOff[(size_t)g * CH + tid];
    const uint32_t buf = seg_buf(s.meta);
    const GMem<K> *src = (const GMem<K> *)(kptr<K>(w, R, buf) + s.off);
    const GMem<uint32_t> *vsrc = (const GMem<uint32_t> *)(vptr(w, R, buf) + s.off);
    // the tile's constants in scalar registers (they stay live across the
    // whole chunk loop)
    GMem<K> *kTmp = (GMem<K> *)uniform_ptr(kptr<K>(w, R, BUF_TMP));
    GMem<K> *kOut = (GMem<K> *)uniform_ptr(kptr<K>(w, R, BUF_OUT));
    GMem<uint32_t> *vTmp = (GMem<uint32_t> *)uniform_ptr(vptr(w, R, BUF_TMP));
    GMem<uint32_t> *vOut = (GMem<uint32_t> *)uniform_ptr(vptr(w, R, BUF_OUT));
    const bool enc = buf == BUF_IN;
    const uint32_t sOff = __builtin_amdgcn_readfirstlane(s.off);
    const uint32_t sSize = __builtin_amdgcn_readfirstlane(s.size);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(t * lv.TC);
    const uint32_t hi = lo + lv.TC < sSize ? lo + lv.TC : sSize;
    // keys are requested one chunk ahead; payloads at the start of their
    // own chunk (they are needed only when the chunk is staged).  Both go
    // through buffer resources over the tile, whose range check returns
    // zeros past its end: the loads need no branches, so the waits for
    // them count exactly and the next chunk's keys stay in flight.
    const Rsrc rk = make_rsrc(uniform_ptr((const K *)src + lo), (hi - lo) * (uint32_t)sizeof(K));
    const Rsrc rv = make_rsrc(uniform_ptr((const uint32_t *)vsrc + lo), (hi - lo) * 4u);
    auto load_keys = [&](uint32_t cb, K (&xk)[KPT]) {
#pragma unroll
      for (uint32_t k = 0; k < KPT; ++k) {
        const uint32_t p = cb - lo + wave * PW + k * 64 + lane;
        xk[k] = buf_load<K>(rk, p * (uint32_t)sizeof(K));
      }
    };
    K xk[KPT];
    load_keys(lo, xk);
    for (uint32_t cb = lo; cb < hi; cb += CHK) {
      uint32_t xv[KPT];
#pragma unroll
      for (uint32_t k = 0; k < KPT; ++k) {
        const uint32_t p = cb - lo + wave * PW + k * 64 + lane;
        xv[k] = buf_load<uint32_t>(rv, p * 4u);
      }
      K nk[KPT];
      load_keys(cb + CHK, nk);  // past the tile's end: zeros
      if (enc) {
#pragma unroll
        for (uint32_t k = 0; k < KPT; ++k) xk[k] = Key<KT>::enc(xk[k]);
      }
      uint32_t xcr[KPT];  // child << 16 | rank among the wavefront's pairs of that child
      classify_batch<K, KPT>(xk, xcr, sTree, logm, eq);
#pragma unroll
      for (uint32_t k = 0; k < KPT; ++k) {
        const bool valid = cb + wave * PW + k * 64 + lane < hi;
        const uint32_t c = valid ? (uint32_t)sI2C[xcr[k]] : 0u;
        const uint64_t peers = match_lanes(c, valid, nbits);
        const uint32_t below = bits_below(peers);
        uint32_t r = 0;
        if (valid) {
          r = row[c] + below;
          if (below == 0) row[c] = (uint16_t)(r + (uint32_t)__popcll(peers));
        }
        xcr[k] = (c << 16) | r;
      }
      __syncthreads();
      // per child: chunk total, its exclusive scan (sL), the offset of every
      // wavefront's pairs (in the rows) and the output index of slot 0
      const uint32_t c = tid;
      uint32_t tot = 0;
      if (c < nch) {
#pragma unroll
        for (uint32_t v = 0; v < NW; ++v) tot += sRow[v * CHP + c];
        sL[c] = tot;
      }
      block_exscan<SCK_THREADS>(sL, nch, sTmp);  // thread c scans its own entry; ends on a barrier
      if (c < nch) {
        uint32_t run = sL[c];
#pragma unroll
        for (uint32_t v = 0; v < NW; ++v) {
          const uint32_t n = sRow[v * CHP + c];
          sRow[v * CHP + c] = (uint16_t)run;
          run += n;
        }
        if ((uint64_t)sBase[c] + tot <= sSize) {
          sRel[c] = sOff + sBase[c] - sL[c];
        } else {  // would overrun the subproblem: dropped and flagged
          raise_error(w.ctr, 16u);
          sRel[c] = 0xFFFFFFFFu;
        }
        sBase[c] += tot;
      }
      __syncthreads();
#pragma unroll
      for (uint32_t k = 0; k < KPT; ++k) {
        if (cb + wave * PW + k * 64 + lane < hi) {
          const uint32_t cc = xcr[k] >> 16;
          const uint32_t q = row[cc] + (xcr[k] & 0xFFFFu);
          stK[q] = xk[k];
          stV[q] = xv[k];
          stC[q] = (uint16_t)cc;
        }
      }
      // this wavefront's row is not read again in this chunk: clear it for
      // the next one (CHP is a multiple of 4, rows are 8-byte aligned)
      for (uint32_t j = lane; j < CHP / 4; j += 64) ((u64_alias *)row)[j] = 0;
      __syncthreads();
      // write out: consecutive slots of a child go to consecutive indices
      // (a child's destination is the TMP or the OUT buffer, both uniform)
      const uint32_t cnt = hi - cb < CHK ? hi - cb : CHK;
#pragma unroll 2
      for (uint32_t k = 0; k < KPT; ++k) {
        const uint32_t q = tid + SCK_THREADS * k;
        if (q < cnt) {
          const uint32_t cc = stC[q];
          const uint32_t rel = sRel[cc];
          if (rel != 0xFFFFFFFFu) {
            const uint32_t cd = sCd[cc];
            const bool toOut = (cd & 15u) == BUF_OUT;
            K x = stK[q];
            if (cd >> 4) x = Key<KT>::dec(x);
            (toOut ? kOut : kTmp)[rel + q] = x;
            (toOut ? vOut : vTmp)[rel + q] = stV[q];
          }
        }
      }
      // no barrier here: the next chunk writes the staging area and the
      // per-child tables only after its first barrier
#pragma unroll
      for (uint32_t k = 0; k < KPT; ++k) xk[k] = nk[k];
    }
  }
}

// ---------------------------------------------------------------------------
// Base case (Section 4.2 all-pairs ranking; Section 6 base case).
// ---------------------------------------------------------------------------
constexpr uint32_t FIN_KPT = CMAX / FIN_THREADS;  // 16 keys per thread
constexpr uint32_t LEAF_STREAM = 0xFFu;

// LDS of one base-case workgroup.  B holds the keys regrouped by bucket plus
// FIN_PAD slots that receive the largest key value as sentinels; the sample,
// its sorted blocks and the splitter tree live inside B until the keys are
// staged there.  Keys-only fits in 80 KiB (two workgroups per CU).
constexpr uint32_t FIN_PAD = 256;

template <typename K> struct FinSmem {
  K *B;             // C + FIN_PAD keys
  uint32_t *vB;     // C payloads (pairs only)
  uint8_t *bid;     // C: bucket index b of each staged key (equality bit recomputed)
  uint32_t *bstart; // 2*FMAX + 4 bucket starts
  uint32_t *wred;   // 2 * 8 words: per-wave totals and maxima of the bucket scan
  uint32_t *cnt;    // bucket counters (keys-only) or 8 per-wave rows (pairs)
  uint32_t *tmp;    // FIN_THREADS words of scan scratch (aliases cnt for keys-only)
  uint32_t *bm;     // C bits: placed positions (keys-only; aliases cnt)
  K *srt;           // FMAX sorted samples; srt[1..f-1] are the splitters
  K *smp, *blk, *tree;  // overlays in the bid region: sample, block-sorted sample, tree
};

template <typename K, bool PAY> AMS_HD size_t fin_cnt_words() { return PAY ? 8 * 2 * FMAX : 2 * FMAX; }

template <typename K> AMS_HD uint32_t fin_bid_bytes(uint32_t C) {
  const uint32_t b = (C + 15) & ~15u, o = 3 * FMAX * (uint32_t)sizeof(K);
  return b > o ? b : o;
}

template <typename K, bool PAY> AMS_DEV FinSmem<K> fin_smem(unsigned char *base, uint32_t C) {
  FinSmem<K> f;
  f.B = (K *)base;
  f.vB = (uint32_t *)(f.B + C + FIN_PAD);
  f.bid = (uint8_t *)(f.vB + (PAY ? C : 0));
  f.bstart = (uint32_t *)(f.bid + fin_bid_bytes<K>(C));
  f.wred = f.bstart + 2 * FMAX + 4;
  f.cnt = f.wred + 16;
  f.tmp = PAY ? f.cnt + fin_cnt_words<K, PAY>() : f.cnt;
  f.bm = f.cnt;
  f.srt = (K *)(f.tmp + (PAY ? FIN_THREADS : fin_cnt_words<K, PAY>()));
  // sample overlays live in the bucket-id region until the split: the
  // sample, its sorted blocks and the splitter tree (FMAX keys each)
  f.smp = (K *)f.bid;
  f.blk = f.smp + FMAX;
  f.tree = f.smp + 2 * FMAX;
  return f;
}

template <typename K, bool PAY> __host__ inline size_t fin_smem_bytes(uint32_t C) {
  return (size_t)(C + FIN_PAD) * sizeof(K) + (PAY ? (size_t)C * 4 : 0) + fin_bid_bytes<K>(C) +
         (2 * FMAX + 4 + 16) * 4 + fin_cnt_words<K, PAY>() * 4 + (PAY ? FIN_THREADS * 4 : 0) +
         FMAX * sizeof(K);
}

// Largest leaf the base case takes for a key width / payload: keys-only
// stays within 80 KiB of LDS so that two workgroups share a CU.
__host__ inline uint32_t fin_capacity(uint32_t kw, bool pay) {
  uint32_t C = CMAX;
  while (C > 1024) {
    size_t b = kw == 8 ? (pay ? fin_smem_bytes<uint64_t, true>(C) : fin_smem_bytes<uint64_t, false>(C))
                       : (pay ? fin_smem_bytes<uint32_t, true>(C) : fin_smem_bytes<uint32_t, false>(C));
    // keep 1 KiB for the kernel's static LDS (barrier reductions)
    if (b <= (pay ? 163840u : 81920u) - 1024u) break;
    C -= 16;
  }
  return C;
}

// classify FIN_KPT keys in two batches of half the width (register pressure)
template <typename K>
AMS_DEV void classify_halves(K (&x)[FIN_KPT], uint32_t (&id)[FIN_KPT], const K *tree,
                             uint32_t logf, bool eq, uint32_t s) {
  constexpr int H = FIN_KPT / 2;
  K xa[H];
  uint32_t ia[H];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h * H * FIN_THREADS >= s) {  // uniform: no key in this half of the slots
#pragma unroll
      for (int u = 0; u < H; ++u) id[h * H + u] = 0;
      continue;
    }
#pragma unroll
    for (int u = 0; u < H; ++u) xa[u] = x[h * H + u];
    classify_batch<K, H>(xa, ia, tree, logf, eq);
#pragma unroll
    for (int u = 0; u < H; ++u) id[h * H + u] = ia[u];
  }
}

// Part of the rank of x (from block b of nbk sorted blocks of 64 keys) among
// the keys of the other blocks: this lane searches blocks part, part + H, ...
// (T of them), side by side one halving step per round so that the LDS reads
// of a round overlap.  Keys of an earlier block count when equal.  A block
// that is b or past nbk is searched at block 0 (valid addresses) and its
// count dropped.
template <typename K, uint32_t T>
AMS_DEV uint32_t cross_block_rank(const K *blk, uint32_t b, K x, uint32_t part, uint32_t H,
                                  uint32_t nbk) {
  uint32_t base[T], ob[T];
  bool use[T];
#pragma unroll
  for (uint32_t t = 0; t < T; ++t) {
    const uint32_t o = part + t * H;
    use[t] = o < nbk && o != b;
    ob[t] = o < nbk ? o : 0u;
    base[t] = 0;
  }
#pragma unroll
  for (uint32_t half = 32; half >= 1; half >>= 1) {
#pragma unroll
    for (uint32_t t = 0; t < T; ++t) {
      const K y = blk[ob[t] * 64 + base[t] + half - 1];
      base[t] += (y < x || (ob[t] < b && y == x)) ? half : 0u;
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (uint32_t t = 0; t < T; ++t) {
    const K y = blk[ob[t] * 64 + base[t]];
    const uint32_t c = base[t] + ((y < x || (ob[t] < b && y == x)) ? 1u : 0u);
    r += use[t] ? c : 0u;
  }
  return r;
}

// Sort s <= C keys from src into dst inside one workgroup.
//  1. a*f sampled keys are ranked: blocks of 64 by comparing all pairs, then
//     across blocks by binary search (Section 4.2); the elements of rank
//     a*j - 1 (j = 1..f-1) become srt[j], the splitters of an f-way split
//     (equality buckets if splitters repeat).
//  2. Every key is classified and placed in LDS by bucket (keys-only: LDS
//     atomics, order inside a bucket arbitrary since equal keys are equal
//     bits; pairs: ballot ranks, input order kept).
//  3. Every bucket is ordered by comparing all its pairs (Section 4.2):
//     pairs: rank(x_q) = #{j : x_j < x_q} + #{j < q : x_j = x_q};
//     keys-only: rank(x_q) = #{j : x_j < x_q}; equal keys then share a rank,
//     and the positions they leave empty are filled with the same bits.
//     Keys after a bucket are larger (buckets follow key order) and the pad
//     holds the largest value, so a scan may run past its bucket unmasked.
// In-LDS fan-out of a leaf of s keys: the smallest power of two f <= fmax
// with s / f <= cutoff / 2 (1 when the leaf is not split).
AMS_DEV uint32_t leaf_fanout(uint32_t s, uint32_t cutoff, uint32_t fmax) {
  uint32_t f = 1;
  if (s > cutoff) {
    const uint32_t tgt = cutoff / 2 > 4 ? cutoff / 2 : 4;
    const uint32_t need = (s + tgt - 1) / tgt;
    f = 2;
    while (f < need && f < fmax) f <<= 1;
  }
  return f;
}
// The range split of uint64 keys without payload may use up to FRMAX
// buckets (one counter per thread): its keys sit in B as offsets from the
// leaf's minimum shifted to the top of the word, whose top bits are the
// bucket, so no bucket byte is stored per key.
constexpr uint32_t FRMAX = FIN_THREADS;
// log2 of the oversampling factor a of a leaf's sample (a = 4, 2, 1; the
// sample a * f holds at most FMAX keys)
AMS_DEV uint32_t leaf_loga(uint32_t logf) { return logf <= 6 ? 2u : 8u - logf; }

template <int KT, bool PAY>
AMS_DEV void lds_sort(const FinSmem<typename Key<KT>::T> &sm,
                      const typename Key<KT>::T *src_, const uint32_t *vsrc_, bool enc_in,
                      typename Key<KT>::T *dst_, uint32_t *vdst_, bool dec_out, uint32_t s,
                      uint32_t C, uint32_t cutoff, uint64_t st, bool sampled_only,
                      uint32_t *nextSlot = nullptr, uint32_t nextVal = 0) {
  typedef typename Key<KT>::T K;
  // global views of the leaf's buffers: global (not flat) loads and stores
  // count only in vmcnt, so the LDS waits of the ranking never wait for them
  const GMem<K> *src = (const GMem<K> *)src_;
  const GMem<uint32_t> *vsrc = (const GMem<uint32_t> *)vsrc_;
  GMem<K> *dst = (GMem<K> *)dst_;
  GMem<uint32_t> *vdst = (GMem<uint32_t> *)vdst_;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t f = leaf_fanout(s, cutoff, FMAX);
  const uint32_t logf = ilog2c(f);
  // placed-position bitmap: position p is bit p / nwb of word p % nwb, so
  // neighbouring positions fall in different words (C <= 32 * nwb)
  constexpr uint32_t nwb = CMAX / 32;
  static_assert(nwb <= 2 * FMAX, "the bitmap lives in the bucket-counter area");
  static_assert(2 * FMAX == FIN_THREADS, "one bucket counter per thread");
  if (!PAY) sm.cnt[tid] = 0;  // keys-only bucket counters (the previous call ended on a barrier)
  K xk[FIN_KPT];
  uint32_t xv[FIN_KPT];
  uint32_t xir[FIN_KPT];  // id << 16 | slot
  // keys into registers; pairs: waves own contiguous ranges (stable split)
  const uint32_t nsteps = (s + 63) / 64, spw = (nsteps + 7) / 8;
  auto slot_pos = [&](uint32_t k) -> uint32_t {
    return PAY ? (wave * spw + k) * 64 + lane : tid + FIN_THREADS * k;
  };
  auto slot_valid = [&](uint32_t k) -> bool {
    return PAY ? (k < spw && slot_pos(k) < s) : slot_pos(k) < s;
  };
#pragma unroll
  for (uint32_t k = 0; k < FIN_KPT; ++k) {
    const uint32_t p = slot_pos(k);
    const bool valid = slot_valid(k);
    K x = valid ? src[p] : (K)0;
    xk[k] = enc_in ? Key<KT>::enc(x) : x;
    if (PAY) xv[k] = valid ? vsrc[p] : 0u;
  }
  // the caller's next leaf, requested before these loads: published once
  // they are in, when its request has long been answered
  if (nextSlot && tid == 0) *nextSlot = gridDim.x + nextVal;

  // Bucket counts, their exclusive scan (bstart) and the largest bucket for
  // ids xir[k] of the valid slots.  Keys only: slot = LDS atomic (the
  // counters are zero on entry); pairs: rank among equal ids of the wave's
  // range by ballots, then per-wave rows, so input order is kept.  Returns
  // the largest bucket; ends with a barrier.
  auto count_scan = [&](uint32_t NB) -> uint32_t {
    uint32_t Lmax = 0;
    if (!PAY) {
#pragma unroll
      for (uint32_t k = 0; k < FIN_KPT; ++k) {
        uint32_t slot = 0;
        if (slot_valid(k)) slot = atomicAdd(&sm.cnt[xir[k]], 1u);
        xir[k] = (xir[k] << 16) | slot;
      }
      __syncthreads();
      const uint32_t cv = tid < NB ? sm.cnt[tid] : 0u;
      const uint32_t inc = wave_incl_scan(cv);
      const uint32_t wmx = wave_max(cv);
      if (lane == 63) {
        sm.wred[wave] = inc;
        sm.wred[8 + wave] = wmx;
      }
      __syncthreads();
      uint32_t off = 0;
#pragma unroll
      for (uint32_t ww = 0; ww < FIN_THREADS / 64; ++ww) {
        off += ww < wave ? sm.wred[ww] : 0u;
        Lmax = sm.wred[8 + ww] > Lmax ? sm.wred[8 + ww] : Lmax;
      }
      if (tid < NB) sm.bstart[tid] = off + inc - cv;
      if (tid == 0) sm.bstart[NB] = s;
      __syncthreads();
    } else {
      const uint32_t nbits = ilog2c(NB);
      for (uint32_t q = tid; q < 8 * NB; q += FIN_THREADS) sm.cnt[q] = 0;
      __syncthreads();
#pragma unroll
      for (uint32_t k = 0; k < FIN_KPT; ++k) {
        const bool valid = slot_valid(k);
        const uint32_t id = valid ? xir[k] : 0u;
        uint64_t peers = match_lanes(id, valid, nbits);
        uint32_t below = bits_below(peers);
        uint32_t r = 0;
        if (valid) {
          uint32_t *c = sm.cnt + wave * NB + id;
          r = *c + below;
          if (below == 0) *c = r + (uint32_t)__popcll(peers);
        }
        xir[k] = (id << 16) | r;
      }
      __syncthreads();
      for (uint32_t id = tid; id < NB; id += FIN_THREADS) {
        uint32_t sum = 0;
        for (uint32_t ww = 0; ww < 8; ++ww) sum += sm.cnt[ww * NB + id];
        sm.bstart[id] = sum;
      }
      __syncthreads();
      block_exscan<FIN_THREADS>(sm.bstart, NB, sm.tmp);
      uint32_t *shMax = sm.wred;
      if (tid == 0) {
        sm.bstart[NB] = s;
        *shMax = 0;
      }
      for (uint32_t id = tid; id < NB; id += FIN_THREADS) {
        uint32_t run = sm.bstart[id];
        for (uint32_t ww = 0; ww < 8; ++ww) {
          uint32_t v = sm.cnt[ww * NB + id];
          sm.cnt[ww * NB + id] = run;
          run += v;
        }
      }
      __syncthreads();
      if (tid < NB) atomicMax(shMax, sm.bstart[tid + 1] - sm.bstart[tid]);
      __syncthreads();
      Lmax = *shMax;
    }
    return Lmax;
  };

  bool eq = false;
  uint32_t NB = 1, Lb = 0;
  bool split = false;  // xir / bstart hold an accepted split
  // uint64 keys only: B holds z = (x - zmn) << zlsh, the offset from the
  // leaf's minimum shifted to the top of the word.  z is monotone in x and
  // its high 32 bits order any two keys whose offsets differ in their
  // leading 32 significant bits, so the ranking compares 32-bit words; keys
  // that tie there share a rank and are put right by the exact pass at the
  // end, like equal keys.
  constexpr bool ZT = KT == KT_U64 && !PAY;
  bool zt = false;
  K zmn = 0;
  uint32_t zlsh = 0;
  // range split of offsets with up to FRMAX buckets: the bucket of the key
  // at B[p] is B[p] >> zbs, and bid is not written
  bool zbuck = false;
  uint32_t zbs = 0;
  const uint32_t fr = ZT ? leaf_fanout(s, cutoff, FRMAX) : f;  // range split's fan-out
  const uint32_t logfr = ilog2c(fr);
  if (fr > 1 && !sampled_only) {
    // ---- split by key range.  After the partition levels a leaf covers a
    // narrow range of keys, which most inputs fill about evenly; bucket b(x)
    // = (x - min) >> sh with sh chosen so that b < f.  b is monotone in x, so
    // buckets follow key order and equal keys share a bucket.  The split is
    // kept when no bucket exceeds 4x the average (at least 64 keys); else
    // the sampled split below is used.
    K mn = (K)~(K)0, mx = (K)0;
#pragma unroll
    for (uint32_t k = 0; k < FIN_KPT; ++k) {
      if (slot_valid(k)) {
        mn = xk[k] < mn ? xk[k] : mn;
        mx = xk[k] > mx ? xk[k] : mx;
      }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    K *red = sm.srt;  // per-wave minima and maxima (the splitters are not drawn yet)
    if (lane == 0) {
      red[wave] = mn;
      red[8 + wave] = mx;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t ww = 0; ww < FIN_THREADS / 64; ++ww) {
      mn = red[ww] < mn ? red[ww] : mn;
      mx = red[8 + ww] > mx ? red[8 + ww] : mx;
    }
    const K range = mx - mn;
    const uint32_t bits = range ? (uint32_t)(8 * sizeof(K)) - (uint32_t)(sizeof(K) == 8
                                       ? __builtin_clzll((unsigned long long)range)
                                       : __builtin_clz((uint32_t)range))
                                : 0u;
    const uint32_t sh = bits > logfr ? bits - logfr : 0u;
#pragma unroll
    for (uint32_t k = 0; k < FIN_KPT; ++k)
      xir[k] = slot_valid(k) ? (uint32_t)((xk[k] - mn) >> sh) : 0u;
    if (ZT && bits > 0) {
      zt = true;
      zmn = mn;
      zlsh = (uint32_t)(8 * sizeof(K)) - bits;
    }
    NB = fr;
    Lb = count_scan(NB);
    const uint32_t avg = (s + fr - 1) / fr;
    split = Lb <= (4 * avg > 64 ? 4 * avg : 64);
    if (!split && !PAY) sm.cnt[tid] = 0;  // counters for the sampled split
    zbuck = ZT && zt && split;
    zbs = zlsh + sh;  // z >> (64 - bits) is x - mn; >> sh more is the bucket
  }
  if (f > 1 && !split) {
    // ---- sampled split: S = a*f keys at random positions of the leaf
    // (SplitMix64 stream); the splitters are the sorted sample's elements of
    // rank a*j - 1, j = 1..f-1.  At most FMAX samples: ranking a larger
    // sample costs more than the better balanced buckets save in the
    // all-pairs step.  Sizes are powers of two (shifts only).
    const uint32_t loga = leaf_loga(logf);               // a = 4, 2, 1
    const uint32_t logS = logf + loga;                   // S <= FMAX = 256
    const uint32_t logH = 9u - logS < 3u ? 9u - logS : 3u;  // H = min(512 / S, 8)
    const uint32_t S = 1u << logS, H = 1u << logH, amask = (1u << loga) - 1u;
    if (tid < S) {
      const K y = src[draw_pos(st, tid, s)];
      sm.smp[tid] = enc_in ? Key<KT>::enc(y) : y;
    }
    __syncthreads();
    // Rank the sample (Section 4.2): inside blocks of up to 64 by comparing
    // all pairs, then across blocks by binary search.  H adjacent lanes share
    // one sample and add their partial counts.  Ties are broken by index, so
    // every sampled key gets a distinct rank.
    const uint32_t bsz = S < 64 ? S : 64, nbk = (S + 63) >> 6;
    const uint32_t i = tid >> logH, part = tid & (H - 1u);
    const bool act = i < S;
    {
      const uint32_t b0 = act ? i & ~63u : 0u, iw = i & 63u;
      const K x = sm.smp[act ? i : 0u];
      const uint32_t chunk = (bsz + H - 1) >> logH;
      const uint32_t j0 = part * chunk < bsz ? part * chunk : bsz;
      const uint32_t j1 = j0 + chunk < bsz ? j0 + chunk : bsz;
      uint32_t c[4] = {0, 0, 0, 0};
      uint32_t j = j0;
      for (; j + 4 <= j1; j += 4) {
        K y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = sm.smp[b0 + j + u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          c[u] += (uint32_t)(y[u] < x) | ((uint32_t)(y[u] == x) & (uint32_t)(j + u < iw));
      }
      for (; j < j1; ++j) {
        const K y = sm.smp[b0 + j];
        c[0] += (uint32_t)(y < x) | ((uint32_t)(y == x) & (uint32_t)(j < iw));
      }
      uint32_t r = (c[0] + c[1]) + (c[2] + c[3]);
      for (uint32_t d = 1; d < H; d <<= 1) r += __shfl_xor(r, (int)d, 64);
      if (act && part == 0) {
        if (nbk > 1) sm.blk[b0 + r] = x;
        else if (((r + 1) & amask) == 0 && ((r + 1) >> loga) < f) sm.srt[(r + 1) >> loga] = x;
      }
    }
    __syncthreads();
    if (nbk > 1) {
      // full blocks of 64 (S = 128 or 256): the H lanes of a sample split
      // the other blocks among them (see cross_block_rank); a wave ranks
      // keys of one block
      const uint32_t b = act ? i >> 6 : 0u;
      const K x = sm.blk[act ? i : 0u];
      static_assert(FMAX == 256, "a sample of at most 4 blocks");
      uint32_t r = nbk * 2 > H ? cross_block_rank<K, 2>(sm.blk, b, x, part, H, nbk)
                               : cross_block_rank<K, 1>(sm.blk, b, x, part, H, nbk);
      for (uint32_t d = 1; d < H; d <<= 1) r += __shfl_xor(r, (int)d, 64);
      r += i & 63u;
      if (act && part == 0 && ((r + 1) & amask) == 0 && ((r + 1) >> loga) < f)
        sm.srt[(r + 1) >> loga] = x;
      __syncthreads();
    }
    bool dup = false;
    if (tid >= 1 && tid < f) {
      sm.tree[eytzinger_slot(tid, f)] = sm.srt[tid];
      dup = tid + 1 < f && sm.srt[tid] == sm.srt[tid + 1];
    }
    eq = __syncthreads_or(dup ? 1 : 0) != 0;
    classify_halves<K>(xk, xir, sm.tree, logf, eq, s);
    NB = eq ? 2 * f - 1 : f;
    Lb = count_scan(NB);
  } else if (f == 1) {
#pragma unroll
    for (uint32_t k = 0; k < FIN_KPT; ++k) xir[k] = 0;
    __syncthreads();  // keys-only counters were cleared on entry
    NB = 1;
    Lb = count_scan(NB);
  }
  if (tid < 65) ((uint32_t *)sm.srt)[tid] = 0;  // work-order counters (splitters are done)
  // ---- place every key at its bucket's range in B
#pragma unroll
  for (uint32_t k = 0; k < FIN_KPT; ++k) {
    if (slot_valid(k)) {
      const uint32_t id = xir[k] >> 16;
      const uint32_t q = (PAY ? sm.cnt[wave * NB + id] : sm.bstart[id]) + (xir[k] & 0xFFFFu);
      sm.B[q] = (ZT && zt) ? (K)((xk[k] - zmn) << zlsh) : xk[k];
      if (PAY) sm.vB[q] = xv[k];
      if (!eq && !zbuck) sm.bid[q] = (uint8_t)id;  // direct order: ids < f <= 256
    }
  }
  if (s + Lb + 8 <= C + FIN_PAD)
    for (uint32_t q = s + tid; q < s + Lb + 8; q += FIN_THREADS) sm.B[q] = (K)~(K)0;
  __syncthreads();
  // scans of at most Lb + 7 slots past a bucket start stay inside B
  const bool padded = s + Lb + 8 <= C + FIN_PAD;
  // Direct order (no equality buckets): lane slot p ranks the key at B
  // position p, whose bucket id the placement wrote to bid[p].  The
  // buckets of one split are about equally long, so a wavefront's trip
  // count is close to its lanes' own without regrouping them.
  const bool direct = !eq;
  // ---- work order.  A wavefront ranks its keys in a common trip count,
  // the longest bucket among its lanes, so the keys are handed to lanes
  // bucket by bucket in order of decreasing bucket size (64 size classes):
  // a wavefront then holds buckets of about one size.  Equality buckets
  // come last (class 64); their keys are not ranked.  Buckets of a class
  // follow one another in the order their atomic adds happened.  Lane slot
  // p belongs to bucket id map(p) and holds the key at B position
  // bstart[id] + p - lofs[id].
  uint16_t *lofs = PAY ? (uint16_t *)sm.cnt : (uint16_t *)(sm.cnt + nwb);  // NB first slots
  uint32_t *hist = (uint32_t *)sm.srt;  // keys per class (cleared in the split); [64]: start of equality slots
  // keys only, after hist in the same area: one flag byte per bucket whose
  // keys tied in the ranking, then a word set when any bucket has one
  constexpr uint32_t TIED_WORDS = 2 * FMAX / 4;
  static_assert((68 + TIED_WORDS + 1) * 4 <= FMAX * sizeof(K), "tie flags fit the splitter area");
  uint32_t *tiedw = hist + 68;
  uint8_t *tied = (uint8_t *)tiedw;
  uint32_t *anyTied = tiedw + TIED_WORDS;
  if (!direct) {
    const bool haveId = tid < NB;
    const bool eqId = eq && (tid & 1u);
    uint32_t L = 0, cls = 0, kslot = 0;
    if (haveId) {
      L = sm.bstart[tid + 1] - sm.bstart[tid];
      cls = eqId ? 64u : 63u - (L < 63u ? L : 63u);
      kslot = atomicAdd(&hist[cls], L);
    }
    __syncthreads();
    if (wave == 0) {  // class starts: exclusive scan of classes 0..63, class 64 after them
      const uint32_t c = hist[lane];
      const uint32_t inc = wave_incl_scan(c);
      hist[lane] = inc - c;
      if (lane == 63) hist[64] = inc;
    }
    __syncthreads();
    if (haveId) {
      const uint32_t lo = hist[cls] + kslot;
      lofs[tid] = (uint16_t)lo;
      const uint32_t bb = eq ? tid >> 1 : tid, word = bb * 0x01010101u;
      uint32_t j = lo;
      const uint32_t hi = lo + L;
      for (; j < hi && (j & 3u); ++j) sm.bid[j] = (uint8_t)bb;
      for (; j + 4 <= hi; j += 4) *(uint32_t *)(sm.bid + j) = word;
      for (; j < hi; ++j) sm.bid[j] = (uint8_t)bb;
    }
  }
  if (!PAY) {
    for (uint32_t w32 = tid; w32 < nwb; w32 += FIN_THREADS) sm.bm[w32] = 0;
    for (uint32_t w32 = tid; w32 <= TIED_WORDS; w32 += FIN_THREADS) tiedw[w32] = 0;
  }
  __syncthreads();
  const uint32_t eqStart = direct ? s : hist[64];
  // ---- all-pairs rank inside every bucket, one slot of FIN_THREADS keys
  // per pass.  B is not modified while ranking, so every key goes straight
  // to its final position in dst once its rank is known.
  // slots ranked together on the offset path, and elements read per slot
  // and trip
  constexpr uint32_t RNS = 3, RNU = 4;
  struct RankSlot {
    K x;
    uint32_t id, bs, q, len, v;
    bool valid, isEq;
  };
  // lane slot k: its bucket, its key and the length to scan
  auto rank_slot = [&](uint32_t k) -> RankSlot {
    RankSlot r;
    const uint32_t ps = tid + FIN_THREADS * k;
    r.valid = ps < s;
    const uint32_t pv = r.valid ? ps : 0u;
    const uint32_t b = zbuck ? (uint32_t)((uint64_t)sm.B[pv] >> zbs) : (uint32_t)sm.bid[pv];
    r.isEq = eq && pv >= eqStart;  // equal keys: any arrangement is final
    const uint32_t id = eq ? 2 * b + (r.isEq ? 1u : 0u) : b;
    r.id = id;
    r.bs = sm.bstart[id];
    const uint32_t be = sm.bstart[id + 1];
    r.q = direct ? pv : r.bs + pv - lofs[id];
    r.x = sm.B[r.q];
    r.len = (r.valid && !r.isEq) ? be - r.bs : 0u;
    r.v = PAY ? sm.vB[r.q] : 0u;
    return r;
  };
  auto emit = [&](const RankSlot &r, uint32_t rk) {
    if (r.valid) {
      const uint32_t pos = r.isEq ? r.q : r.bs + rk;
      const K xr = (ZT && zt) ? (K)(zmn + ((uint64_t)r.x >> zlsh)) : r.x;
      const K out = dec_out ? Key<KT>::dec(xr) : xr;
      // keys-only: equal keys share a rank, so they all land on its first
      // position; every written position is marked (no return value, so the
      // store does not wait) and the positions left empty are filled below;
      // a wavefront's marks hit different words and do not serialise
      if (!PAY) atomicOr(&sm.bm[pos % nwb], 1u << (pos / nwb));
      dst[pos] = out;
      if (PAY) vdst[pos] = r.v;
    }
  };
#pragma unroll 1
  for (uint32_t k = 0; k < FIN_KPT;) {
    if (FIN_THREADS * k >= s) break;  // uniform: no key in this or later slots
    if (padded && k + RNS <= FIN_KPT) {
      // RNS slots at a time so that their LDS reads overlap; every scan
      // runs to the longest trip count, which is safe past a bucket's end
      // (later buckets and the pad hold larger values)
      RankSlot r[RNS];
      uint32_t lm = 0;
#pragma unroll
      for (uint32_t j = 0; j < RNS; ++j) {
        r[j] = rank_slot(k + j);
        lm = r[j].len > lm ? r[j].len : lm;
      }
      const uint32_t ml = __builtin_amdgcn_readfirstlane(wave_max(lm));
      // T: the compared word, the high 32 bits of an offset (odd 32-bit
      // words of B) or the whole key
      auto scan = [&](auto tag) {
        typedef decltype(tag) T;
        constexpr uint32_t STEP = (uint32_t)(sizeof(K) / sizeof(T));
        const T *a[RNS];
        T xw[RNS];
        uint32_t c[RNS][2], qb[RNS];
#pragma unroll
        for (uint32_t j = 0; j < RNS; ++j) {
          qb[j] = r[j].q - r[j].bs;  // the key's own position in its bucket
          a[j] = (const T *)(sm.B + r[j].bs) + (STEP - 1);
          if constexpr (sizeof(T) < sizeof(K)) xw[j] = (T)((uint64_t)r[j].x >> 32);
          else xw[j] = (T)r[j].x;
          c[j][0] = c[j][1] = 0;
        }
        for (uint32_t d = 0; d < ml; d += RNU) {
          T y[RNS][RNU];
#pragma unroll
          for (uint32_t u = 0; u < RNU; ++u)
#pragma unroll
            for (uint32_t j = 0; j < RNS; ++j) y[j][u] = a[j][STEP * (d + u)];
          if constexpr (sizeof(K) == 4 || PAY) {
            // 32-bit keys repeat often, and pairs must keep input order:
            // equal keys are ordered by their position in B here (input
            // order for pairs), so no position is left empty
#pragma unroll
            for (uint32_t u = 0; u < RNU; ++u)
#pragma unroll
              for (uint32_t j = 0; j < RNS; ++j)
                c[j][u & 1] += (uint32_t)(y[j][u] < xw[j]) |
                               ((uint32_t)(y[j][u] == xw[j]) & (uint32_t)(d + u < qb[j]));
          } else {
#pragma unroll
            for (uint32_t u = 0; u < RNU; ++u)
#pragma unroll
              for (uint32_t j = 0; j < RNS; ++j) c[j][u & 1] += (uint32_t)(y[j][u] < xw[j]);
          }
        }
#pragma unroll
        for (uint32_t j = 0; j < RNS; ++j) emit(r[j], c[j][0] + c[j][1]);
      };
      if (ZT && zt) scan(uint32_t{});
      else scan(K{});
      k += RNS;
      continue;
    }
    const RankSlot r = rank_slot(k);
    const K x = r.x;
    // wave-uniform trip count, held in a scalar register
    const uint32_t ml = __builtin_amdgcn_readfirstlane(wave_max(r.len));
    uint32_t rk = 0;
    if (padded) {
      const K *a = sm.B + r.bs;
      // one counter per unrolled element: each compare then feeds a single
      // add-with-carry instead of a packed mask and a population count
      uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (ZT && zt) {
        // high words of the offsets (odd 32-bit words of B), 32-bit compares
        const uint32_t *a32 = (const uint32_t *)a + 1;
        const uint32_t xw = (uint32_t)((uint64_t)x >> 32);
        for (uint32_t d = 0; d < ml; d += 8) {
          uint32_t y[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) y[u] = a32[2 * (d + u)];
#pragma unroll
          for (int u = 0; u < 8; ++u) c[u] += (uint32_t)(y[u] < xw);
        }
      } else if (!PAY) {
        for (uint32_t d = 0; d < ml; d += 8) {
          K y[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) y[u] = a[d + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) c[u] += (uint32_t)(y[u] < x);
        }
      } else {
        const uint32_t qb = r.q - r.bs;  // j < q  <=>  d + u < qb
        for (uint32_t d = 0; d < ml; d += 8) {
          K y[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) y[u] = a[d + u];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            c[u] += (uint32_t)(y[u] < x) | ((uint32_t)(y[u] == x) & (uint32_t)(d + u < qb));
        }
      }
      rk = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
    } else {
      for (uint32_t d = 0; d < ml; d += 4) {
        K y[4];
        uint32_t jj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          jj[u] = d + u < r.len ? r.bs + d + u : r.q;
          y[u] = sm.B[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          rk += (uint32_t)(d + u < r.len) &
                ((uint32_t)(y[u] < x) | ((uint32_t)(y[u] == x) & (uint32_t)(jj[u] < r.q)));
      }
    }
    emit(r, rk);
    ++k;
  }
  __syncthreads();
  if (!PAY) {
    // An empty position follows a run of keys that tied at one rank in
    // their bucket (equal keys or, with offsets, equal high words): flag
    // the buckets that hold empty positions.
    for (uint32_t wi = tid; wi < nwb; wi += FIN_THREADS) {
      // bits b of word wi with b * nwb + wi < s
      const uint32_t nb = wi < s ? (s - wi + nwb - 1) / nwb : 0u;
      const uint32_t full = nb >= 32 ? 0xFFFFFFFFu : (1u << nb) - 1u;
      uint32_t holes = full & ~sm.bm[wi];
      while (holes) {
        const uint32_t p = (uint32_t)__builtin_ctz(holes) * nwb + wi;
        holes &= holes - 1u;
        // the bucket holding position p: the last id whose start is <= p
        uint32_t id = 0;
        for (uint32_t span = 1u << ilog2c(NB); span; span >>= 1)
          if (id + span < NB && sm.bstart[id + span] <= p) id += span;
        tied[id] = 1;
        *anyTied = 1;
      }
    }
    __syncthreads();
    if (*anyTied) {
      // The keys of flagged buckets are ranked again with the full keys,
      // ties broken by position in B, which gives every key its own
      // position; all of the bucket is written again.  The first writes
      // must be complete before the second ones are issued.
      __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
#pragma unroll 1
      for (uint32_t k = 0; k < FIN_KPT; ++k) {
        if (FIN_THREADS * k >= s) break;
        const RankSlot r = rank_slot(k);
        if (r.valid && !r.isEq && tied[r.id]) {
          const uint32_t qb = r.q - r.bs;
          uint32_t rk = 0;
          for (uint32_t j = 0; j < r.len; ++j) {
            const K y = sm.B[r.bs + j];
            rk += (uint32_t)(y < r.x) | ((uint32_t)(y == r.x) & (uint32_t)(j < qb));
          }
          const K xr = (ZT && zt) ? (K)(zmn + ((uint64_t)r.x >> zlsh)) : r.x;
          dst[r.bs + rk] = dec_out ? Key<KT>::dec(xr) : xr;
        }
      }
    }
    __syncthreads();
  }
}

// Stable merge of sorted A[0..na) and B[0..nb) (A first on ties) into out,
// split across the workgroup by output position (merge path).
template <int KT, bool PAY>
AMS_DEV void wg_merge(const typename Key<KT>::T *A_, const uint32_t *vA_, uint32_t na,
                      const typename Key<KT>::T *B_, const uint32_t *vB_, uint32_t nb,
                      typename Key<KT>::T *out_, uint32_t *vout_, bool dec_out) {
  typedef typename Key<KT>::T K;
  const GMem<K> *A = (const GMem<K> *)A_, *B = (const GMem<K> *)B_;
  const GMem<uint32_t> *vA = (const GMem<uint32_t> *)vA_, *vB = (const GMem<uint32_t> *)vB_;
  GMem<K> *out = (GMem<K> *)out_;
  GMem<uint32_t> *vout = (GMem<uint32_t> *)vout_;
  const uint32_t len = na + nb;
  const uint32_t per = (len + FIN_THREADS - 1) / FIN_THREADS;
  const uint32_t k0 = threadIdx.x * per < len ? threadIdx.x * per : len;
  const uint32_t k1 = k0 + per < len ? k0 + per : len;
  if (k0 >= k1) return;
  // co-rank: number of A elements among the first k0 outputs
  uint32_t lo = k0 > nb ? k0 - nb : 0, hi = k0 < na ? k0 : na;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (A[mid] <= B[k0 - mid - 1]) lo = mid + 1; else hi = mid;
  }
  uint32_t i = lo, j = k0 - lo;
  for (uint32_t k = k0; k < k1; ++k) {
    bool takeA = j >= nb || (i < na && A[i] <= B[j]);
    K x;
    uint32_t v = 0;
    if (takeA) {
      x = A[i];
      if (PAY) v = vA[i];
      ++i;
    } else {
      x = B[j];
      if (PAY) v = vB[j];
      ++j;
    }
    out[k] = dec_out ? Key<KT>::dec(x) : x;
    if (PAY) vout[k] = v;
  }
}

// Last resort for a range of n > C keys that the partition below could not
// split into pieces of at most C: runs of C keys sorted in LDS, then pairs of
// runs merged, ping-ponging between the range's TMP and OUT buffers so that
// the last pass lands in OUT.  src may be either buffer (a run is read
// completely before it is written).
template <int KT, bool PAY>
AMS_DEV void merge_fallback(const Ws &w, const Root &R, uint32_t off, uint32_t n,
                            const typename Key<KT>::T *src, const uint32_t *vsrc, bool enc_in,
                            const FinSmem<typename Key<KT>::T> &sm, uint32_t C, uint32_t cutoff,
                            uint64_t seed, uint32_t root, bool sampled_only) {
  typedef typename Key<KT>::T K;
  if (threadIdx.x == 0) {
    atomicAdd(&w.ctr->nmerge, 1u);
    atomicAdd(&w.ctr->merge_keys, (unsigned long long)n);
  }
  const uint32_t runs = (n + C - 1) / C;
  const uint32_t passes = ilog2c(runs);
  K *bufK[2] = {kptr<K>(w, R, BUF_TMP) + off, kptr<K>(w, R, BUF_OUT) + off};
  uint32_t *bufV[2] = {PAY ? vptr(w, R, BUF_TMP) + off : nullptr,
                       PAY ? vptr(w, R, BUF_OUT) + off : nullptr};
  uint32_t curb = (passes & 1u) ? 0u : 1u;  // run buffer: OUT after an even number of passes
  for (uint32_t r = 0; r < runs; ++r) {
    uint32_t o = r * C, sz = n - o < C ? n - o : C;
    lds_sort<KT, PAY>(sm, src + o, PAY ? vsrc + o : nullptr, enc_in, bufK[curb] + o,
                      PAY ? bufV[curb] + o : nullptr, passes == 0, sz, C, cutoff,
                      stream_state(seed, LEAF_STREAM, root, off + o), sampled_only);
  }
  for (uint32_t pz = 0; pz < passes; ++pz) {
    const uint32_t width = C << pz;
    const uint32_t nxt = curb ^ 1u;
    const bool last = pz + 1 == passes;
    for (uint32_t a = 0; a < n; a += 2 * width) {
      uint32_t na = n - a < width ? n - a : width;
      uint32_t nb = n - a - na < width ? n - a - na : width;
      wg_merge<KT, PAY>(bufK[curb] + a, PAY ? bufV[curb] + a : nullptr, na,
                        bufK[curb] + a + na, PAY ? bufV[curb] + a + na : nullptr, nb,
                        bufK[nxt] + a, PAY ? bufV[nxt] + a : nullptr, last);
    }
    __syncthreads();
    curb = nxt;
  }
}

// An oversized leaf (a group larger than the base case's capacity C after
// the planned levels) gets one more partition level, in HBM, from the
// workgroup that owns it (Section 6: groups are split again until they fit
// a processor).  16 f keys at random positions are ranked in LDS; f - 1 of
// them split the leaf into f buckets of about n / f <= C / 4 keys, with an
// equality bucket after every splitter (Appendix D; 2f - 1 ids in key order).
// A count pass and a stable scatter pass move the keys bucket by bucket into
// the range's other buffer (TMP or OUT, the one the leaf is not in).  The
// caller then sorts every bucket of at most C keys in LDS into OUT, copies
// the equality buckets (their keys are equal) and hands a bucket still
// larger than C on: it is partitioned once more, and what is still larger
// than C after that goes to the merge fallback.
constexpr uint32_t BIG_A = 16;         // samples per bucket
constexpr uint32_t BIG_SAMPLE = 1024;  // sample room (BIG_A * BIG_FMAX)
constexpr uint32_t BIG_FMAX = 64;          // buckets per partition
constexpr uint32_t BIG_IDS = 2 * BIG_FMAX;  // ids (2f - 1 used), one counter each
constexpr uint32_t BIG_RPT = 8;             // keys per thread and count or scatter chunk
static_assert(BIG_A * BIG_FMAX <= BIG_SAMPLE, "the sample fits its LDS room");
// LDS of the partition: sample, sorted sample, splitters, then the counters
template <typename K> __host__ __device__ constexpr size_t big_smem_bytes() {
  return (2 * BIG_SAMPLE + BIG_FMAX) * sizeof(K) +
         (BIG_IDS + 1 + BIG_IDS + (FIN_THREADS / 64) * BIG_IDS) * sizeof(uint32_t);
}

// Returns the number of ids NB; lane l of every wavefront receives the
// starts of buckets l and l + 64 in bs0 and bs1 (bucket_start), start NB
// being the leaf's size.  The buckets sit in buffer sbuf of the leaf's range.
template <int KT, bool PAY>
AMS_DEV uint32_t big_partition(const Ws &w, const Root &R, const Seg &L, unsigned char *smem,
                               uint32_t C, uint64_t seed, uint32_t sbuf, uint32_t &bs0,
                               uint32_t &bs1) {
  typedef typename Key<KT>::T K;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  constexpr uint32_t NW = FIN_THREADS / 64;
  const uint32_t n = L.size, buf = seg_buf(L.meta);
  const bool enc = buf == BUF_IN;
  const GMem<K> *src = (const GMem<K> *)(kptr<K>(w, R, buf) + L.off);
  const GMem<uint32_t> *vsrc = PAY ? (const GMem<uint32_t> *)(vptr(w, R, buf) + L.off) : nullptr;
  K *stK_ = kptr<K>(w, R, sbuf) + L.off;
  uint32_t *stV_ = PAY ? vptr(w, R, sbuf) + L.off : nullptr;
  GMem<K> *stK = (GMem<K> *)stK_;
  GMem<uint32_t> *stV = (GMem<uint32_t> *)stV_;
  // LDS (the base case's layout is not in use until the buckets are sorted)
  K *smp = (K *)smem;                       // BIG_SAMPLE sample keys
  K *srt = smp + BIG_SAMPLE;                // the sample in order
  K *spl = srt + BIG_SAMPLE;                // spl[1..f-1]: splitters
  uint32_t *hist = (uint32_t *)(spl + BIG_FMAX);  // BIG_IDS + 1: counts, then starts
  uint32_t *cur = hist + BIG_IDS + 1;             // BIG_IDS: next free slot per id
  uint32_t *rows = cur + BIG_IDS;                 // NW x BIG_IDS: per-wave counts, then bases
  // f: the smallest power of two with n / f <= C / 4 (at least 2, at most BIG_FMAX)
  uint32_t f = 2;
  while (f < BIG_FMAX && (uint64_t)f * (C / 4) < n) f <<= 1;
  const uint32_t logf = ilog2c(f), NB = 2 * f - 1, S = BIG_A * f;
  // ---- sample and splitters
  const uint64_t st = stream_state(seed, LEAF_STREAM - 1, L.root, L.off);
  for (uint32_t t = tid; t < S; t += FIN_THREADS) {
    const K y = src[draw_pos(st, t, n)];
    smp[t] = enc ? Key<KT>::enc(y) : y;
  }
  for (uint32_t q = tid; q < BIG_IDS + 1; q += FIN_THREADS) hist[q] = 0;
  for (uint32_t q = tid; q < NW * BIG_IDS; q += FIN_THREADS) rows[q] = 0;
  __syncthreads();
  for (uint32_t t = tid; t < S; t += FIN_THREADS) {
    // rank among all samples, ties broken by index (Section 4.2)
    const K x = smp[t];
    uint32_t r = 0;
    for (uint32_t j = 0; j < S; ++j) {
      const K y = smp[j];
      r += (uint32_t)(y < x) | ((uint32_t)(y == x) & (uint32_t)(j < t));
    }
    srt[r] = x;
  }
  __syncthreads();
  if (tid >= 1 && tid < f) spl[tid] = srt[BIG_A * tid - 1];
  __syncthreads();
  // id of x: 2b for the regular bucket b (b = splitters below x), 2b + 1 when
  // x equals the splitter above it
  auto classify_big = [&](K x) -> uint32_t {
    uint32_t b = 0;
    for (uint32_t half = f >> 1; half; half >>= 1)
      if (b + half < f && spl[b + half] < x) b += half;
    const bool eqb = b + 1 < f && spl[b + 1] == x;
    return 2 * b + (eqb ? 1u : 0u);
  };
  // ---- count (BIG_RPT loads per thread in flight at a time)
  for (uint32_t base = 0; base < n; base += FIN_THREADS * BIG_RPT) {
    K xs[BIG_RPT];
#pragma unroll
    for (uint32_t k = 0; k < BIG_RPT; ++k) {
      const uint32_t p = base + k * FIN_THREADS + tid;
      xs[k] = p < n ? (K)src[p] : (K)0;
    }
#pragma unroll
    for (uint32_t k = 0; k < BIG_RPT; ++k) {
      if (base + k * FIN_THREADS + tid < n)
        atomicAdd(&hist[classify_big(enc ? Key<KT>::enc(xs[k]) : xs[k])], 1u);
    }
  }
  __syncthreads();
  if (wave == 0) {  // exclusive scan of the NB <= 127 counts, two per lane
    const uint32_t c0 = 2 * lane < NB ? hist[2 * lane] : 0u;
    const uint32_t c1 = 2 * lane + 1 < NB ? hist[2 * lane + 1] : 0u;
    const uint32_t inc = wave_incl_scan(c0 + c1);
    const uint32_t e = inc - c0 - c1;
    if (2 * lane < NB) cur[2 * lane] = e;
    if (2 * lane + 1 < NB) cur[2 * lane + 1] = e + c0;
  }
  __syncthreads();
  for (uint32_t q = tid; q < NB; q += FIN_THREADS) hist[q] = cur[q];  // bucket starts
  if (tid == 0) hist[NB] = n;
  // ---- stable scatter: wavefront v takes the v-th eighth of each chunk of
  // FIN_THREADS * BIG_RPT keys, as BIG_RPT rows of 64 keys in input order
  for (uint32_t base = 0; base < n; base += FIN_THREADS * BIG_RPT) {
    K xs[BIG_RPT];
    uint32_t vs[BIG_RPT], ir[BIG_RPT];  // id << 16 | rank inside the wavefront's range
#pragma unroll
    for (uint32_t k = 0; k < BIG_RPT; ++k) {  // every load of the chunk first
      const uint32_t p = base + (wave * BIG_RPT + k) * 64 + lane;
      const bool valid = p < n;
      xs[k] = valid ? (K)src[p] : (K)0;
      vs[k] = (PAY && valid) ? (uint32_t)vsrc[p] : 0u;
    }
#pragma unroll
    for (uint32_t k = 0; k < BIG_RPT; ++k) {
      const uint32_t p = base + (wave * BIG_RPT + k) * 64 + lane;
      const bool valid = p < n;
      if (enc) xs[k] = Key<KT>::enc(xs[k]);
      const K x = xs[k];
      const uint32_t id = valid ? classify_big(x) : 0u;
      const uint64_t peers = match_lanes(id, valid, logf + 1);
      const uint32_t below = bits_below(peers);
      uint32_t r = 0;
      if (valid) {
        uint32_t *c = rows + wave * BIG_IDS + id;
        r = *c + below;
        if (below == 0) *c = r + (uint32_t)__popcll(peers);
      }
      ir[k] = valid ? (id << 16) | r : 0xFFFFFFFFu;
    }
    __syncthreads();
    if (tid < NB) {  // per id: wavefront bases in order, then the next free slot
      uint32_t run = cur[tid];
      for (uint32_t v = 0; v < NW; ++v) {
        const uint32_t c = rows[v * BIG_IDS + tid];
        rows[v * BIG_IDS + tid] = run;
        run += c;
      }
      cur[tid] = run;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < BIG_RPT; ++k) {
      if (ir[k] != 0xFFFFFFFFu) {
        const uint32_t d = rows[wave * BIG_IDS + (ir[k] >> 16)] + (ir[k] & 0xFFFFu);
        stK[d] = xs[k];
        if (PAY) stV[d] = vs[k];
      }
    }
    __syncthreads();
    for (uint32_t q = tid; q < NW * BIG_IDS; q += FIN_THREADS) rows[q] = 0;
    __syncthreads();
  }
  // bucket starts into registers (the LDS is handed to the base case next)
  bs0 = lane <= NB ? hist[lane] : n;
  bs1 = lane + 64 <= NB ? hist[lane + 64] : n;
  // the stores above must be complete before the buckets are read back
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  return NB;
}

AMS_DEV uint32_t bucket_start(uint32_t bs0, uint32_t bs1, uint32_t id) {
  return id < 64 ? (uint32_t)__builtin_amdgcn_readlane((int)bs0, (int)id)
                 : (uint32_t)__builtin_amdgcn_readlane((int)bs1, (int)(id - 64));
}

// Keys of an equality bucket are equal: copied in order (decoded).
template <int KT, bool PAY>
AMS_DEV void copy_range(const typename Key<KT>::T *src, const uint32_t *vsrc,
                        typename Key<KT>::T *dst, uint32_t *vdst, uint32_t n) {
  typedef typename Key<KT>::T K;
  for (uint32_t q = threadIdx.x; q < n; q += FIN_THREADS) {
    ((GMem<K> *)dst)[q] = Key<KT>::dec(((const GMem<K> *)src)[q]);
    if (PAY) ((GMem<uint32_t> *)vdst)[q] = ((const GMem<uint32_t> *)vsrc)[q];
  }
}

// Oversized leaves, before the base case: each is partitioned once more by one
// workgroup (big_partition).  Its buckets join the leaf list that k_finish
// sorts (regular buckets as leaves, equality buckets as copies, all of one
// partition in one block of entries).  A regular bucket still larger than C,
// and every bucket when the leaf list has no room left, goes to the
// remainder list that k_big_rest finishes after the base case.  No base
// case in this kernel: it needs little LDS and few registers, so many
// workgroups partition side by side.
template <int KT, bool PAY>
__global__ void __launch_bounds__(FIN_THREADS, PAY ? 4 : 8) k_big_part(Ws w, uint32_t C, uint64_t seed,
                                                             uint32_t flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ uint32_t sSlot;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  uint32_t nb = w.ctr->nbl;
  if (nb > w.capBig) nb = w.capBig;
  for (uint32_t li = blockIdx.x; li < nb; li += gridDim.x) {
    const Seg L = w.bigLeaves[li];
    const Root R = w.roots[L.root];
    if ((uint64_t)L.off + L.size > R.n || seg_kind(L.meta) != LEAF_BIG) {
      if (tid == 0) raise_error(w.ctr, 32u);
      continue;
    }
    const uint32_t sbuf = seg_buf(L.meta) == BUF_OUT ? BUF_TMP : BUF_OUT;
    uint32_t b0, b1;
    const uint32_t NB = big_partition<KT, PAY>(w, R, L, smem_raw, C, seed, sbuf, b0, b1);
    if (tid == 0) sSlot = atomicAdd(&w.ctr->nleaf, NB);
    __syncthreads();
    const uint32_t base = sSlot;
    __syncthreads();
    const bool room = (uint64_t)base + NB <= w.capLeaf && !(flags & AMS_FLAG_TEST_NO_PIECE_ROOM);
    if (!room && tid == 0) {
      // no room for its pieces: the whole leaf goes to the remainder list
      const uint32_t r = atomicAdd(&w.ctr->nrest, 1u);
      if (r < 2 * w.capBig) w.bigLeaves[w.capBig + r] = L; else raise_error(w.ctr, 1u);
    }
    if (tid < 64) {
#pragma unroll
      for (uint32_t h = 0; h < 2; ++h) {
        const uint32_t id = lane + 64 * h;
        // starts of buckets id and id + 1 (every lane takes part in the shuffles)
        const uint32_t s0 = __shfl(b0, (int)(id & 63u), 64), s1 = __shfl(b1, (int)(id & 63u), 64);
        const uint32_t n1 = (id + 1) & 63u;
        const uint32_t e0 = __shfl(b0, (int)n1, 64), e1 = __shfl(b1, (int)n1, 64);
        const uint32_t lo = id < 64 ? s0 : s1, hi = id + 1 < 64 ? e0 : e1;
        if (id < NB) {
          const bool eqb = (id & 1u) != 0;
          const uint32_t sz = hi - lo;
          const bool big = !eqb && sz > C;
          const Seg piece{L.off + lo, sz, L.root,
                          make_meta(sbuf, eqb ? LEAF_COPY : (big ? LEAF_BIG : LEAF_REG), 0, 0, 0)};
          // every entry of the block that exists is written (an empty one
          // for a piece that is finished elsewhere)
          if (base + id < w.capLeaf)
            w.leaves[base + id] = (room && !big) ? piece
                                                 : Seg{L.off + lo, 0, L.root,
                                                       make_meta(sbuf, LEAF_COPY, 0, 0, 0)};
          if (room && big) {  // more than C keys: partitioned once more by k_big_rest
            const uint32_t r = atomicAdd(&w.ctr->nrest, 1u);
            if (r < 2 * w.capBig) w.bigLeaves[w.capBig + r] = piece; else raise_error(w.ctr, 1u);
          }
        }
      }
    }
  }
}

// The remainder of the oversized leaves, after the base case (its list is
// normally empty): buckets that one partition left larger than C, and
// oversized leaves whose pieces found no room in the leaf list.  Each is
// partitioned (once more); its buckets of at most C keys are sorted in LDS,
// its equality buckets copied, and a bucket still larger than C is sorted by
// the merge fallback.
template <int KT, bool PAY>
__global__ void __launch_bounds__(FIN_THREADS, PAY ? 2 : 4) k_big_rest(Ws w, uint32_t C,
                                                          uint32_t cutoff, uint64_t seed,
                                                          uint32_t flags) {
  const bool sampled_only = (flags & AMS_FLAG_SAMPLED_LEAF_SPLIT) != 0;
  typedef typename Key<KT>::T K;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  FinSmem<K> sm = fin_smem<K, PAY>(smem_raw, C);
  uint32_t nr = w.ctr->nrest;
  if (nr > 2 * w.capBig) nr = 2 * w.capBig;
  for (uint32_t li = blockIdx.x; li < nr; li += gridDim.x) {
    const Seg L = w.bigLeaves[w.capBig + li];
    const Root R = w.roots[L.root];
    const uint32_t buf = seg_buf(L.meta);
    if ((uint64_t)L.off + L.size > R.n || seg_kind(L.meta) != LEAF_BIG) {
      if (threadIdx.x == 0) raise_error(w.ctr, 32u);
      continue;
    }
    K *oK = (K *)R.kout + L.off;
    uint32_t *oV = PAY ? R.vout + L.off : nullptr;
    const uint32_t sbuf = buf == BUF_OUT ? BUF_TMP : BUF_OUT;
    uint32_t b0, b1;
    const uint32_t NB = big_partition<KT, PAY>(w, R, L, smem_raw, C, seed, sbuf, b0, b1);
    K *bK = kptr<K>(w, R, sbuf) + L.off;
    uint32_t *bV = PAY ? vptr(w, R, sbuf) + L.off : nullptr;
    for (uint32_t id = 0; id < NB; ++id) {
      const uint32_t lo = bucket_start(b0, b1, id), sz = bucket_start(b0, b1, id + 1) - lo;
      if (sz == 0) continue;
      if (id & 1u)
        copy_range<KT, PAY>(bK + lo, PAY ? bV + lo : nullptr, oK + lo, PAY ? oV + lo : nullptr, sz);
      else if (sz <= C)
        lds_sort<KT, PAY>(sm, bK + lo, PAY ? bV + lo : nullptr, false, oK + lo,
                          PAY ? oV + lo : nullptr, true, sz, C, cutoff,
                          stream_state(seed, LEAF_STREAM, L.root, L.off + lo), sampled_only);
      else
        merge_fallback<KT, PAY>(w, R, L.off + lo, sz, bK + lo, PAY ? bV + lo : nullptr, false, sm,
                                C, cutoff, seed, L.root, sampled_only);
    }
  }
}

// The base case over the leaf list (regular leaves, copies of final
// children and the pieces of oversized leaves), one workgroup per leaf.
template <int KT, bool PAY>
__global__ void __launch_bounds__(FIN_THREADS, PAY ? 2 : 4) k_finish(Ws w, uint32_t C, uint32_t cutoff,
                                                        uint64_t seed, uint32_t flags) {
  const bool sampled_only = (flags & AMS_FLAG_SAMPLED_LEAF_SPLIT) != 0;
  typedef typename Key<KT>::T K;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  FinSmem<K> sm = fin_smem<K, PAY>(smem_raw, C);
  const uint32_t tid = threadIdx.x;
  uint32_t nleaf = w.ctr->nleaf;
  if (nleaf > w.capLeaf) nleaf = w.capLeaf;
  // Leaves differ in size: after its first leaf a workgroup takes the next
  // unclaimed one from a counter, so the leaves still go out in list order
  // (neighbouring leaves side by side, as with a stride) but no workgroup
  // ends far behind the others.  The next index is requested as a leaf
  // starts and published by lds_sort once the leaf's keys are in.
  __shared__ uint32_t sNext;
  uint32_t li = blockIdx.x;
  while (li < nleaf) {
    const Seg L = w.leaves[li];
    uint32_t nx = 0;  // leaves handed out after the first gridDim.x, before this request
    if (tid == 0) nx = atomicInc(&w.ctr->finNext, 0xFFFFFFFFu);
    const Root R = w.roots[L.root];
    const uint32_t kind = seg_kind(L.meta), buf = seg_buf(L.meta);
    // defensive: never touch memory outside the root, nor more than C keys
    const bool bad =
        (uint64_t)L.off + L.size > R.n || (kind == LEAF_REG && L.size > C) || kind == LEAF_BIG;
    const K *src = kptr<K>(w, R, buf) + L.off;
    const uint32_t *vsrc = PAY ? vptr(w, R, buf) + L.off : nullptr;
    K *dst = (K *)R.kout + L.off;
    uint32_t *vdst = PAY ? R.vout + L.off : nullptr;
    if (bad || kind == LEAF_COPY) {
      if (bad && tid == 0) raise_error(w.ctr, 32u);
      if (!bad) copy_range<KT, PAY>(src, vsrc, dst, vdst, L.size);
      if (tid == 0) sNext = gridDim.x + nx;
    } else {
      lds_sort<KT, PAY>(sm, src, vsrc, buf == BUF_IN, dst, vdst, true, L.size, C, cutoff,
                        stream_state(seed, LEAF_STREAM, L.root, L.off), sampled_only, &sNext,
                        nx);
    }
    __syncthreads();
    li = sNext;
    __syncthreads();  // every thread has read sNext before thread 0 writes it again
  }
}

// ---------------------------------------------------------------------------
// Plain streaming copy: the practical HBM ceiling the level passes are
// measured against.  Each workgroup copies one contiguous chunk, eight
// 16-byte words per lane in flight (the fastest of the grid-stride and
// chunked layouts measured on this GPU).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_copy16(const v4u32 *src_, v4u32 *dst_, uint64_t n16,
                                                uint64_t per) {
  const GMem<v4u32> *src = (const GMem<v4u32> *)src_;
  GMem<v4u32> *dst = (GMem<v4u32> *)dst_;
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint64_t hi = lo + per < n16 ? lo + per : n16;
  uint64_t i = lo + threadIdx.x;
  for (; i + 7 * 256 < hi; i += 8 * 256) {
    v4u32 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) dst[i + u * 256] = v[u];
  }
  for (; i < hi; i += 256) dst[i] = src[i];
}

__global__ void k_copy_tail(const unsigned char *src, unsigned char *dst, uint64_t n) {
  for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

ams_status device_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------------------
// Workspace of the no-allocation entry point: a fixed array that every GPU
// the library runs on holds until the process ends.  Host code never uses
// its name as an address (that is a host-side stand-in); the device address
// comes from hipGetSymbolAddress, once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

const char *last_error() { return g_err; }

// ---------------------------------------------------------------------------
// Kernel tracing: when on, every launch of the calling thread is bracketed by
// a pair of events on the launch stream; ams_trace_stop sums them per kernel.
// ---------------------------------------------------------------------------
thread_local bool g_trace_on = false;
thread_local std::vector<TraceRec> *g_trace = nullptr;
static thread_local std::vector<ams_trace_entry> *g_trace_acc = nullptr;

TraceScope::TraceScope(const char *name, uint32_t level, hipStream_t st) : on(g_trace_on), s(st) {
  if (!on) return;
  if (level == 0xFFFFFFFFu) snprintf(rec.name, sizeof rec.name, "%s", name);
  else snprintf(rec.name, sizeof rec.name, "%s.L%u", name, level);
  (void)hipEventCreate(&rec.e0);
  (void)hipEventCreate(&rec.e1);
  (void)hipEventRecord(rec.e0, s);
}

TraceScope::~TraceScope() {
  if (!on) return;
  (void)hipEventRecord(rec.e1, s);
  g_trace->push_back(rec);
}

ams_status trace_start() {
  if (!g_trace) g_trace = new std::vector<TraceRec>();
  for (auto &r : *g_trace) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  g_trace->clear();
  if (g_trace_acc) g_trace_acc->clear();
  g_trace_on = true;
  return AMS_OK;
}

// Aggregates pending records (waiting for their events) into per-name totals,
// kept until the next trace_start; returns the number of names.
int trace_stop(ams_trace_entry *out, int max) {
  g_trace_on = false;
  if (!g_trace_acc) g_trace_acc = new std::vector<ams_trace_entry>();
  std::vector<ams_trace_entry> &acc = *g_trace_acc;
  if (g_trace) {
    for (auto &r : *g_trace) {
      (void)hipEventSynchronize(r.e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, r.e0, r.e1);
      ams_trace_entry *e = nullptr;
      for (auto &a : acc)
        if (!strcmp(a.name, r.name)) e = &a;
      if (!e) {
        ams_trace_entry z;
        memset(&z, 0, sizeof z);
        snprintf(z.name, sizeof z.name, "%s", r.name);
        acc.push_back(z);
        e = &acc.back();
      }
      e->launches += 1;
      e->total_ms += ms;
      if (ms > e->max_ms) e->max_ms = ms;
      (void)hipEventDestroy(r.e0);
      (void)hipEventDestroy(r.e1);
    }
    g_trace->clear();
  }
  if (out)
    for (int i = 0; i < (int)acc.size() && i < max; ++i) out[i] = acc[i];
  return (int)acc.size();
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// Device errors and run statistics
// ---------------------------------------------------------------------------
ams_status device_errors(hipStream_t s, uint32_t *bits, bool clear) {
  uint32_t v = 0;
  hipError_t e = hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_dev_errors), 4, 0,
                                          hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && clear && v) {
    const uint32_t zero = 0;
    e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_dev_errors), &zero, 4, 0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) {
    set_error("reading the device error word: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  if (bits) *bits = v;
  return AMS_OK;
}

size_t run_error_offset() { return offsetof(Ctr, overflow); }

__global__ void k_fold_errors(const uint32_t *word) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *word) atomicOr(&g_dev_errors, *word);
}

// ORs an error word that another kernel family keeps (RLM-sort's) into the
// device's error word, in stream order.
ams_status fold_device_errors(const uint32_t *d_word, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_errors, dim3(1), dim3(64), 0, s, d_word);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

// Device address of `scratch` on the current device, looked up on the first
// call per device (with that device current) and kept.
ams_status noalloc_scratch(void **ptr) {
  static std::mutex mu;
  static void *addr[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= (int)MAX_DEVICES) {
    set_error("no usable current device (%s)", hipGetErrorString(e));
    return AMS_EHIP;
  }
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return AMS_EHIP;
    }
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return AMS_OK;
}

ams_status device_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  if (n16) {
    // chunks of 16 KiB (1024 words), at most 2^20 workgroups
    uint64_t per = 1024;
    while ((n16 + per - 1) / per > (1u << 20)) per *= 2;
    const uint32_t grid = (uint32_t)((n16 + per - 1) / per);
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const v4u32 *)src, (v4u32 *)dst,
                       n16, per);
  }
  if (bytes % 16)
    hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, (const unsigned char *)src + n16 * 16,
                       (unsigned char *)dst + n16 * 16, (uint64_t)(bytes % 16));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

// Errors raised by the run whose counters sit at the start of ws (waits for s).
ams_status run_errors(const void *ws, hipStream_t s, uint32_t *bits) {
  uint32_t v = 0;
  hipError_t e = hipMemcpyAsync(&v, (const char *)ws + offsetof(Ctr, overflow), 4,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("reading the run's error word: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  *bits = v;
  return AMS_OK;
}

ams_status run_stats(const void *ws, hipStream_t s, ams_run_stats *out) {
  Ctr c;
  hipError_t e = hipMemcpyAsync(&c, ws, sizeof c, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("reading the run's counters: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  memset(out, 0, sizeof *out);
  out->device_errors = c.overflow;
  out->levels = c.L;
  for (uint32_t l = 0; l < MAXLEV && l < 4; ++l) {
    out->subproblems[l] = c.lv_sub[l];
    out->keys[l] = c.lv_keys[l];
    out->final_keys[l] = c.lv_final[l];
    out->max_child[l] = c.lv_maxchild[l];
    out->tiles[l] = c.lv_tiles[l];
    out->imbalance_max[l] = c.lv_imb_max[l] / 65536.0;
    out->imbalance_mean[l] = c.lv_sub[l] ? (double)c.lv_imb_sum[l] / 65536.0 / c.lv_sub[l] : 0.0;
  }
  out->leaves = c.nleaf;
  out->big_leaves = c.nbig;
  out->leaf_keys = c.leaf_keys[LEAF_REG];
  out->copy_keys = c.leaf_keys[LEAF_COPY];
  out->big_keys = c.leaf_keys[LEAF_BIG];
  out->merge_ranges = c.nmerge;
  out->merge_keys = c.merge_keys;
  return AMS_OK;
}

ams_status make_plan(Plan &pl, int kt, bool pay, const uint64_t *sizes, uint32_t nroots,
                     uint64_t n_single, const ams_params *p) {
  memset(&pl, 0, sizeof pl);
  if (kt != KT_U32 && kt != KT_U64 && kt != KT_F32) {
    set_error("unknown key type %d", kt);
    return AMS_EINVAL;
  }
  pl.kt = kt;
  pl.pay = pay;
  pl.kw = kt == KT_U64 ? 8 : 4;
  pl.nroots = nroots;
  uint64_t total = 0, mx = 0;
  for (uint32_t i = 0; i < nroots; ++i) {
    uint64_t n = sizes ? sizes[i] : n_single;
    if (n > AMS_MAX_SEGMENT) {
      set_error("segment of %llu elements: at most %llu are supported", (unsigned long long)n,
                (unsigned long long)AMS_MAX_SEGMENT);
      return AMS_EUNSUPPORTED;
    }
    total += n;
    mx = std::max(mx, n);
  }
  pl.ntotal = total;
  pl.maxroot = mx;
  // zero fields take the autotuner's choice for this shape class, if it has
  // made one, and the built-in defaults otherwise
  ams_params merged;
  {
    ams_params tuned;
    if (tuned_lookup(kt, pay, total, mx, nroots, &tuned)) {
      merged = p ? *p : tuned;
      if (p) {
        if (!merged.levels) merged.levels = tuned.levels;
        if (!merged.k) merged.k = tuned.k;
        if (!merged.overpartition_b) merged.overpartition_b = tuned.overpartition_b;
        if (!merged.base_cutoff) merged.base_cutoff = tuned.base_cutoff;
        if (!merged.tile_keys) merged.tile_keys = tuned.tile_keys;
      }
      p = &merged;
    }
  }
  uint32_t C = fin_capacity(pl.kw, pay);
  if (p && p->leaf_capacity) {
    // the base case needs room for its sample overlays (3 * FMAX keys); step
    // entry points that never run the base case may go lower
    const uint32_t lo = (p->flags & FLAG_NO_BASE_CASE) ? 64 : 1024;
    C = std::max<uint32_t>(lo, std::min<uint32_t>(p->leaf_capacity, C) & ~15u);
  }
  pl.C = C;
  uint64_t keysBig = 0;
  for (uint32_t i = 0; i < nroots; ++i) {
    uint64_t n = sizes ? sizes[i] : n_single;
    if (n > C) {
      ++pl.nbig;
      keysBig += n;
    }
  }
  pl.cutoff = (p && p->base_cutoff) ? std::min<uint32_t>(std::max<uint32_t>(p->base_cutoff, 2), 1024) : 32;
  pl.seed = (p && p->seed) ? p->seed : 14106754ull;
  pl.flags = p ? p->flags : 0;
  // defaults: r = 256, b = 4 for one sort; r = 128, b = 2 for a batch, where
  // subproblems are smaller and fewer buckets cost less per level
  const bool batch = nroots > 1;
  uint32_t r = (p && p->k) ? p->k : (batch ? 128 : 256);
  if (r < 2 || r > 1024 || (r & (r - 1))) {
    set_error("k must be a power of two in 2..1024 (got %u)", r);
    return AMS_EINVAL;
  }
  uint32_t b = (p && p->overpartition_b) ? p->overpartition_b : (batch ? 2 : 4);
  if (b < 1 || (b & (b - 1))) {
    set_error("overpartition_b must be a power of two (got %u)", b);
    return AMS_EINVAL;
  }
  if (r * b > 2048) b = std::max<uint32_t>(1, 2048 / r);
  // tiles of 64 Ki keys once there are at least 2048 of them (8 per CU):
  // fewer per-tile histograms and tile starts to reduce and scan
  uint32_t TC = (p && p->tile_keys) ? p->tile_keys : (keysBig >= (1ull << 27) ? 65536 : 32768);
  // (with segments of at most 2^32 - 2^20 keys, tile bounds up to 2^19 keys
  // stay below 2^32 in the kernels' 32-bit tile arithmetic)
  if (TC % 4096 || TC == 0 || TC > (1u << 19)) {
    set_error("tile_keys must be a positive multiple of 4096, at most 2^19 (got %u)", TC);
    return AMS_EINVAL;
  }
  const uint32_t Scap = 65536 / pl.kw;
  // levels: enough that an average group of the largest segment fills at
  // most 55% of the leaf capacity (the rest absorbs the imbalance of the
  // grouping at each level); for a batch, at most 120%: its few largest
  // segments then send some groups to the merge fallback, which costs less
  // than another level over all segments
  const double fill = batch ? 1.2 : 0.55;
  uint32_t L = 0;
  if (mx > C) {
    if (p && p->levels) {
      L = std::min<uint32_t>(p->levels, MAXLEV);
    } else {
      L = 1;
      double cap = (double)r;
      while (L < MAXLEV && (double)mx / cap > fill * C) {
        ++L;
        cap *= r;
      }
    }
  }
  pl.L = L;
  // below the first level, b = 2 when the leaves will be small (on average
  // at most 30% of the base case's capacity): half the buckets cost less in
  // every pass, and the less even groups still fit a leaf
  double capL = 1.0;
  for (uint32_t l = 0; l < L; ++l) capL *= r;
  const bool smallLeaves = (double)mx / capL <= 0.3 * C;
  uint64_t P = pl.nbig, keys = keysBig;
  uint64_t leaves = nroots + 64;
  for (uint32_t l = 0; l < L; ++l) {
    LevelShape &ls = pl.lev[l];
    ls.rmax = r;
    ls.b = (l > 0 && smallLeaves && !(p && p->overpartition_b)) ? std::min<uint32_t>(b, 2) : b;
    // samples per bucket: 8 for the split of the whole input; 2 below,
    // where a subproblem's sample costs more than its slightly less even
    // buckets (the grouping absorbs them)
    ls.a = (p && p->samples_per_bucket) ? p->samples_per_bucket : (l == 0 ? 8 : 2);
    ls.mmax = std::min<uint32_t>(2048, r * ls.b);
    ls.Smax = (uint32_t)std::min<uint64_t>(Scap, align256((uint64_t)ls.a * ls.mmax));
    if (ls.Smax < 256) ls.Smax = 256;
    ls.TC = TC;
    ls.TB = 64;
    ls.HS = 2 * ls.mmax;
    ls.CH = 3 * r;
    ls.P = (uint32_t)std::max<uint64_t>(P, 1);
    ls.tiles = (uint32_t)(keys / TC + P + 2);
    ls.blocks = ls.tiles / ls.TB + (uint32_t)P + 2;
    ls.sblocks = (uint32_t)(P * (ls.Smax / 256) + 1);
    uint32_t nb = ls.Smax / 256;
    uint64_t want = (P * nb + 1023) / 1024;
    ls.rankG = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(nb, want));
    leaves += P * ls.CH + keys / C + 2;
    uint64_t nextP = std::min<uint64_t>(P * ls.CH, keys / (C + 1));
    P = nextP;
  }
  // leaves, plus room for the pieces of oversized leaves (2 * BIG_FMAX - 1
  // per partition; more pieces than that are finished by their partitioner)
  pl.capLeaf = (uint32_t)std::min<uint64_t>(leaves + total / C + 2 + 2 * BIG_FMAX * 1024ull,
                                            0xFFFFFFF0ull);
  // test hook: a leaf table of one entry, so that a sort needing more leaves
  // takes the device's table-overflow path (raises AMS_DEVERR_TABLE)
  // an oversized leaf holds more than C keys
  pl.capBig = (uint32_t)std::min<uint64_t>(total / (C + 1) + nroots + 2, 0xFFFFFFF0ull);
  if (pl.flags & AMS_FLAG_TEST_TINY_TABLES) pl.capLeaf = 1;
  uint32_t capAct = 1, capTile = 1, capBlk = 1, capS = 1, maxHS = 2, maxCH = 3, maxM = 2, maxS = 256;
  for (uint32_t l = 0; l < L; ++l) {
    const LevelShape &ls = pl.lev[l];
    capAct = std::max(capAct, ls.P);
    capTile = std::max(capTile, ls.tiles);
    capBlk = std::max(capBlk, ls.blocks);
    capS = std::max(capS, ls.sblocks);
    maxHS = std::max(maxHS, ls.HS);
    maxCH = std::max(maxCH, ls.CH);
    maxM = std::max(maxM, ls.mmax);
    maxS = std::max(maxS, ls.Smax);
  }
  pl.capActMax = capAct;
  pl.capTile = capTile;
  pl.capBlk = capBlk;
  pl.capSBlk = capS;
  pl.maxHS = maxHS;
  pl.maxCH = maxCH;
  pl.maxM = maxM;
  pl.maxS = maxS;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  // the run's counters come first, so ams_workspace_stats finds them at the
  // start of any workspace
  pl.o_ctr = take(sizeof(Ctr));
  pl.o_tmpK = take(L ? total * pl.kw : 0);
  pl.o_tmpV = take(L && pay ? total * 4 : 0);
  pl.o_roots = take((size_t)nroots * sizeof(Root));
  for (uint32_t l = 0; l <= MAXLEV; ++l)
    pl.o_act[l] = take(l < L ? (size_t)pl.lev[l].P * sizeof(Seg) : 0);
  pl.o_leaves = take((size_t)pl.capLeaf * sizeof(Seg));
  pl.o_big = take((size_t)pl.capBig * 3 * sizeof(Seg));  // oversized leaves, then the remainder
  const bool any = L > 0;
  // per-subproblem and per-tile tables: the kernels index them with the
  // level's own strides, so each holds the largest level's rows
  size_t eSamp = 0, eM = 0, eHist = 0, eBlk = 0, eTot = 0, eOff = 0, eCF = 0, eCS = 0, eCD = 0;
  for (uint32_t l = 0; l < L; ++l) {
    const LevelShape &ls = pl.lev[l];
    eSamp = std::max(eSamp, (size_t)ls.P * ls.Smax);
    eM = std::max(eM, (size_t)ls.P * ls.mmax);
    eHist = std::max(eHist, (size_t)ls.tiles * ls.HS);
    eBlk = std::max(eBlk, (size_t)ls.blocks * ls.HS);
    eTot = std::max(eTot, (size_t)ls.P * ls.HS);
    eOff = std::max(eOff, (size_t)ls.tiles * ls.CH);
    eCF = std::max(eCF, (size_t)ls.P * 2 * (ls.CH + 1));
    eCS = std::max(eCS, (size_t)ls.P * (ls.CH + 1));
    eCD = std::max(eCD, (size_t)ls.P * ls.CH);
  }
  pl.o_tileStart = take(any ? (size_t)(capAct + 1) * 4 : 0);
  pl.o_blkStart = take(any ? (size_t)(capAct + 1) * 4 : 0);
  pl.o_sampStart = take(any ? (size_t)(capAct + 1) * 4 : 0);
  pl.o_samp = take(eSamp * pl.kw);
  pl.o_spl = take(eM * pl.kw);
  pl.o_tree = take(eM * pl.kw);
  pl.o_eq = take(any ? capAct : 0);
  pl.o_hist = take(eHist * 4);
  pl.o_blkHist = take(eBlk * 4);
  pl.o_totals = take(eTot * 4);
  pl.o_tileOff = take(eOff * 4);
  pl.o_i2c = take(eTot * 2);
  pl.o_cfirst = take(eCF * 2);
  pl.o_cstart = take(eCS * 4);
  pl.o_cdst = take(eCD);
  pl.o_nch = take(any ? (size_t)capAct * 4 : 0);
  {
    size_t ns = 0;  // strata of the subproblems of every level below the first
    if (pl.flags & AMS_FLAG_STRATIFIED)
      for (uint32_t l = 1; l < L; ++l) ns = std::max(ns, (size_t)pl.lev[l].P);
    pl.o_strata = take(ns * sizeof(Strata));
  }
  pl.o_dbg = take((size_t)(nroots + 1) * 8);  // batch offsets upload / step outputs
  pl.o_sink = take(SINK_WORDS * 8);
  pl.bytes = o;
  return AMS_OK;
}

static Ws carve(const Plan &pl, char *base) {
  Ws w;
  memset(&w, 0, sizeof w);
  w.roots = (Root *)(base + pl.o_roots);
  w.nroots = pl.nroots;
  w.tmpK = base + pl.o_tmpK;
  w.tmpV = (uint32_t *)(base + pl.o_tmpV);
  w.ctr = (Ctr *)(base + pl.o_ctr);
  for (uint32_t l = 0; l <= MAXLEV; ++l) {
    w.act[l] = (Seg *)(base + pl.o_act[l]);
    w.capAct[l] = l < pl.L ? pl.lev[l].P : 0;
  }
  w.leaves = (Seg *)(base + pl.o_leaves);
  w.capLeaf = pl.capLeaf;
  w.bigLeaves = (Seg *)(base + pl.o_big);
  w.capBig = pl.capBig;
  w.tileStart = (uint32_t *)(base + pl.o_tileStart);
  w.blkStart = (uint32_t *)(base + pl.o_blkStart);
  w.sampStart = (uint32_t *)(base + pl.o_sampStart);
  w.samp = base + pl.o_samp;
  w.spl = base + pl.o_spl;
  w.tree = base + pl.o_tree;
  w.eqOn = (uint8_t *)(base + pl.o_eq);
  w.hist = (uint32_t *)(base + pl.o_hist);
  w.blkHist = (uint32_t *)(base + pl.o_blkHist);
  w.totals = (uint32_t *)(base + pl.o_totals);
  w.tileOff = (uint32_t *)(base + pl.o_tileOff);
  w.i2c = (uint16_t *)(base + pl.o_i2c);
  w.cfirst = (uint16_t *)(base + pl.o_cfirst);
  w.cstart = (uint32_t *)(base + pl.o_cstart);
  w.cdst = (uint8_t *)(base + pl.o_cdst);
  w.nch = (uint32_t *)(base + pl.o_nch);
  w.strata = (Strata *)(base + pl.o_strata);
  w.sink = (uint64_t *)(base + pl.o_sink);
  w.capTile = pl.capTile;
  w.capBlk = pl.capBlk;
  w.capSBlk = pl.capSBlk;
  return w;
}

static LevTable lev_table(const Plan &pl, bool shrink_last) {
  LevTable lt;
  memset(&lt, 0, sizeof lt);
  for (uint32_t l = 0; l < pl.L; ++l) {
    const LevelShape &ls = pl.lev[l];
    Lev &v = lt.l[l];
    v.level = l;
    v.L = pl.L;
    v.last = l + 1 == pl.L;
    v.shrink = shrink_last && v.last;
    v.rmax = ls.rmax;
    v.b = ls.b;
    v.a = ls.a;
    v.mmax = ls.mmax;
    v.Smax = ls.Smax;
    v.TC = ls.TC;
    v.TB = ls.TB;
    v.HS = ls.HS;
    v.CH = ls.CH;
    v.rankG = ls.rankG;
    v.C = pl.C;
    v.flags = pl.flags;
    v.Scap = 65536 / pl.kw;
    v.capTile = ls.tiles;
    v.capBlk = ls.blocks;
    v.capSBlk = ls.sblocks;
    v.seed = pl.seed;
    v.kw = pl.kw;
    const bool strat = (pl.flags & AMS_FLAG_STRATIFIED) != 0;
    v.strata = strat && l >= 1;
    v.strataNext = strat && l + 1 < pl.L;
  }
  return lt;
}

static uint32_t grid_for(uint64_t items, uint32_t cap) {
  if (items < 1) items = 1;
  uint64_t g = std::min<uint64_t>(items, cap);
  if (g >= 8) g &= ~7ull;
  return (uint32_t)g;
}

template <typename F> static void allow_lds(F *kernel, size_t bytes) {
  static thread_local bool done = false;
  (void)done;
  (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)std::min<size_t>(bytes, 163840));
}

template <int KT, bool PAY>
static ams_status run_typed(const Plan &pl, void *wsv, const RootSource &rs, hipStream_t s,
                            uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                            const void *given, bool shrink_last) {
  typedef typename Key<KT>::T K;
  char *base = (char *)wsv;
  Ws w = carve(pl, base);
  w.dbgHist = dbg_hist;
  w.dbgChildren = dbg_children;
  w.dbgNChild = dbg_nchild;
  LevTable lt = lev_table(pl, shrink_last);
  { TraceScope ts("reset", 0xFFFFFFFFu, s); hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w); }
  uint32_t gi = (uint32_t)std::min<uint64_t>((pl.nroots + 255) / 256, 1024);
  {
    TraceScope ts("init", 0xFFFFFFFFu, s);
    hipLaunchKernelGGL(k_init_roots, dim3(std::max(gi, 1u)), dim3(256), 0, s, w, lt, pl.L, pl.C,
                       rs.mode, rs.single, rs.kin, rs.vin, rs.kout, rs.vout, rs.d_offsets, pl.kw);
  }
  for (uint32_t l = 0; l < pl.L; ++l) {
    const LevelShape &ls = pl.lev[l];
    const Lev &lv = lt.l[l];
    {
      TraceScope ts("plan", l, s);
      hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, w, lv);
    }
    if (given && l == 0) {
      hipLaunchKernelGGL(k_set_splitters<KT>, dim3(1), dim3(256), 0, s, w, lv, given);
    } else {
      {
        TraceScope ts("sample_blocks", l, s);
        hipLaunchKernelGGL(k_sample_blocks<KT>, dim3(grid_for(ls.sblocks, 2048)), dim3(256), 0,
                           s, w, lv);
      }
      if (lv.strata) {
        size_t lds = 2 * (size_t)ls.Smax * sizeof(K);
        allow_lds(k_sample_strata<KT>, lds);
        TraceScope ts("sample_rank", l, s);
        hipLaunchKernelGGL(k_sample_strata<KT>, dim3(grid_for(ls.P, 1024)), dim3(256), lds, s, w,
                           lv);
      } else {
        size_t lds = (size_t)ls.Smax * sizeof(K);
        allow_lds(k_sample_rank<KT>, lds);
        uint32_t ng = (ls.Smax / 256 + ls.rankG - 1) / ls.rankG;
        TraceScope ts("sample_rank", l, s);
        hipLaunchKernelGGL(k_sample_rank<KT>, dim3(grid_for((uint64_t)ls.P * ng, 1024)),
                           dim3(256), lds, s, w, lv);
      }
    }
    size_t ldsC = (size_t)ls.mmax * sizeof(K) + (size_t)ls.HS * 4;
    allow_lds(k_count<KT>, ldsC);
    {
      TraceScope ts("count", l, s);
      // one workgroup per tile (ls.tiles bounds the level's tile count)
      hipLaunchKernelGGL(k_count<KT>, dim3(8 * ((ls.tiles + 7) / 8)), dim3(256), ldsC, s, w, lv);
    }
    {
      TraceScope ts("block_reduce", l, s);
      hipLaunchKernelGGL(k_block_reduce, dim3(grid_for((uint64_t)ls.blocks * ((ls.HS + 255) / 256), 2048)),
                         dim3(256), 0, s, w, lv);
    }
    {
      TraceScope ts("block_scan", l, s);
      hipLaunchKernelGGL(k_block_scan, dim3(grid_for((uint64_t)ls.P * ((ls.HS + 255) / 256), 1024)),
                         dim3(256), 0, s, w, lv);
    }
    size_t po[14];
    size_t ldsP = pack_layout(ls.HS, ls.CH, po);
    allow_lds(k_pack, ldsP);
    {
      TraceScope ts("pack", l, s);
      hipLaunchKernelGGL(k_pack, dim3(grid_for(ls.P, 1024)), dim3(256), ldsP, s, w, lv, lt);
    }
    {
      TraceScope ts("tile_scan", l, s);
      hipLaunchKernelGGL(k_tile_scan, dim3(grid_for((uint64_t)ls.blocks * ((ls.CH + 255) / 256), 2048)),
                         dim3(256), 0, s, w, lv);
    }
    if (!PAY && (pl.flags & AMS_FLAG_STABLE_PARTITION)) {
      constexpr int KPT = 16;
      constexpr uint32_t CHK = 256 * KPT;
      size_t ldsS = (size_t)ls.mmax * sizeof(K) + CHK * sizeof(K) + CHK * 2 + (size_t)ls.HS * 2 +
                    (size_t)ls.CH * 4 * 3 + 4 + (size_t)ls.CH * 16 + 256 * 4 + ls.CH + 64;
      allow_lds(k_scatter<KT, false, KPT>, ldsS);
      TraceScope ts("scatter", l, s);
      hipLaunchKernelGGL((k_scatter<KT, false, KPT>), dim3(grid_for(ls.tiles, 512)), dim3(256),
                         ldsS, s, w, lv);
    } else if (PAY) {
      // 8192-pair chunks when one thread per child and the LDS allow it
      const size_t ldsP = (size_t)ls.mmax * sizeof(K) +
                          (size_t)SCK_THREADS * SCP_KPT * (sizeof(K) + 4 + 2) +
                          (size_t)(SCK_THREADS / 64) * ((ls.CH + 3) & ~3u) * 2 +
                          (size_t)((ls.HS + 1) & ~1u) * 2 + (size_t)ls.CH * 4 * 3 +
                          SCK_THREADS / 64 * 4 + ls.CH + 64;
      TraceScope ts("scatter", l, s);
      if (ls.CH <= SCK_THREADS && ldsP <= 163840) {
        allow_lds(k_scatter_pairs<KT>, ldsP);
        hipLaunchKernelGGL(k_scatter_pairs<KT>, dim3(grid_for(ls.tiles, 512)), dim3(SCK_THREADS),
                           ldsP, s, w, lv);
      } else {
        constexpr int KPT = 8;
        constexpr uint32_t CHK = 256 * KPT;
        size_t ldsS = (size_t)ls.mmax * sizeof(K) + CHK * sizeof(K) + CHK * 4 + CHK * 2 +
                      (size_t)ls.HS * 2 + (size_t)ls.CH * 4 * 3 + 4 + (size_t)ls.CH * 16 +
                      256 * 4 + ls.CH + 64;
        allow_lds(k_scatter<KT, true, KPT>, ldsS);
        hipLaunchKernelGGL((k_scatter<KT, true, KPT>), dim3(grid_for(ls.tiles, 512)), dim3(256),
                           ldsS, s, w, lv);
      }
    } else {
      // chunks of 8192 keys, or 4096 when the tables of a wide level
      // (large k * b) leave too little LDS for the larger staging area
      auto lds_keys = [&](uint32_t kpt) {
        const size_t chk = (size_t)SCK_THREADS * kpt;
        return (size_t)ls.mmax * sizeof(K) + chk * sizeof(K) + (size_t)(ls.CH + 2) * 8 + chk * 2 +
               (size_t)ls.HS * 2 + (size_t)ls.CH * 4 * 3 + SCK_THREADS / 64 * 4 + ls.CH + 64;
      };
      // with at most SCK_PCH children: per-wavefront scans and two counter
      // banks in place of the block scan's offsets and counters
      const size_t ldsPriv = lds_keys(8) - (size_t)ls.CH * 8 + (size_t)2 * SCK_PCH * 4 +
                             (size_t)(SCK_THREADS / 64) * SCK_PCH * 2;
      TraceScope ts("scatter", l, s);
      // (the counter banks are read 16 bytes at a time: the tree area before
      // them must keep that alignment)
      if (ls.CH <= SCK_PCH && ldsPriv <= 163840 && (ls.mmax * sizeof(K)) % 16 == 0) {
        allow_lds(k_scatter_keys<KT, 8, true>, ldsPriv);
        hipLaunchKernelGGL((k_scatter_keys<KT, 8, true>), dim3(grid_for(ls.tiles, 512)),
                           dim3(SCK_THREADS), ldsPriv, s, w, lv);
      } else if (lds_keys(8) <= 163840) {
        allow_lds(k_scatter_keys<KT, 8, false>, lds_keys(8));
        hipLaunchKernelGGL((k_scatter_keys<KT, 8, false>), dim3(grid_for(ls.tiles, 512)),
                           dim3(SCK_THREADS), lds_keys(8), s, w, lv);
      } else {
        allow_lds(k_scatter_keys<KT, 4, false>, lds_keys(4));
        hipLaunchKernelGGL((k_scatter_keys<KT, 4, false>), dim3(grid_for(ls.tiles, 512)),
                           dim3(SCK_THREADS), lds_keys(4), s, w, lv);
      }
    }
  }
  if (!dbg_hist) {
    const size_t ldsF = fin_smem_bytes<K, PAY>(pl.C);
    if (pl.L > 0) {
      allow_lds(k_big_part<KT, PAY>, big_smem_bytes<K>());
      TraceScope ts("big_part", 0xFFFFFFFFu, s);
      hipLaunchKernelGGL((k_big_part<KT, PAY>), dim3(grid_for(pl.capBig, 1024)), dim3(FIN_THREADS),
                         big_smem_bytes<K>(), s, w, pl.C, pl.seed, pl.flags);
    }
    allow_lds(k_finish<KT, PAY>, ldsF);
    {
      TraceScope ts("finish", 0xFFFFFFFFu, s);
      hipLaunchKernelGGL((k_finish<KT, PAY>), dim3(grid_for(pl.capLeaf, PAY ? 256 : 512)),
                         dim3(FIN_THREADS), ldsF, s, w, pl.C, pl.cutoff, pl.seed, pl.flags);
    }
    if (pl.L > 0) {
      const size_t ldsR = std::max(ldsF, big_smem_bytes<K>());
      allow_lds(k_big_rest<KT, PAY>, ldsR);
      TraceScope ts("big_rest", 0xFFFFFFFFu, s);
      hipLaunchKernelGGL((k_big_rest<KT, PAY>), dim3(grid_for(pl.capBig, PAY ? 256 : 512)),
                         dim3(FIN_THREADS), ldsR, s, w, pl.C, pl.cutoff, pl.seed, pl.flags);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

ams_status run_plan_ex(const Plan &pl, void *ws, const RootSource &src, hipStream_t s,
                       uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                       const void *given_splitters, bool shrink_last) {
#define AMS_RUN(KT_, PAY_)                                                                      \
  return run_typed<KT_, PAY_>(pl, ws, src, s, dbg_hist, dbg_children, dbg_nchild,              \
                              given_splitters, shrink_last)
  if (pl.kt == KT_U32) { if (pl.pay) AMS_RUN(KT_U32, true); AMS_RUN(KT_U32, false); }
  if (pl.kt == KT_U64) { if (pl.pay) AMS_RUN(KT_U64, true); AMS_RUN(KT_U64, false); }
  if (pl.pay) AMS_RUN(KT_F32, true);
  AMS_RUN(KT_F32, false);
#undef AMS_RUN
}

ams_status run_plan(const Plan &pl, void *ws, const RootSource &src, hipStream_t s,
                    uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                    const void *given_splitters) {
  return run_plan_ex(pl, ws, src, s, dbg_hist, dbg_children, dbg_nchild, given_splitters, true);
}

// ---------------------------------------------------------------------------
// Tile sort: consecutive tiles of T keys of one array (the last one ragged),
// each sorted in LDS by the base case, written decoded to `out` (which may
// be `in`: a tile is read whole before it is written).  RLM-sort's local
// sort ("every PE sorts locally first", Section 5).
// ---------------------------------------------------------------------------
__global__ void k_tile_leaves(Ws w, uint64_t n, uint32_t T) {
  const uint32_t nt = (uint32_t)((n + T - 1) / T);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt && i < w.capLeaf;
       i += gridDim.x * blockDim.x) {
    const uint64_t off = (uint64_t)i * T;
    const uint32_t sz = (uint32_t)(n - off < T ? n - off : T);
    w.leaves[i] = Seg{(uint32_t)off, sz, 0, make_meta(BUF_IN, LEAF_REG, 0, 0, 0)};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctr->nleaf = nt < w.capLeaf ? nt : w.capLeaf;
}

uint32_t base_case_capacity(uint32_t kw, bool pay) { return fin_capacity(kw, pay); }

size_t tile_sort_ws_bytes(uint64_t n, uint32_t T) {
  const uint64_t nt = (n + T - 1) / T;
  return align256(sizeof(Ctr)) + align256(sizeof(Root)) + align256(nt * sizeof(Seg));
}

template <int KT, bool PAY>
static ams_status tile_sort_typed(const void *in, const uint32_t *vin, void *out, uint32_t *vout,
                                  uint64_t n, uint32_t T, void *wsv, hipStream_t s) {
  typedef typename Key<KT>::T K;
  const uint32_t C = fin_capacity(sizeof(K), PAY);
  if (T > C || T == 0) {
    set_error("tile of %u keys exceeds the base case's %u", T, C);
    return AMS_EINVAL;
  }
  char *base = (char *)wsv;
  Ws w;
  memset(&w, 0, sizeof w);
  w.ctr = (Ctr *)base;
  w.roots = (Root *)(base + align256(sizeof(Ctr)));
  w.leaves = (Seg *)(base + align256(sizeof(Ctr)) + align256(sizeof(Root)));
  w.nroots = 1;
  const uint64_t nt = (n + T - 1) / T;
  w.capLeaf = (uint32_t)nt;
  Root R;
  R.kin = in;
  R.vin = vin;
  R.kout = out;
  R.vout = vout;
  R.n = n;
  R.tmp_off = 0;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w);
  hipError_t e = hipMemcpyAsync(w.roots, &R, sizeof R, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    set_error("root upload: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  hipLaunchKernelGGL(k_tile_leaves, dim3((uint32_t)std::min<uint64_t>((nt + 255) / 256, 1024)),
                     dim3(256), 0, s, w, n, T);
  size_t ldsF = fin_smem_bytes<K, PAY>(C);
  allow_lds(k_finish<KT, PAY>, ldsF);
  {
    TraceScope ts("tile_sort", 0xFFFFFFFFu, s);
    hipLaunchKernelGGL((k_finish<KT, PAY>), dim3(grid_for(nt, PAY ? 256 : 512)),
                       dim3(FIN_THREADS), ldsF, s, w, C, 32u, 14106754ull, 0u);
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

ams_status run_tile_sort(int kt, bool pay, const void *in, const uint32_t *vin, void *out,
                         uint32_t *vout, uint64_t n, uint32_t T, void *ws, hipStream_t s) {
  if (kt == KT_U64) return pay ? tile_sort_typed<KT_U64, true>(in, vin, out, vout, n, T, ws, s)
                               : tile_sort_typed<KT_U64, false>(in, vin, out, vout, n, T, ws, s);
  if (kt == KT_U32) return pay ? tile_sort_typed<KT_U32, true>(in, vin, out, vout, n, T, ws, s)
                               : tile_sort_typed<KT_U32, false>(in, vin, out, vout, n, T, ws, s);
  return pay ? tile_sort_typed<KT_F32, true>(in, vin, out, vout, n, T, ws, s)
             : tile_sort_typed<KT_F32, false>(in, vin, out, vout, n, T, ws, s);
}

// Step entry point helpers -------------------------------------------------
ams_status run_pack_only(const uint32_t *d_w, uint32_t nb, uint32_t r, uint32_t *d_out,
                         hipStream_t s) {
  size_t lds = (size_t)((nb + 7) & ~7u) * 4 + 64;
  allow_lds(k_pack_only, lds);
  hipLaunchKernelGGL(k_pack_only, dim3(1), dim3(256), lds, s, d_w, nb, r, d_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

// Copy the sorted splitters of the first active subproblem of level 0.
ams_status copy_splitters(const Plan &pl, void *ws, void *d_out, uint32_t m, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d_out, (char *)ws + pl.o_spl, (size_t)(m - 1) * pl.kw,
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

ams_status run_sample_only(const Plan &pl, void *wsv, const RootSource &rs, hipStream_t s) {
  // levels up to the splitters of level 0 only
  Plan p2 = pl;
  (void)p2;
  char *base = (char *)wsv;
  Ws w = carve(pl, base);
  LevTable lt = lev_table(pl, false);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w);
  hipLaunchKernelGGL(k_init_roots, dim3(1), dim3(256), 0, s, w, lt, pl.L, pl.C, rs.mode,
                     rs.single, rs.kin, rs.vin, rs.kout, rs.vout, rs.d_offsets, pl.kw);
  const LevelShape &ls = pl.lev[0];
  const Lev &lv = lt.l[0];
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, w, lv);
  uint32_t ng = (ls.Smax / 256 + ls.rankG - 1) / ls.rankG;
  if (pl.kt == KT_U64) {
    hipLaunchKernelGGL(k_sample_blocks<KT_U64>, dim3(grid_for(ls.sblocks, 2048)), dim3(256), 0,
                       s, w, lv);
    size_t lds = (size_t)ls.Smax * 8;
    allow_lds(k_sample_rank<KT_U64>, lds);
    hipLaunchKernelGGL(k_sample_rank<KT_U64>, dim3(grid_for(ng, 1024)), dim3(256), lds, s, w, lv);
  } else if (pl.kt == KT_U32) {
    hipLaunchKernelGGL(k_sample_blocks<KT_U32>, dim3(grid_for(ls.sblocks, 2048)), dim3(256), 0,
                       s, w, lv);
    size_t lds = (size_t)ls.Smax * 4;
    allow_lds(k_sample_rank<KT_U32>, lds);
    hipLaunchKernelGGL(k_sample_rank<KT_U32>, dim3(grid_for(ng, 1024)), dim3(256), lds, s, w, lv);
  } else {
    hipLaunchKernelGGL(k_sample_blocks<KT_F32>, dim3(grid_for(ls.sblocks, 2048)), dim3(256), 0,
                       s, w, lv);
    size_t lds = (size_t)ls.Smax * 4;
    allow_lds(k_sample_rank<KT_F32>, lds);
    hipLaunchKernelGGL(k_sample_rank<KT_F32>, dim3(grid_for(ng, 1024)), dim3(256), lds, s, w, lv);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return AMS_OK;
}

}  // namespace ams
