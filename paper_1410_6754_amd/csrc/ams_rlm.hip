// RLM-sort (recurse-last multiway mergesort, Section 5) on gfx950.
//
// One GPU plays the whole machine: a tile of T keys plays a PE's local data.
//   tile sort       every tile sorted in LDS by the base case (every PE
//                   sorts locally first)
// then, level by level, over every group of sorted sequences at once:
//   k_rlm_children  each group's parts: r parts of equal size (part j holds
//                   ranks [floor(jN/r), floor((j+1)N/r))), or, once parts of
//                   r tiles would be too small, just enough parts of at most
//                   T keys; their positions and table bases
//   k_rlm_select    multisequence selection (Section 4.1) of every part
//                   boundary of the level side by side: a random pivot from
//                   the remaining windows, a binary search in every
//                   sequence, the side that holds the rank kept
//   k_rlm_cut       the cut of every sequence at every boundary
//   k_rlm_pieces    per part, the prefix sums of its piece sizes over the
//                   sequences (where each piece lands)
//   k_rlm_merge     per slice of T keys of a part (a PE of the group): its
//                   pieces gathered into LDS and merged pairwise by merge
//                   paths into one sorted sequence of the next level, or
//                   into the output at the last level
// Every level moves the keys once; the groups of a level are the parts of
// the level before, so a part's keys never leave its final rank range.
#include <string.h>

#include <algorithm>
#include <vector>

#include "ams_engine.h"

namespace ams {

ams_status fold_device_errors(const uint32_t *d_word, hipStream_t s);

namespace {

constexpr uint32_t RLM_NT = 256;        // selection threads (one sequence each)
constexpr uint32_t RLM_M = 8;           // pivots per selection step
constexpr uint32_t RLM_NONE = 0xFFu;    // "keep this end of the windows"
constexpr uint32_t RLM_GROUP_SEQ = RLM_NT;  // groups of at most this many sequences: whole selections per workgroup
constexpr uint32_t RLM_MT = 512;        // merge threads
constexpr uint32_t RLM_TMAX = 4096;     // largest tile (LDS of the merge)
constexpr uint32_t RLM_MAXLEV = 16;
constexpr uint32_t RLM_STREAM = 0xE0u;  // sampling-stream tag of the pivots

// A group of one level (and a part = a group of the next level).
struct RGroup {
  uint32_t start, size;  // keys [start, start + size) of the level's buffer
  uint32_t parent, j;    // parent group and part index in it (level >= 1)
  uint32_t rank;         // rank of the part's first key inside its parent
  uint32_t last;         // 1: the parent's last part
  uint32_t cutBase;      // row of S_parent entries in LO / HI / CC / CUT
  uint32_t blkBase;      // first selection block
  uint32_t qBase;        // S_parent + 1 piece offsets
  uint32_t sliceBase;    // first slice of the part in this level's merge
  uint32_t pad[2];
};

// One selection: the boundary in front of a part (j >= 1).  Each step
// draws up to RLM_M pivots from the remaining windows; the next step keeps
// the windows between the two pivots whose ranks bracket the sought one.
struct RSel {
  uint64_t pv[RLM_M];            // pivots' ord values
  uint32_t pq[RLM_M], pt[RLM_M]; // their sequences and positions
  uint32_t np;                   // pivots of the current step
  uint32_t krem;                 // rank still sought inside the windows (1-based)
  uint32_t total;                // keys in the windows
  uint32_t mlo, mhi;             // decision to apply: windows [cc[mlo], cc[mhi]) (RLM_NONE: keep)
  uint32_t done;                 // 1: the windows' upper ends (after the decision) are the cut
  uint32_t iter;
};

struct RHdr {
  uint32_t overflow;  // AMS_DEVERR_* bits
  uint32_t nGroups;   // groups of the current level
  uint32_t nChildren; // groups of the next level
  uint32_t cnt[4];    // totals of the child tables: cut entries, blocks, piece offsets, slices
  uint32_t pad[9];
};

struct RLev {
  uint32_t T, r, level;
  uint32_t force;      // nonzero: every group is split into this many parts (step entry)
  uint32_t last;       // the merge writes the output
  uint32_t itmax;      // steps a single-block selection may take
  uint32_t capChildren, capCut, capBlk, capQ, capSlice;
  uint64_t seed;
};

struct RWs {
  RHdr *hdr;
  RGroup *groups, *children;
  RSel *sel;
  uint32_t *lo, *hi, *cut, *q;
  uint32_t *cc;        // RLM_M rows of capCut: window keys before each pivot
  uint32_t *bl;        // per selection block: RLM_M + 1 partial sums
  uint32_t *blkOwner;  // selection block -> part
  uint32_t *sliceOwner;  // merge slice -> part
  uint32_t *sliceI0, *sliceI1;  // merge slice -> its first piece, one past its last
  uint32_t capCut;
  uint32_t *scratch;   // per group: five counts (exscan space), 5 (G + 1) entries
};

AMS_DEV void rlm_error(const RWs &w, uint32_t bits) { atomicOr(&w.hdr->overflow, bits); }

// A selection's control words as another block of this launch may have left
// them (the pivots are read the same way, word by word).
AMS_DEV uint32_t vload(const uint32_t *p) { return *(const volatile uint32_t *)p; }
AMS_DEV uint64_t vload64(const uint64_t *p) { return *(const volatile uint64_t *)p; }

AMS_DEV uint32_t seq_len(const RGroup &g, uint32_t i, uint32_t T) {
  const uint32_t a = i * T;
  return g.size - a < T ? g.size - a : T;
}

AMS_DEV uint32_t level_parts(uint32_t N, uint32_t r, uint32_t T) {
  if ((uint64_t)N > (uint64_t)r * T) return r;
  return N == 0 ? 1u : (N + T - 1) / T;
}

// ---------------------------------------------------------------------------
// Parts of every group: one workgroup of 1024 threads (a level has at most a
// few ten thousand groups).  The parts of a group share its sequence count
// S, so their cut, block and piece-offset tables have equal sizes: five
// exclusive scans over the groups (parts, and the four table sizes) place
// every part's tables; only the slices differ from part to part.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_rlm_children(RWs w, RLev lv) {
  __shared__ uint32_t tmp[1024 / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t G = w.hdr->nGroups;
  // per group (G + 1 entries each): parts, cut entries, selection blocks,
  // piece offsets, slices
  uint32_t *pc = w.scratch, *pcut = pc + (G + 1), *pblk = pcut + (G + 1);
  uint32_t *pq = pblk + (G + 1), *psl = pq + (G + 1);
  for (uint32_t g = tid; g < G; g += 1024) {
    const uint32_t N = w.groups[g].size;
    const uint32_t parts = lv.force ? lv.force : level_parts(N, lv.r, lv.T);
    const uint32_t S = (N + lv.T - 1) / lv.T;
    uint32_t sl = 0;
    for (uint32_t j = 0; j < parts; ++j) {
      const uint32_t a = (uint32_t)(((uint64_t)j * N) / parts);
      const uint32_t b = (uint32_t)(((uint64_t)(j + 1) * N) / parts);
      sl += (b - a + lv.T - 1) / lv.T;
    }
    pc[g] = parts;
    pcut[g] = parts * S;
    pblk[g] = parts * ((S + RLM_NT - 1) / RLM_NT);
    pq[g] = parts * (S + 1);
    psl[g] = sl;
  }
  __syncthreads();
  const uint32_t nc = block_exscan<1024>(pc, G, tmp);
  uint32_t tot[4];
  tot[0] = block_exscan<1024>(pcut, G, tmp);
  tot[1] = block_exscan<1024>(pblk, G, tmp);
  tot[2] = block_exscan<1024>(pq, G, tmp);
  tot[3] = block_exscan<1024>(psl, G, tmp);
  const uint32_t caps[4] = {lv.capCut, lv.capBlk, lv.capQ, lv.capSlice};
  bool over = nc > lv.capChildren;
  for (int f = 0; f < 4; ++f) over = over || tot[f] > caps[f];
  if (over) {
    if (tid == 0) {
      rlm_error(w, nc > lv.capChildren ? AMS_DEVERR_GROUPS : AMS_DEVERR_TILES);
      w.hdr->nChildren = 0;
    }
    return;
  }
  for (uint32_t g = tid; g < G; g += 1024) {
    const RGroup P = w.groups[g];
    const uint32_t parts = lv.force ? lv.force : level_parts(P.size, lv.r, lv.T);
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    const uint32_t nbS = (S + RLM_NT - 1) / RLM_NT;
    uint32_t sl = psl[g];
    for (uint32_t j = 0; j < parts; ++j) {
      const uint32_t a = (uint32_t)(((uint64_t)j * P.size) / parts);
      const uint32_t b = (uint32_t)(((uint64_t)(j + 1) * P.size) / parts);
      RGroup c;
      c.start = P.start + a;
      c.size = b - a;
      c.parent = g;
      c.j = j;
      c.rank = a;
      c.last = j + 1 == parts;
      c.cutBase = pcut[g] + j * S;
      c.blkBase = pblk[g] + j * nbS;
      c.qBase = pq[g] + j * (S + 1);
      c.sliceBase = sl;
      c.pad[0] = c.pad[1] = 0;
      sl += (c.size + lv.T - 1) / lv.T;
      w.children[pc[g] + j] = c;
    }
  }
  if (tid == 0) {
    for (int f = 0; f < 4; ++f) w.hdr->cnt[f] = tot[f];
    w.hdr->nChildren = nc;
  }
}

// Owner tables of a level: selection block -> part, merge slice -> part.
__global__ void __launch_bounds__(RLM_NT) k_rlm_owners(RWs w, RLev lv) {
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    const uint32_t nb = (S + RLM_NT - 1) / RLM_NT, ns = (C.size + lv.T - 1) / lv.T;
    for (uint32_t k = threadIdx.x; k < nb; k += RLM_NT) w.blkOwner[C.blkBase + k] = c;
    for (uint32_t k = threadIdx.x; k < ns; k += RLM_NT) w.sliceOwner[C.sliceBase + k] = c;
  }
}

// Elements of x[lo, hi) (raw keys, sorted by their ord value) that precede
// the pivot (ord value v, sequence q, position t) in the order (key,
// sequence, position), for sequence i.
template <int KT>
AMS_DEV uint32_t count_before(const GMem<typename Key<KT>::T> *x, uint32_t lo, uint32_t hi,
                              typename Key<KT>::T v, uint32_t i, uint32_t q, uint32_t t) {
  typedef typename Key<KT>::T K;
  if (i == q) return t < lo ? lo : (t > hi ? hi : t);
  const bool le = i < q;  // earlier sequences: equal keys come first
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const K y = Key<KT>::enc(x[mid]);
    const bool before = le ? (y <= v) : (y < v);
    if (before) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// count_before for every pivot of a step at once: all searches run over the
// same window, so they advance in lock step (the window halves each round
// whatever the comparisons give) and the loads of a round overlap.
template <int KT>
AMS_DEV void count_before_all(const GMem<typename Key<KT>::T> *x, uint32_t lo, uint32_t hi,
                              const uint64_t *pv, const uint32_t *pq, const uint32_t *pt,
                              uint32_t np, uint32_t i, uint32_t (&cnt)[RLM_M]) {
  typedef typename Key<KT>::T K;
  uint32_t base[RLM_M];
  bool le[RLM_M];
#pragma unroll
  for (uint32_t m = 0; m < RLM_M; ++m) {
    base[m] = lo;
    le[m] = i < pq[m];  // earlier sequences: equal keys come first
  }
  uint32_t n = hi - lo;
  if (n) {
    // invariant: the count lies in [base, base + n]
    while (n > 1) {
      const uint32_t half = n >> 1;
      K y[RLM_M];
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) y[m] = Key<KT>::enc(x[base[m] + half - 1]);
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) {
        const K v = (K)pv[m];
        const bool before = le[m] ? (y[m] <= v) : (y[m] < v);
        base[m] += before ? half : 0u;
      }
      n -= half;
    }
    K y[RLM_M];
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) y[m] = Key<KT>::enc(x[base[m]]);
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) {
      const K v = (K)pv[m];
      const bool before = le[m] ? (y[m] <= v) : (y[m] < v);
      base[m] += before ? 1u : 0u;
    }
  }
#pragma unroll
  for (uint32_t m = 0; m < RLM_M; ++m) {
    uint32_t c = base[m];
    if (i == pq[m]) c = pt[m] < lo ? lo : (pt[m] > hi ? hi : pt[m]);  // the pivot's own sequence
    cnt[m] = m < np ? c : lo;
  }
}

// The decision of a step from the pivots' left counts: the windows between
// the pivot of largest rank below the sought one and the pivot of smallest
// rank at or above it.  Returns the new (mlo, mhi, krem, total, done).
struct RDecision {
  uint32_t mlo, mhi, krem, total, done;
};
AMS_DEV RDecision decide(const uint32_t *left, uint32_t np, uint32_t krem, uint32_t total) {
  uint32_t mlo = RLM_NONE, mhi = RLM_NONE, vlo = 0, vhi = total;
  for (uint32_t m = 0; m < np; ++m) {
    const uint32_t v = left[m];
    if (v >= krem) {
      if (v < vhi || mhi == RLM_NONE) {
        vhi = v;
        mhi = m;
      }
    } else if (v >= vlo) {
      vlo = v;
      mlo = m;
    }
  }
  RDecision d;
  d.mlo = mlo;
  d.mhi = mhi;
  d.krem = krem - vlo;
  d.total = vhi - vlo;
  d.done = d.total == d.krem;
  return d;
}

// Pivot stream of a selection: draw m of step `iter`.
AMS_DEV uint32_t pivot_draw(const RLev &lv, uint32_t c, uint32_t iter, uint32_t m,
                            uint32_t total) {
  const uint64_t st = stream_state(lv.seed, RLM_STREAM + lv.level, c, iter);
  return draw_pos(st, m, total);
}

// Windows of every selection: the whole of every sequence.  The first
// step's pivots (Section 4.1 leaves the choice open): pivot m is the key at
// the sought rank's proportional position in sequence q_m, drawn uniformly.
// Where the keys are spread alike over the sequences (every sequence is a
// sorted tile of the same mix) such a key's rank lies within about
// N / sqrt(T) of the sought one, so the first step's bracket is some
// hundred times narrower than that of uniformly drawn keys; any other input
// only loses that head start.  Later steps draw uniformly from the windows.
template <int KT>
__global__ void __launch_bounds__(RLM_NT) k_rlm_sel_init(RWs w, RLev lv, const void *src_) {
  typedef typename Key<KT>::T K;
  const GMem<K> *src = (const GMem<K> *)src_;
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    for (uint32_t i = threadIdx.x; i < S; i += RLM_NT) {
      w.lo[C.cutBase + i] = 0;
      w.hi[C.cutBase + i] = seq_len(P, i, lv.T);
    }
    if (threadIdx.x < RLM_M) {
      const uint32_t m = threadIdx.x;
      RSel *sp = w.sel + c;
      const uint32_t np = P.size < RLM_M ? P.size : RLM_M;
      if (m < np && C.j != 0) {
        const uint32_t q = pivot_draw(lv, c, 0, m, S);
        const uint32_t lq = seq_len(P, q, lv.T);
        uint32_t t = (uint32_t)(((uint64_t)C.rank * lq) / P.size);
        t = t < lq ? t : lq - 1;
        sp->pq[m] = q;
        sp->pt[m] = t;
        sp->pv[m] = (uint64_t)Key<KT>::enc(src[P.start + (size_t)q * lv.T + t]);
      }
      if (m == 0) {
        sp->np = np;
        sp->krem = C.rank;
        sp->total = P.size;
        sp->mlo = RLM_NONE;
        sp->mhi = RLM_NONE;
        sp->done = C.j == 0 ? 1u : 0u;  // the first part starts at rank 0
        sp->iter = 0;
      }
    }
  }
}

// Applies the previous decision to sequence i's window and counts the
// window keys before each pivot of the step; returns the window.
template <int KT>
AMS_DEV void sel_entry(const RWs &w, const RGroup &P, uint32_t e, uint32_t i, uint32_t T,
                       uint32_t mlo, uint32_t mhi, uint32_t np, const uint64_t *pv,
                       const uint32_t *pq, const uint32_t *pt, const GMem<typename Key<KT>::T> *src,
                       uint32_t (&L)[RLM_M], uint32_t &W) {
  typedef typename Key<KT>::T K;
  uint32_t lo = w.lo[e], hi = w.hi[e];
  if (mlo != RLM_NONE) lo = w.cc[(size_t)mlo * w.capCut + e];
  if (mhi != RLM_NONE) hi = w.cc[(size_t)mhi * w.capCut + e];
  if (hi < lo) {  // only a sequence that is not sorted inverts a window
    rlm_error(w, AMS_DEVERR_RANGE);
    hi = lo;
  }
  w.lo[e] = lo;
  w.hi[e] = hi;
  const GMem<K> *x = src + P.start + (size_t)i * T;
  uint32_t cnt[RLM_M];
  count_before_all<KT>(x, lo, hi, pv, pq, pt, np, i, cnt);
#pragma unroll
  for (uint32_t m = 0; m < RLM_M; ++m) {
    if (m < np) w.cc[(size_t)m * w.capCut + e] = cnt[m];
    L[m] = cnt[m] - lo;
  }
  W = hi - lo;
}

// Segments of G lanes (G a power of two) inside a workgroup of RLM_NT
// threads: sums and inclusive scans over a segment.  G <= 64 stays inside a
// wavefront; G = 128 or 256 spans waves and meets in LDS (every thread of
// the workgroup must call these: they hold barriers then).
AMS_DEV void seg_sum8(uint32_t (&v)[RLM_M], uint32_t G, uint32_t *red) {
  constexpr uint32_t NW = RLM_NT / 64;
  if (G <= 64) {
    for (uint32_t d = 1; d < G; d <<= 1) {
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) v[m] += __shfl_xor(v[m], d, 64);
    }
    return;
  }
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll
  for (uint32_t m = 0; m < RLM_M; ++m) v[m] = wave_sum(v[m]);
  if (lane == 0) {
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) red[m * NW + wave] = v[m];
  }
  __syncthreads();
  const uint32_t gw = G >> 6, w0 = wave & ~(gw - 1u);
#pragma unroll
  for (uint32_t m = 0; m < RLM_M; ++m) {
    uint32_t s = 0;
    for (uint32_t q = 0; q < gw; ++q) s += red[m * NW + w0 + q];
    v[m] = s;
  }
}

AMS_DEV uint32_t seg_incl_scan(uint32_t v, uint32_t G, uint32_t *carry) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  if (G <= 64) {
    const uint32_t k = lane & (G - 1u);
    for (uint32_t d = 1; d < G; d <<= 1) {
      const uint32_t y = __shfl_up(v, d, 64);
      if (k >= d) v += y;
    }
    return v;
  }
  v = wave_incl_scan(v);
  if (lane == 63) carry[wave] = v;
  __syncthreads();
  const uint32_t w0 = wave & ~((G >> 6) - 1u);
  for (uint32_t q = w0; q < wave; ++q) v += carry[q];
  return v;
}

// Groups of at most RLM_GROUP_SEQ sequences: a workgroup runs whole
// selections, every step, one sequence per thread, the windows in
// registers.  A segment of G threads (G a power of two, at least the
// group's sequence count) holds one selection, so a workgroup holds
// RLM_NT / G selections; a step counts, sums the counts over the segment,
// decides (every thread of the segment alike), and draws the next pivots
// from the windows that remain (Section 4.1).
template <int KT>
__global__ void __launch_bounds__(RLM_NT) k_rlm_select_group(RWs w, RLev lv, const void *src_,
                                                             uint32_t G) {
  typedef typename Key<KT>::T K;
  constexpr uint32_t NW = RLM_NT / 64, SMAX = RLM_NT / 4;  // G >= 4
  const GMem<K> *src = (const GMem<K> *)src_;
  __shared__ uint32_t red[RLM_M * NW];
  __shared__ uint32_t carry[NW];
  __shared__ uint64_t spv[2][SMAX * RLM_M];  // the next pivots, by step parity
  __shared__ uint32_t spq[2][SMAX * RLM_M], spt[2][SMAX * RLM_M];
  const uint32_t tid = threadIdx.x, nc = w.hdr->nChildren;
  const uint32_t per = RLM_NT / G, sl = tid / G, i = tid & (G - 1u);
  for (uint32_t c0 = blockIdx.x * per; c0 < nc; c0 += gridDim.x * per) {
    const uint32_t c = c0 + sl;
    bool valid = c < nc;
    RGroup C, P;
    uint32_t S = 0;
    if (valid) {
      C = w.children[c];
      P = w.groups[C.parent];
      S = (P.size + lv.T - 1) / lv.T;
      valid = S <= G;  // wider groups: the block kernels'
    }
    RSel *sp = w.sel + (valid ? c : 0u);
    uint32_t np = 0, krem = 0, total = 0, done = 1, iter = 0;
    uint64_t pv[RLM_M];
    uint32_t pq[RLM_M], pt[RLM_M];
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) {
      pv[m] = 0;
      pq[m] = pt[m] = 0;
    }
    if (valid) {
      np = sp->np;
      krem = sp->krem;
      total = sp->total;
      done = sp->done;
      iter = sp->iter;
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) {
        pv[m] = sp->pv[m];
        pq[m] = sp->pq[m];
        pt[m] = sp->pt[m];
      }
    }
    const bool mine = valid && i < S;  // this thread's sequence exists
    const uint32_t e = mine ? C.cutBase + i : 0u;
    uint32_t lo = 0, hi = 0;
    if (mine) {
      lo = w.lo[e];
      hi = w.hi[e];
    }
    const GMem<K> *x = src + (mine ? P.start + (size_t)i * lv.T : 0);
    uint32_t err = 0;
    for (uint32_t step = 0; step < lv.itmax; ++step) {
      if (!__syncthreads_or(done ? 0 : 1)) break;  // every selection here is done
      const uint32_t par = step & 1u;
      uint32_t cnt[RLM_M];
      if (mine && !done) {
        count_before_all<KT>(x, lo, hi, pv, pq, pt, np, i, cnt);
      } else {
#pragma unroll
        for (uint32_t m = 0; m < RLM_M; ++m) cnt[m] = lo;
      }
      uint32_t left[RLM_M];
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) left[m] = cnt[m] - lo;
      seg_sum8(left, G, red);
      uint32_t z = 0;
      if (!done) {
        const RDecision d = decide(left, np, krem, total);
        uint32_t nlo = lo, nhi = hi;
#pragma unroll
        for (uint32_t m = 0; m < RLM_M; ++m) {
          nlo = m == d.mlo ? cnt[m] : nlo;
          nhi = m == d.mhi ? cnt[m] : nhi;
        }
        if (nhi < nlo) {  // only a sequence that is not sorted inverts a window
          err = 1;
          nhi = nlo;
        }
        lo = nlo;
        hi = nhi;
        krem = d.krem;
        total = d.total;
        done = d.done;
        ++iter;
        z = done ? 0u : hi - lo;
      }
      const uint32_t incl = seg_incl_scan(z, G, carry);
      if (!done) {
        // the draws: key u of the windows in sequence order lies in the
        // window of the thread whose scan range holds it
        np = total < RLM_M ? total : RLM_M;
        const uint32_t excl = incl - z;
        for (uint32_t m = 0; m < np; ++m) {
          const uint32_t u = pivot_draw(lv, c, iter, m, total);
          if (u >= excl && u < incl) {
            const uint32_t t = lo + (u - excl);
            spv[par][sl * RLM_M + m] = (uint64_t)Key<KT>::enc(x[t]);
            spq[par][sl * RLM_M + m] = i;
            spt[par][sl * RLM_M + m] = t;
          }
        }
        if (i == G - 1u && incl != total) err = 1;  // the windows must hold `total` keys
      }
      __syncthreads();
      if (!done) {
#pragma unroll
        for (uint32_t m = 0; m < RLM_M; ++m) {
          if (m < np) {
            pv[m] = spv[par][sl * RLM_M + m];
            pq[m] = spq[par][sl * RLM_M + m];
            pt[m] = spt[par][sl * RLM_M + m];
          }
        }
      }
    }
    if (err) rlm_error(w, AMS_DEVERR_RANGE);
    if (mine) {
      w.lo[e] = lo;
      w.hi[e] = hi;
    }
    if (valid && i == 0) {
      sp->np = np;
      sp->krem = krem;
      sp->total = total;
      sp->mlo = RLM_NONE;  // the windows above are final
      sp->mhi = RLM_NONE;
      sp->done = done;
      sp->iter = iter;
    }
  }
}

// Wider groups, one step of every unfinished selection per pair of
// launches.  Count: an item is (selection, block of RLM_NT sequences); each
// applies the previous decision to its windows, counts the keys before each
// pivot and leaves the block's sums.  The kernel boundary orders those sums
// before the decide kernel reads them.
template <int KT>
__global__ void __launch_bounds__(RLM_NT) k_rlm_sel_count(RWs w, RLev lv, const void *src_) {
  typedef typename Key<KT>::T K;
  const GMem<K> *src = (const GMem<K> *)src_;
  constexpr uint32_t NW = RLM_NT / 64;
  constexpr uint32_t PB = RLM_M + 1;  // partials per block
  __shared__ uint32_t red[PB * NW];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t nb = w.hdr->cnt[1];
  for (uint32_t item = blockIdx.x; item < nb; item += gridDim.x) {
    const uint32_t c = w.blkOwner[item];
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    if (S <= RLM_GROUP_SEQ) continue;  // the group kernel's
    const RSel *sp = w.sel + c;
    if (sp->done) continue;
    const uint32_t b = item - C.blkBase;
    const uint32_t np = sp->np, mlo = sp->mlo, mhi = sp->mhi;
    uint64_t pv[RLM_M];
    uint32_t pq[RLM_M], pt[RLM_M];
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) {
      pv[m] = sp->pv[m];
      pq[m] = sp->pq[m];
      pt[m] = sp->pt[m];
    }
    uint32_t L[RLM_M], Wi = 0;
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) L[m] = 0;
    const uint32_t i = b * RLM_NT + tid;
    if (i < S) sel_entry<KT>(w, P, C.cutBase + i, i, lv.T, mlo, mhi, np, pv, pq, pt, src, L, Wi);
#pragma unroll
    for (uint32_t m = 0; m < RLM_M; ++m) L[m] = wave_sum(L[m]);
    Wi = wave_sum(Wi);
    if (lane == 0) {
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) red[m * NW + wave] = L[m];
      red[RLM_M * NW + wave] = Wi;
    }
    __syncthreads();
    if (tid < PB) {
      uint32_t v = 0;
      for (uint32_t q = 0; q < NW; ++q) v += red[tid * NW + q];
      w.bl[(size_t)(C.blkBase + b) * PB + tid] = v;
    }
    __syncthreads();
  }
}

// Decide: one workgroup per unfinished selection sums the block sums,
// decides which windows remain and draws the next pivots from them.
template <int KT>
__global__ void __launch_bounds__(RLM_NT) k_rlm_sel_decide(RWs w, RLev lv, const void *src_) {
  typedef typename Key<KT>::T K;
  const GMem<K> *src = (const GMem<K> *)src_;
  constexpr uint32_t NW = RLM_NT / 64;
  constexpr uint32_t PB = RLM_M + 1;
  __shared__ uint32_t red[PB * NW];
  __shared__ uint32_t sleft[RLM_M];
  __shared__ uint32_t sbq[RLM_M], srr[RLM_M];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    if (S <= RLM_GROUP_SEQ) continue;
    RSel *sp = w.sel + c;
    if (sp->done) continue;
    const uint32_t nblk = (S + RLM_NT - 1) / RLM_NT;
    const uint32_t np = sp->np;
    const uint32_t *blp = w.bl + (size_t)C.blkBase * PB;
    {
      uint32_t acc[RLM_M];
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) acc[m] = 0;
      for (uint32_t q = tid; q < nblk; q += RLM_NT) {
#pragma unroll
        for (uint32_t m = 0; m < RLM_M; ++m) acc[m] += blp[(size_t)q * PB + m];
      }
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) acc[m] = wave_sum(acc[m]);
      if (lane == 0) {
#pragma unroll
        for (uint32_t m = 0; m < RLM_M; ++m) red[m * NW + wave] = acc[m];
      }
      __syncthreads();
      if (tid < RLM_M) {
        uint32_t v = 0;
        for (uint32_t q = 0; q < NW; ++q) v += red[tid * NW + q];
        sleft[tid] = v;
      }
      __syncthreads();
    }
    const RDecision d = decide(sleft, np, sp->krem, sp->total);
    const uint32_t iter = sp->iter + 1;
    const uint32_t np2 = d.total < RLM_M ? d.total : RLM_M;
    if (!d.done) {
      // level 1: per-block sizes of the new windows over contiguous chunks
      // of blocks per thread, scanned; the thread whose chunk holds draw m
      // finds its block and the rank inside it
      const uint32_t per = (nblk + RLM_NT - 1) / RLM_NT;
      const uint32_t q0 = tid * per < nblk ? tid * per : nblk;
      const uint32_t q1 = q0 + per < nblk ? q0 + per : nblk;
      auto bsize = [&](uint32_t q) -> uint32_t {
        const uint32_t *r = blp + (size_t)q * PB;
        const uint32_t hiv = d.mhi == RLM_NONE ? r[RLM_M] : r[d.mhi];
        const uint32_t lov = d.mlo == RLM_NONE ? 0u : r[d.mlo];
        return hiv - lov;
      };
      uint32_t mine = 0;
      for (uint32_t q = q0; q < q1; ++q) mine += bsize(q);
      const uint32_t incl = wave_incl_scan(mine);
      __syncthreads();
      if (lane == 63) red[wave] = incl;
      if (tid < RLM_M) sbq[tid] = 0xFFFFFFFFu;
      __syncthreads();
      uint32_t off = 0;
      for (uint32_t q = 0; q < wave; ++q) off += red[q];
      const uint32_t first = off + incl - mine;
      for (uint32_t m = 0; m < np2; ++m) {
        const uint32_t u = pivot_draw(lv, c, iter, m, d.total);
        if (mine && u >= first && u < first + mine) {
          uint32_t r = u - first, q = q0;
          for (; q < q1; ++q) {
            const uint32_t z = bsize(q);
            if (r < z) break;
            r -= z;
          }
          sbq[m] = q;
          srr[m] = r;
        }
      }
      __syncthreads();
      // level 2: inside each draw's block, the sequence holding its rank
      uint32_t za[RLM_M], zs[RLM_M];
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) {
        const uint32_t bq = m < np2 && sbq[m] < nblk ? sbq[m] : 0xFFFFFFFFu;
        const uint32_t ii = bq == 0xFFFFFFFFu ? S : bq * RLM_NT + tid;
        za[m] = 0;
        zs[m] = 0;
        if (ii < S) {
          const uint32_t e = C.cutBase + ii;
          const uint32_t lo_ = d.mlo == RLM_NONE ? w.lo[e] : w.cc[(size_t)d.mlo * w.capCut + e];
          const uint32_t hi_ = d.mhi == RLM_NONE ? w.hi[e] : w.cc[(size_t)d.mhi * w.capCut + e];
          za[m] = lo_;
          zs[m] = hi_ > lo_ ? hi_ - lo_ : 0u;  // inverted only over unsorted sequences
        }
      }
      uint32_t inc2[RLM_M];
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) inc2[m] = wave_incl_scan(zs[m]);
      __syncthreads();
      if (lane == 63) {
#pragma unroll
        for (uint32_t m = 0; m < RLM_M; ++m) red[m * NW + wave] = inc2[m];
      }
      __syncthreads();
#pragma unroll
      for (uint32_t m = 0; m < RLM_M; ++m) {
        if (m >= np2 || sbq[m] >= nblk) continue;
        uint32_t off2 = 0;
        for (uint32_t q = 0; q < wave; ++q) off2 += red[m * NW + q];
        const uint32_t f2 = off2 + inc2[m] - zs[m];
        const uint32_t rr = srr[m];
        if (zs[m] && rr >= f2 && rr < f2 + zs[m]) {
          const uint32_t ii = sbq[m] * RLM_NT + tid;
          const uint32_t t = za[m] + (rr - f2);
          sp->pq[m] = ii;
          sp->pt[m] = t;
          sp->pv[m] = (uint64_t)Key<KT>::enc(src[P.start + (size_t)ii * lv.T + t]);
        }
      }
      if (tid == 0) {
        for (uint32_t m = 0; m < np2; ++m)
          if (sbq[m] >= nblk) rlm_error(w, AMS_DEVERR_RANGE);  // a draw outside the windows
      }
    }
    __syncthreads();
    if (tid == 0) {
      sp->np = np2;
      sp->krem = d.krem;
      sp->total = d.total;
      sp->mlo = d.mlo;
      sp->mhi = d.mhi;
      sp->done = d.done;
      sp->iter = iter;
    }
    __syncthreads();
  }
}

// Cut positions: the windows' upper ends once the last decision is applied.
__global__ void __launch_bounds__(RLM_NT) k_rlm_cut(RWs w, RLev lv) {
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    const RSel *sp = w.sel + c;
    const uint32_t done = sp->done, mhi = sp->mhi;
    if (threadIdx.x == 0 && !done) rlm_error(w, AMS_DEVERR_RANGE);
    for (uint32_t i = threadIdx.x; i < S; i += RLM_NT) {
      const uint32_t e = C.cutBase + i;
      uint32_t v;
      if (C.j == 0) v = 0;
      else v = mhi == RLM_NONE ? w.hi[e] : w.cc[(size_t)mhi * w.capCut + e];
      w.cut[e] = v;
    }
  }
}

// Piece offsets of every part: Q[i] = keys of the part in sequences < i.
template <uint32_t NT>
__global__ void __launch_bounds__(NT) k_rlm_pieces(RWs w, RLev lv) {
  __shared__ uint32_t tmp[NT / 64];
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    uint32_t *Q = w.q + C.qBase;
    for (uint32_t i = threadIdx.x; i < S; i += NT) {
      const uint32_t a = w.cut[C.cutBase + i];
      // the next part's cut row follows this one (same parent, same S)
      const uint32_t b = C.last ? seq_len(P, i, lv.T) : w.cut[C.cutBase + S + i];
      Q[i] = b >= a ? b - a : 0u;
    }
    __syncthreads();
    const uint32_t tot = block_exscan<NT>(Q, S, tmp);
    if (threadIdx.x == 0) {
      Q[S] = tot;
      if (tot != C.size) rlm_error(w, AMS_DEVERR_RANGE);
    }
    __syncthreads();
    if (tot != C.size) continue;
    // the pieces each slice of T keys overlaps: slice k starts in the piece
    // holding key k*T and ends in the piece holding its last key
    const uint32_t nsl = (C.size + lv.T - 1) / lv.T;
    for (uint32_t i = threadIdx.x; i < S; i += NT) {
      const uint32_t qa = Q[i], qb = Q[i + 1];
      if (qa >= qb) continue;  // empty piece
      for (uint32_t k = (qa + lv.T - 1) / lv.T; k < nsl && k * lv.T < qb; ++k)
        w.sliceI0[C.sliceBase + k] = i;
      const uint32_t k0 = qa / lv.T;  // slices whose last key may lie in [qa, qb)
      for (uint32_t k = k0; k < nsl; ++k) {
        const uint32_t lastKey = ((k + 1) * lv.T < C.size ? (k + 1) * lv.T : C.size) - 1;
        if (lastKey >= qb) break;
        if (lastKey >= qa) w.sliceI1[C.sliceBase + k] = i + 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Merge of one slice: the keys [a, a+len) of a part's piece concatenation
// (pieces in sequence order), gathered into LDS and merged pairwise.
// ---------------------------------------------------------------------------
template <typename K>
AMS_DEV uint32_t upper_le(const uint32_t *v, uint32_t n, uint32_t x) {
  // largest k in [0, n) with v[k] <= x (v[0] <= x)
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (v[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Key slots of the merge buffer: one spare slot after every 8 keys.  A
// thread's 8 outputs of a merge round (keys 8t .. 8t+7) then sit in 8
// consecutive slots, and threads whose runs lie 4 to 8 keys apart meet in
// different LDS banks.
AMS_DEV uint32_t lpad(uint32_t x) { return x + (x >> 3); }
AMS_HD uint32_t lpad_size(uint32_t T) { return T + (T >> 3); }

template <int KT>
__global__ void __launch_bounds__(RLM_MT, 6) k_rlm_merge(RWs w, RLev lv, const void *src_,
                                                         void *dst_) {
  typedef typename Key<KT>::T K;
  constexpr uint32_t PT = RLM_TMAX / RLM_MT;  // keys per thread and slice
  constexpr uint32_t NW = RLM_MT / 64;
  const GMem<K> *src = (const GMem<K> *)src_;
  GMem<K> *dst = (GMem<K> *)dst_;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t T = lv.T;
  // the slice, merged in place (a round's outputs wait in registers until
  // every thread has read its inputs), and two segment lists (the current
  // round's and the next one's), T + 1 starts relative to the slice each
  K *buf = (K *)smem_raw;
  uint16_t *segA = (uint16_t *)(buf + lpad_size(T));
  uint16_t *segB = segA + (T + 1);
  __shared__ uint32_t ccount[PT * NW];  // piece starts per 64 keys (many pieces)
  __shared__ uint32_t shd[2];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t ns = w.hdr->cnt[3];
  for (uint32_t item = blockIdx.x; item < ns; item += gridDim.x) {
    const RGroup C = w.children[w.sliceOwner[item]];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + T - 1) / T;
    const uint32_t *Q = w.q + C.qBase;
    const uint32_t *cut = w.cut + C.cutBase;
    if (Q[S] != C.size) continue;  // the piece offsets raised an error already
    const uint32_t a = (item - C.sliceBase) * T;
    const uint32_t len = C.size - a < T ? C.size - a : T;
    // pieces overlapping [a, a + len), found by k_rlm_pieces
    const uint32_t i0 = w.sliceI0[item], i1 = w.sliceI1[item];
    if (i0 >= i1 || i1 > S) {  // cannot happen
      if (tid == 0) rlm_error(w, AMS_DEVERR_RANGE);
      continue;
    }
    const uint32_t np = i1 - i0;
    // piece offsets relative to the slice: max(Q[i] - a, 0), at most len;
    // the first piece starts a - Q[i0] keys before the slice
    const bool cached = np <= T;
    if (cached)
      for (uint32_t k = tid; k <= np; k += RLM_MT) {
        const uint32_t q = Q[i0 + k];
        segA[k] = (uint16_t)(q > a ? (q - a < len ? q - a : len) : 0u);
      }
    if (tid == 0) shd[0] = a - Q[i0];
    __syncthreads();
    const uint32_t lead = shd[0];
    // gather: key x of the slice comes from the piece holding a + x; each
    // key's load is issued as soon as its piece is found, all in flight
    // together before the first is stored
    K v[PT];
    bool st[PT];
#pragma unroll
    for (uint32_t u = 0; u < PT; ++u) {
      const uint32_t x = tid + u * RLM_MT;
      uint32_t k = 0, rel = 0;
      if (x < len) {
        if (cached) {
          uint32_t l = 0, h = np;  // last k with seg[k] <= x
          while (h - l > 1) {
            const uint32_t m = (l + h) >> 1;
            if (segA[m] <= x) l = m; else h = m;
          }
          k = l;
          rel = segA[k];
        } else {
          k = upper_le<K>(Q + i0, np, a + x);
          rel = Q[i0 + k] > a ? Q[i0 + k] - a : 0u;
        }
      }
      const uint32_t i = i0 + k;
      // position in sequence i: the piece's cut plus the keys of the piece
      // before x (the first piece also counts those before the slice)
      const uint32_t pos = cut[i] + (x - rel) + (k == 0 ? lead : 0u);
      st[u] = x < len && (x == 0 || (k != 0 && rel == x));  // a piece starts here
      const bool ok = x < len && pos < seq_len(P, i, T);
      if (x < len && !ok) rlm_error(w, AMS_DEVERR_RANGE);  // cannot happen
      v[u] = ok ? Key<KT>::enc(src[P.start + (size_t)i * T + pos]) : (K)0;
    }
    // slot of key tid + u RLM_MT: lpad(tid) + u (RLM_MT + RLM_MT / 8)
    K *gb = buf + lpad(tid);
#pragma unroll
    for (uint32_t u = 0; u < PT; ++u)
      if (tid + u * RLM_MT < len) gb[u * (RLM_MT + RLM_MT / 8)] = v[u];
    __syncthreads();  // every piece search done before the piece list is compacted
    uint32_t nseg;
    if (cached) {
      // the merge's segments are the non-empty pieces: their starts,
      // compacted in place by the first wave (an entry moves down only)
      if (tid < 64) {
        uint32_t base = 0;
        for (uint32_t k0 = 0; k0 < np; k0 += 64) {
          const uint32_t k = k0 + tid;
          const uint32_t s0 = k < np ? segA[k] : 0u, s1 = k < np ? segA[k + 1] : 0u;
          const bool keep = k < np && s1 > s0;
          const uint64_t mk = ballot(keep);
          if (keep) segA[base + bits_below(mk)] = (uint16_t)s0;
          base += (uint32_t)__builtin_popcountll(mk);
        }
        if (tid == 0) {
          segA[base] = (uint16_t)len;
          shd[1] = base;
        }
      }
      __syncthreads();
      nseg = shd[1];
    } else {
      // the piece starts in key order: ballots per 64 keys, then each 64
      // keys' offset among all starts (chunk (u, wave) holds keys
      // [u * RLM_MT + 64 wave, + 64))
      uint64_t mk[PT];
#pragma unroll
      for (uint32_t u = 0; u < PT; ++u) {
        mk[u] = ballot(st[u]);
        if (lane == 0) ccount[u * NW + wave] = (uint32_t)__builtin_popcountll(mk[u]);
      }
      __syncthreads();
      nseg = 0;
      uint32_t before[PT];
#pragma unroll
      for (uint32_t u = 0; u < PT; ++u) before[u] = 0;
      for (uint32_t j = 0; j < PT * NW; ++j) {
        const uint32_t c = ccount[j];
#pragma unroll
        for (uint32_t u = 0; u < PT; ++u) before[u] += j < u * NW + wave ? c : 0u;
        nseg += c;
      }
#pragma unroll
      for (uint32_t u = 0; u < PT; ++u)
        if (st[u]) segA[before[u] + bits_below(mk[u])] = (uint16_t)(tid + u * RLM_MT);
      if (tid == 0) segA[nseg] = (uint16_t)len;
    }
    __syncthreads();
    // pairwise merge rounds: segments (2m, 2m+1) -> m, A first on ties.
    // Thread outputs [x0, x1): the pair holding x0 and the merge-path split
    // (pa, pb) of its two segments; both heads stay in registers, so a step
    // reads one key; where the range reaches the next pair, that pair
    // starts at its beginning.
    uint32_t nsg = nseg;
    uint16_t *sin = segA, *sout = segB;
    const uint32_t x0 = tid * PT < len ? tid * PT : len;  // outputs [x0, x1)
    const uint32_t x1 = x0 + PT < len ? x0 + PT : len;
    K *ob = buf + lpad(x0);  // their slots: ob[0 .. x1 - x0)
    while (nsg > 1) {
      K o[PT];
#pragma unroll
      for (uint32_t k = 0; k < PT; ++k) o[k] = (K)0;
      if (x0 < x1) {
        uint32_t l = 0, h = (nsg + 1) / 2;  // pairs
        while (h - l > 1) {
          const uint32_t m = (l + h) >> 1;
          if (sin[2 * m] <= x0) l = m; else h = m;
        }
        uint32_t m = l;
        uint32_t as = sin[2 * m], ae = sin[2 * m + 1];
        uint32_t be = 2 * m + 2 <= nsg ? sin[2 * m + 2] : ae;
        const uint32_t rho = x0 - as;
        const uint32_t na = ae - as, nb = be - ae;
        uint32_t clo = rho > nb ? rho - nb : 0, chi = rho < na ? rho : na;
        while (clo < chi) {
          const uint32_t mid = (clo + chi) >> 1;
          if (buf[lpad(as + mid)] <= buf[lpad(ae + rho - mid - 1)]) clo = mid + 1; else chi = mid;
        }
        uint32_t pa = as + clo, pb = ae + (rho - clo);
        K ha = pa < ae ? buf[lpad(pa)] : (K)0, hb = pb < be ? buf[lpad(pb)] : (K)0;
#pragma unroll
        for (uint32_t k = 0; k < PT; ++k) {
          const uint32_t x = x0 + k;
          if (x < x1) {
            if (x == be) {  // the next pair, from its beginning
              ++m;
              as = be;
              ae = sin[2 * m + 1];
              be = 2 * m + 2 <= nsg ? sin[2 * m + 2] : ae;
              pa = as;
              pb = ae;
              ha = pa < ae ? buf[lpad(pa)] : (K)0;
              hb = pb < be ? buf[lpad(pb)] : (K)0;
            }
            const bool takeA = pb >= be || (pa < ae && ha <= hb);
            o[k] = takeA ? ha : hb;
            pa += takeA ? 1u : 0u;
            pb += takeA ? 0u : 1u;
            const uint32_t pn = takeA ? pa : pb;
            const K nv = pn < (takeA ? ae : be) ? buf[lpad(pn)] : (K)0;
            ha = takeA ? nv : ha;
            hb = takeA ? hb : nv;
          }
        }
      }
      const uint32_t nn = (nsg + 1) / 2;
      __syncthreads();  // every input read
#pragma unroll
      for (uint32_t k = 0; k < PT; ++k)
        if (x0 + k < x1) ob[k] = o[k];
      // segments of the next round: every other boundary
      for (uint32_t k = tid; k < nn; k += RLM_MT) sout[k] = sin[2 * k];
      if (tid == 0) sout[nn] = (uint16_t)len;
      __syncthreads();
      nsg = nn;
      uint16_t *t = sin;
      sin = sout;
      sout = t;
    }
    // keys leave LDS as raw bits at every level (the next level encodes
    // them again on load, as it does the tile sort's output).  The loop
    // starts sh keys before the slice, at a 128-byte line, so that every
    // wavefront stores whole lines (only the slice's first and last lines
    // are shared with its neighbours).
    constexpr uint32_t LK = 128 / sizeof(K);  // keys per 128-byte line
    const uint32_t sh = (uint32_t)((C.start + a) & (LK - 1u));
    for (uint32_t y = tid; y < len + sh; y += RLM_MT)
      if (y >= sh) dst[C.start + a + (y - sh)] = Key<KT>::dec(buf[lpad(y - sh)]);
    __syncthreads();
  }
}

__global__ void k_rlm_root(RWs w, uint32_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    RGroup g;
    memset(&g, 0, sizeof g);
    g.size = n;
    g.last = 1;
    w.groups[0] = g;
    memset(w.hdr, 0, sizeof(RHdr));
    w.hdr->nGroups = 1;
  }
}

__global__ void k_rlm_next(RWs w) {
  if (threadIdx.x == 0 && blockIdx.x == 0) w.hdr->nGroups = w.hdr->nChildren;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct RPlan {
  int kt;
  uint32_t kw, T, r, L;
  uint64_t n, seed;
  uint32_t flags;
  // per level: groups entering it, and the largest tables it fills
  uint32_t maxGroups, maxChildren, maxCut, maxBlk, maxQ, maxSlice;
  uint32_t itmax[RLM_MAXLEV];
  uint64_t maxS[RLM_MAXLEV];  // largest group of each level, in sequences
  size_t o_hdr, o_tmp, o_tile, o_g0, o_g1, o_sel, o_lo, o_hi, o_cc, o_cut, o_bl, o_bown, o_sown,
      o_si0, o_si1, o_q, o_scr, bytes;
};

// Steps a selection over N keys may take: with RLM_M pivots per step the
// windows shrink about (RLM_M + 1)-fold per step, so about log2(N) / 3
// steps are expected; this bound leaves ample room.
uint32_t sel_steps(uint64_t N) { return (64 - __builtin_clzll(N | 1)) / 2 + 12; }

uint32_t host_parts(uint64_t N, uint32_t r, uint32_t T) {
  if (N > (uint64_t)r * T) return r;
  return N == 0 ? 1u : (uint32_t)((N + T - 1) / T);
}

ams_status make_rlm_plan(RPlan &pl, ams_key_t t, uint64_t n, const ams_rlm_params *p) {
  memset(&pl, 0, sizeof pl);
  if (t != AMS_U32 && t != AMS_U64 && t != AMS_F32) {
    set_error("unknown key type %d", (int)t);
    return AMS_EINVAL;
  }
  if (n > AMS_MAX_SEGMENT) {
    set_error("%llu keys: at most %llu are supported", (unsigned long long)n,
              (unsigned long long)AMS_MAX_SEGMENT);
    return AMS_EUNSUPPORTED;
  }
  pl.kt = (int)t;
  pl.kw = t == AMS_U64 ? 8 : 4;
  pl.n = n;
  pl.r = (p && p->ways) ? p->ways : 16;
  pl.T = (p && p->tile_keys) ? p->tile_keys : RLM_TMAX;
  pl.seed = (p && p->seed) ? p->seed : 14106754ull;
  pl.flags = p ? p->flags : 0;
  if (pl.r < 2 || pl.r > 1024) {
    set_error("ways must be in 2..1024 (got %u)", pl.r);
    return AMS_EINVAL;
  }
  const uint32_t C = base_case_capacity(pl.kw, false);
  if (pl.T < 64 || pl.T > RLM_TMAX || pl.T > C || pl.T % 64) {
    set_error("tile_keys must be a multiple of 64 in 64..%u (got %u)", std::min(RLM_TMAX, C), pl.T);
    return AMS_EINVAL;
  }
  // the level structure: group sizes follow from n, r and T alone
  std::vector<uint64_t> sizes{n}, next;
  uint32_t L = 0;
  pl.maxGroups = 1;
  while (n > pl.T) {
    uint64_t mx = 0;
    for (uint64_t s : sizes) mx = std::max(mx, s);
    if (mx <= pl.T) break;
    if (L == RLM_MAXLEV) {
      set_error("too many levels");
      return AMS_EUNSUPPORTED;
    }
    next.clear();
    uint64_t cut = 0, blk = 0, q = 0, slc = 0;
    for (uint64_t N : sizes) {
      const uint32_t parts = host_parts(N, pl.r, pl.T);
      const uint64_t S = (N + pl.T - 1) / pl.T;
      for (uint32_t j = 0; j < parts; ++j) {
        const uint64_t a = j * N / parts, b = (j + 1) * N / parts;
        next.push_back(b - a);
        cut += S;
        blk += (S + RLM_NT - 1) / RLM_NT;
        q += S + 1;
        slc += (b - a + pl.T - 1) / pl.T;
      }
    }
    uint64_t maxS = 0;
    for (uint64_t N : sizes) maxS = std::max(maxS, (N + pl.T - 1) / pl.T);
    pl.maxS[L] = maxS;
    pl.itmax[L] = sel_steps(mx);
    pl.maxChildren = std::max<uint32_t>(pl.maxChildren, (uint32_t)next.size());
    pl.maxCut = std::max<uint32_t>(pl.maxCut, (uint32_t)cut);
    pl.maxBlk = std::max<uint32_t>(pl.maxBlk, (uint32_t)blk);
    pl.maxQ = std::max<uint32_t>(pl.maxQ, (uint32_t)q);
    pl.maxSlice = std::max<uint32_t>(pl.maxSlice, (uint32_t)slc);
    pl.maxGroups = std::max<uint32_t>(pl.maxGroups, (uint32_t)next.size());
    sizes.swap(next);
    ++L;
  }
  pl.L = L;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o = al256(o + b);
    return at;
  };
  pl.o_hdr = take(sizeof(RHdr));
  pl.o_tmp = take(L ? n * pl.kw : 0);
  pl.o_tile = take(tile_sort_ws_bytes(n, pl.T));
  const size_t ng = std::max<uint32_t>(pl.maxGroups, 1);
  pl.o_g0 = take(ng * sizeof(RGroup));
  pl.o_g1 = take(ng * sizeof(RGroup));
  pl.o_sel = take((size_t)pl.maxChildren * sizeof(RSel));
  pl.o_lo = take((size_t)pl.maxCut * 4);
  pl.o_hi = take((size_t)pl.maxCut * 4);
  pl.o_cc = take((size_t)RLM_M * pl.maxCut * 4);
  pl.o_cut = take((size_t)pl.maxCut * 4);
  pl.o_bl = take((size_t)(RLM_M + 1) * pl.maxBlk * 4);
  pl.o_bown = take((size_t)pl.maxBlk * 4);
  pl.o_sown = take((size_t)pl.maxSlice * 4);
  pl.o_si0 = take((size_t)pl.maxSlice * 4);
  pl.o_si1 = take((size_t)pl.maxSlice * 4);
  pl.o_q = take((size_t)pl.maxQ * 4);
  pl.o_scr = take(5 * (ng + 1) * 4);
  pl.bytes = o;
  return AMS_OK;
}

uint32_t grid_cap(uint64_t items, uint32_t cap) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(items, cap));
}

// Segment width of the group kernel: a power of two, at least 4 (so a
// workgroup holds at most RLM_NT / 4 selections), at least the level's
// largest group up to RLM_GROUP_SEQ sequences.
uint32_t group_width(uint64_t maxS) {
  uint32_t G = 4;
  while (G < maxS && G < RLM_GROUP_SEQ) G <<= 1;
  return G;
}

// All selections of a level: the group kernel runs the small groups' whole
// selections in one launch; the wider groups take one step per pair of
// count and decide launches.
template <int KT>
void select_level(const RWs &w, const RLev &lv, const void *src, uint32_t maxChildren,
                  uint32_t maxBlk, uint64_t maxS, hipStream_t s) {
  hipLaunchKernelGGL(k_rlm_sel_init<KT>, dim3(grid_cap(maxChildren, 2048)), dim3(RLM_NT), 0, s, w,
                     lv, src);
  const uint32_t G = group_width(maxS), per = RLM_NT / G;
  hipLaunchKernelGGL(k_rlm_select_group<KT>, dim3(grid_cap((maxChildren + per - 1) / per, 4096)),
                     dim3(RLM_NT), 0, s, w, lv, src, G);
  if (maxS > RLM_GROUP_SEQ)
    for (uint32_t it = 0; it < lv.itmax; ++it) {
      hipLaunchKernelGGL(k_rlm_sel_count<KT>, dim3(grid_cap(maxBlk, 4096)), dim3(RLM_NT), 0, s, w,
                         lv, src);
      hipLaunchKernelGGL(k_rlm_sel_decide<KT>, dim3(grid_cap(maxChildren, 2048)), dim3(RLM_NT), 0,
                         s, w, lv, src);
    }
  hipLaunchKernelGGL(k_rlm_cut, dim3(grid_cap(maxChildren, 2048)), dim3(RLM_NT), 0, s, w, lv);
}

template <int KT>
ams_status rlm_typed(const RPlan &pl, const void *in, void *out, void *wsv, hipStream_t s) {
  typedef typename Key<KT>::T K;
  char *base = (char *)wsv;
  RWs w;
  w.hdr = (RHdr *)(base + pl.o_hdr);
  w.groups = (RGroup *)(base + pl.o_g0);
  w.children = (RGroup *)(base + pl.o_g1);
  w.sel = (RSel *)(base + pl.o_sel);
  w.lo = (uint32_t *)(base + pl.o_lo);
  w.hi = (uint32_t *)(base + pl.o_hi);
  w.cc = (uint32_t *)(base + pl.o_cc);
  w.cut = (uint32_t *)(base + pl.o_cut);
  w.bl = (uint32_t *)(base + pl.o_bl);
  w.blkOwner = (uint32_t *)(base + pl.o_bown);
  w.sliceOwner = (uint32_t *)(base + pl.o_sown);
  w.sliceI0 = (uint32_t *)(base + pl.o_si0);
  w.sliceI1 = (uint32_t *)(base + pl.o_si1);
  w.q = (uint32_t *)(base + pl.o_q);
  w.capCut = pl.maxCut;
  w.scratch = (uint32_t *)(base + pl.o_scr);
  void *tmp = base + pl.o_tmp;
  // buffer of level l's output: the last level writes `out`
  auto buf = [&](uint32_t l) -> void * { return ((pl.L - l) & 1u) ? tmp : out; };
  hipLaunchKernelGGL(k_rlm_root, dim3(1), dim3(64), 0, s, w, (uint32_t)pl.n);
  ams_status st = run_tile_sort(KT, false, in, nullptr, buf(0), nullptr, pl.n, pl.T,
                                base + pl.o_tile, s);
  if (st) return st;
  const size_t ldsM = (size_t)lpad_size(pl.T) * sizeof(K) + 2 * ((size_t)pl.T + 1) * 2;
  (void)hipFuncSetAttribute((const void *)k_rlm_merge<KT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsM);
  for (uint32_t l = 0; l < pl.L; ++l) {
    RLev lv;
    memset(&lv, 0, sizeof lv);
    lv.T = pl.T;
    lv.r = pl.r;
    lv.level = l;
    lv.last = l + 1 == pl.L;
    lv.itmax = pl.itmax[l];
    lv.capChildren = pl.maxChildren;
    lv.capCut = pl.maxCut;
    lv.capBlk = pl.maxBlk;
    lv.capQ = pl.maxQ;
    lv.capSlice = pl.maxSlice;
    lv.seed = pl.seed;
    const void *src = buf(l);
    void *dst = buf(l + 1);
    {
      TraceScope ts("rlm_children", l, s);
      hipLaunchKernelGGL(k_rlm_children, dim3(1), dim3(1024), 0, s, w, lv);
      hipLaunchKernelGGL(k_rlm_owners, dim3(grid_cap(pl.maxChildren, 2048)), dim3(RLM_NT), 0, s, w,
                         lv);
    }
    {
      TraceScope ts("rlm_select", l, s);
      select_level<KT>(w, lv, src, pl.maxChildren, pl.maxBlk, pl.maxS[l], s);
    }
    {
      TraceScope ts("rlm_pieces", l, s);
      // wide groups (up to 65,536 sequences at the first level) scan with
      // 1024 threads per part
      if (pl.maxS[l] > 4096)
        hipLaunchKernelGGL(k_rlm_pieces<1024>, dim3(grid_cap(pl.maxChildren, 2048)), dim3(1024), 0,
                           s, w, lv);
      else
        hipLaunchKernelGGL(k_rlm_pieces<RLM_NT>, dim3(grid_cap(pl.maxChildren, 2048)),
                           dim3(RLM_NT), 0, s, w, lv);
    }
    {
      TraceScope ts("rlm_merge", l, s);
      hipLaunchKernelGGL(k_rlm_merge<KT>, dim3(grid_cap(pl.maxSlice, 2048)), dim3(RLM_MT), ldsM,
                         s, w, lv, src, dst);
    }
    // the parts become the next level's groups
    std::swap(w.groups, w.children);
    hipLaunchKernelGGL(k_rlm_next, dim3(1), dim3(64), 0, s, w);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch failed: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  return fold_device_errors(&w.hdr->overflow, s);
}

ams_status rlm_run(const RPlan &pl, const void *in, void *out, void *ws, hipStream_t s) {
  if (pl.kt == KT_U64) return rlm_typed<KT_U64>(pl, in, out, ws, s);
  if (pl.kt == KT_U32) return rlm_typed<KT_U32>(pl, in, out, ws, s);
  return rlm_typed<KT_F32>(pl, in, out, ws, s);
}

// The last cut row of a step selection: every run's length.
__global__ void k_rlm_last_row(uint32_t *cuts, uint32_t parts, uint32_t S, uint64_t n, uint32_t T) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) {
    const uint64_t a = (uint64_t)i * T;
    cuts[(size_t)parts * S + i] = (uint32_t)(n - a < T ? n - a : T);
  }
}

template <int KT>
ams_status step_select_typed(const void *d_runs, uint64_t n, uint32_t T, uint32_t parts,
                             uint64_t seed, uint32_t *d_cuts, hipStream_t s) {
  const uint64_t S = (n + T - 1) / T;
  RPlan pl;
  memset(&pl, 0, sizeof pl);
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o = al256(o + b);
    return at;
  };
  const uint64_t cut = S * parts, blk = (uint64_t)parts * ((S + RLM_NT - 1) / RLM_NT);
  pl.o_hdr = take(sizeof(RHdr));
  pl.o_g0 = take(sizeof(RGroup));
  pl.o_g1 = take(parts * sizeof(RGroup));
  pl.o_sel = take(parts * sizeof(RSel));
  pl.o_lo = take(cut * 4);
  pl.o_hi = take(cut * 4);
  pl.o_cc = take(RLM_M * cut * 4);
  pl.o_bl = take((RLM_M + 1) * blk * 4);
  pl.o_bown = take(blk * 4);
  pl.o_sown = take((S + parts) * 4);
  pl.o_scr = take(5 * 2 * 4);  // one group
  void *ws = nullptr;
  if (hipMallocAsync(&ws, o, s) != hipSuccess) {
    set_error("hipMallocAsync(%zu) failed", o);
    return AMS_ENOMEM;
  }
  char *base = (char *)ws;
  RWs w;
  memset(&w, 0, sizeof w);
  w.hdr = (RHdr *)(base + pl.o_hdr);
  w.groups = (RGroup *)(base + pl.o_g0);
  w.children = (RGroup *)(base + pl.o_g1);
  w.sel = (RSel *)(base + pl.o_sel);
  w.lo = (uint32_t *)(base + pl.o_lo);
  w.hi = (uint32_t *)(base + pl.o_hi);
  w.cc = (uint32_t *)(base + pl.o_cc);
  w.cut = d_cuts;  // rows j = 0..parts-1 land in the caller's table directly
  w.bl = (uint32_t *)(base + pl.o_bl);
  w.blkOwner = (uint32_t *)(base + pl.o_bown);
  w.sliceOwner = (uint32_t *)(base + pl.o_sown);
  w.capCut = (uint32_t)cut;
  w.scratch = (uint32_t *)(base + pl.o_scr);
  RLev lv;
  memset(&lv, 0, sizeof lv);
  lv.T = T;
  lv.r = parts;
  lv.force = parts;
  lv.itmax = sel_steps(n);
  lv.capChildren = parts;
  lv.capCut = (uint32_t)cut;
  lv.capBlk = (uint32_t)blk;
  lv.capQ = (uint32_t)(cut + parts);
  lv.capSlice = (uint32_t)(S + parts);
  lv.seed = seed ? seed : 14106754ull;
  hipLaunchKernelGGL(k_rlm_root, dim3(1), dim3(64), 0, s, w, (uint32_t)n);
  hipLaunchKernelGGL(k_rlm_children, dim3(1), dim3(1024), 0, s, w, lv);
  hipLaunchKernelGGL(k_rlm_owners, dim3(grid_cap(parts, 2048)), dim3(RLM_NT), 0, s, w, lv);
  select_level<KT>(w, lv, d_runs, parts, (uint32_t)blk, S, s);
  hipLaunchKernelGGL(k_rlm_last_row, dim3(grid_cap((S + 255) / 256, 1024)), dim3(256), 0, s,
                     d_cuts, parts, (uint32_t)S, n, T);
  uint32_t bits = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&bits, w.hdr, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFreeAsync(ws, s);
  if (e != hipSuccess) {
    set_error("step_multiselect: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  if (bits) {
    set_error("the device raised error bits 0x%x", bits);
    return AMS_EDEVICE;
  }
  return AMS_OK;
}

}  // namespace

}  // namespace ams

using namespace ams;

extern "C" {

size_t ams_rlm_workspace_bytes(ams_key_t t, size_t n, const ams_rlm_params *p) {
  RPlan pl;
  if (make_rlm_plan(pl, t, n, p)) return 0;
  return pl.bytes;
}

ams_status ams_rlm_sort_keys(ams_key_t t, const void *d_in, void *d_out, size_t n, void *d_ws,
                             size_t ws_bytes, void *stream, const ams_rlm_params *p) {
  set_error("");
  RPlan pl;
  ams_status st = make_rlm_plan(pl, t, n, p);
  if (st) return st;
  if (n == 0) return AMS_OK;
  if (!d_in || !d_out) {
    set_error("NULL device pointer with n = %zu", n);
    return AMS_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  void *ws = d_ws;
  bool owned = false;
  if (ws) {
    if (ws_bytes < pl.bytes) {
      set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, pl.bytes);
      return AMS_ENOMEM;
    }
  } else {
    if (hipMallocAsync(&ws, pl.bytes, s) != hipSuccess) {
      set_error("hipMallocAsync(%zu) failed", pl.bytes);
      return AMS_ENOMEM;
    }
    owned = true;
  }
  st = rlm_run(pl, d_in, d_out, ws, s);
  if (!st && (pl.flags & AMS_FLAG_CHECK)) {
    uint32_t bits = 0;
    hipError_t e = hipMemcpyAsync(&bits, ws, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = AMS_EHIP;
    else if (bits) {
      set_error("the device raised error bits 0x%x", bits);
      st = AMS_EDEVICE;
    }
  }
  if (owned) (void)hipFreeAsync(ws, s);
  return st;
}

ams_status ams_step_multiselect(ams_key_t t, const void *d_runs, size_t n, uint32_t run_keys,
                                uint32_t parts, uint64_t seed, uint32_t *d_cuts, void *stream) {
  set_error("");
  if ((t != AMS_U32 && t != AMS_U64 && t != AMS_F32) || !d_runs || !d_cuts || n == 0 ||
      run_keys == 0 || parts < 1 || parts > 1024 || n > AMS_MAX_SEGMENT ||
      (uint64_t)parts > n) {
    set_error("bad arguments");
    return AMS_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (t == AMS_U64) return step_select_typed<KT_U64>(d_runs, n, run_keys, parts, seed, d_cuts, s);
  if (t == AMS_U32) return step_select_typed<KT_U32>(d_runs, n, run_keys, parts, seed, d_cuts, s);
  return step_select_typed<KT_F32>(d_runs, n, run_keys, parts, seed, d_cuts, s);
}

}  // extern "C"
