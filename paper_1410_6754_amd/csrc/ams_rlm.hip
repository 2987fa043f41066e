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

// One selection: the boundary in front of a part (j >= 1).
struct RSel {
  uint64_t pivot;    // ord value of the pivot
  uint32_t q, t;     // its sequence and position
  uint32_t krem;     // rank still sought inside the windows (1-based)
  uint32_t total;    // keys in the windows
  uint32_t dir;      // decision to apply at the next step: 0 none, 1 left, 2 right
  uint32_t done;     // 1: the windows' upper ends (after dir) are the cut
  uint32_t arrive;   // blocks of the current step that have finished
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
  uint32_t *lo, *hi, *cc, *cut, *bl, *br, *q;
  uint32_t *scratch;  // per group: part counts (exscan space)
};

AMS_DEV void rlm_error(const RWs &w, uint32_t bits) { atomicOr(&w.hdr->overflow, bits); }

// A selection's state as another block of this launch may have left it.
AMS_DEV RSel load_sel(const RSel *p) {
  const volatile RSel *v = p;
  RSel s;
  s.pivot = v->pivot;
  s.q = v->q;
  s.t = v->t;
  s.krem = v->krem;
  s.total = v->total;
  s.dir = v->dir;
  s.done = v->done;
  s.arrive = v->arrive;
  s.iter = v->iter;
  return s;
}

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
// few ten thousand groups).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_rlm_children(RWs w, RLev lv) {
  __shared__ uint32_t tmp[1024 / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t G = w.hdr->nGroups;
  uint32_t *pc = w.scratch;  // G + 1 entries
  for (uint32_t g = tid; g < G; g += 1024)
    pc[g] = lv.force ? lv.force : level_parts(w.groups[g].size, lv.r, lv.T);
  __syncthreads();
  const uint32_t nc = block_exscan<1024>(pc, G, tmp);
  if (nc > lv.capChildren) {
    if (tid == 0) {
      rlm_error(w, AMS_DEVERR_GROUPS);
      w.hdr->nChildren = 0;
    }
    return;
  }
  // children, with their table sizes in the base fields (scanned below)
  for (uint32_t g = tid; g < G; g += 1024) {
    const RGroup P = w.groups[g];
    const uint32_t parts = lv.force ? lv.force : level_parts(P.size, lv.r, lv.T);
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
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
      c.cutBase = S;
      c.blkBase = (S + RLM_NT - 1) / RLM_NT;
      c.qBase = S + 1;
      c.sliceBase = (c.size + lv.T - 1) / lv.T;
      c.pad[0] = c.pad[1] = 0;
      w.children[pc[g] + j] = c;
    }
  }
  __syncthreads();
  // bases by four exclusive scans over the children
  uint32_t *cb = (uint32_t *)w.children;
  const uint32_t stride = sizeof(RGroup) / 4;
  const uint32_t fields[4] = {offsetof(RGroup, cutBase) / 4, offsetof(RGroup, blkBase) / 4,
                              offsetof(RGroup, qBase) / 4, offsetof(RGroup, sliceBase) / 4};
  for (int f = 0; f < 4; ++f) {
    for (uint32_t c = tid; c < nc; c += 1024) pc[c] = cb[(size_t)c * stride + fields[f]];
    __syncthreads();
    const uint32_t tot = block_exscan<1024>(pc, nc, tmp);
    for (uint32_t c = tid; c < nc; c += 1024) cb[(size_t)c * stride + fields[f]] = pc[c];
    if (tid == 0) w.hdr->cnt[f] = tot;
    __syncthreads();
  }
  const uint32_t caps[4] = {lv.capCut, lv.capBlk, lv.capQ, lv.capSlice};
  bool over = false;
  for (int f = 0; f < 4; ++f) over = over || w.hdr->cnt[f] > caps[f];
  if (tid == 0) {
    if (over) rlm_error(w, AMS_DEVERR_TILES);
    w.hdr->nChildren = over ? 0 : nc;
  }
}

// Windows of every selection: the whole of every sequence; the first pivot
// drawn uniformly from the parent group.
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
      w.cc[C.cutBase + i] = 0;
    }
    if (threadIdx.x == 0) {
      RSel s;
      memset(&s, 0, sizeof s);
      s.krem = C.rank;
      s.total = P.size;
      s.done = C.j == 0 ? 1u : 0u;  // the first part starts at rank 0: nothing to select
      if (!s.done) {
        const uint64_t st = stream_state(lv.seed, RLM_STREAM + lv.level, c, 0);
        const uint32_t u = draw_pos(st, 0, P.size);
        s.q = u / lv.T;
        s.t = u - s.q * lv.T;
        s.pivot = (uint64_t)Key<KT>::enc(src[P.start + u]);
      }
      w.sel[c] = s;
    }
  }
}

// Elements of x[lo, hi) (raw keys, sorted by their ord value) that precede
// the pivot (ord value v, sequence q, position t) in the order (key,
// sequence, position), for sequence i.
template <int KT>
AMS_DEV uint32_t count_before(const GMem<typename Key<KT>::T> *x, uint32_t lo, uint32_t hi,
                              typename Key<KT>::T v, uint32_t i, uint32_t q, uint32_t t) {
  typedef typename Key<KT>::T K;
  if (i == q) return t;
  const bool le = i < q;  // earlier sequences: equal keys come first
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const K y = Key<KT>::enc(x[mid]);
    const bool before = le ? (y <= v) : (y < v);
    if (before) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One step of every unfinished selection; each item is (selection, block of
// RLM_NT sequences).  The last block of a selection to finish its step
// decides the side and draws the next pivot.  A selection with a single
// block runs its steps back to back inside the launch (at most lv.itmax).
template <int KT>
__global__ void __launch_bounds__(RLM_NT) k_rlm_select(RWs w, RLev lv, const void *src_) {
  typedef typename Key<KT>::T K;
  const GMem<K> *src = (const GMem<K> *)src_;
  __shared__ uint32_t red[2 * RLM_NT / 64];
  __shared__ uint32_t sh[4];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t nc = w.hdr->nChildren, nb = w.hdr->cnt[1];
  for (uint32_t item = blockIdx.x; item < nb; item += gridDim.x) {
    // owner: the last child whose first block is <= item
    uint32_t lo_c = 0, hi_c = nc;
    while (hi_c - lo_c > 1) {
      const uint32_t mid = (lo_c + hi_c) >> 1;
      if (w.children[mid].blkBase <= item) lo_c = mid; else hi_c = mid;
    }
    const uint32_t c = lo_c;
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    const uint32_t nblk = (S + RLM_NT - 1) / RLM_NT;
    const uint32_t b = item - C.blkBase;
    const uint32_t rounds = nblk == 1 ? lv.itmax : 1u;
    for (uint32_t round = 0; round < rounds; ++round) {
      const RSel s = load_sel(w.sel + c);
      if (s.done) break;
      const uint32_t i = b * RLM_NT + tid;
      uint32_t L = 0, R = 0;
      if (i < S) {
        const uint32_t e = C.cutBase + i;
        uint32_t lo = w.lo[e], hi = w.hi[e];
        const uint32_t prev = w.cc[e];
        if (s.dir == 1) hi = prev;
        else if (s.dir == 2) lo = prev;
        const uint32_t cnt = count_before<KT>(src + P.start + (size_t)i * lv.T, lo, hi,
                                              (K)s.pivot, i, s.q, s.t);
        w.lo[e] = lo;
        w.hi[e] = hi;
        w.cc[e] = cnt;
        L = cnt - lo;
        R = hi - cnt;
      }
      L = wave_sum(L);
      R = wave_sum(R);
      if (lane == 0) {
        red[wave] = L;
        red[RLM_NT / 64 + wave] = R;
      }
      __syncthreads();
      if (tid == 0) {
        uint32_t bl = 0, br = 0;
        for (uint32_t q = 0; q < RLM_NT / 64; ++q) {
          bl += red[q];
          br += red[RLM_NT / 64 + q];
        }
        w.bl[C.blkBase + b] = bl;
        w.br[C.blkBase + b] = br;
        __threadfence();
        const uint32_t old = atomicAdd(&w.sel[c].arrive, 1u);
        sh[0] = old + 1 == nblk ? 1u : 0u;
      }
      __syncthreads();
      if (!sh[0]) break;  // another block finishes this step
      __threadfence();
      // --- last block of the step: decide, then draw the next pivot ------
      uint32_t left = 0;
      for (uint32_t q = tid; q < nblk; q += RLM_NT) left += ((volatile uint32_t *)w.bl)[C.blkBase + q];
      left = wave_sum(left);
      __syncthreads();
      if (lane == 0) red[wave] = left;
      __syncthreads();
      left = 0;
      for (uint32_t q = 0; q < RLM_NT / 64; ++q) left += red[q];
      uint32_t krem = s.krem, total, dir;
      if (left >= krem) {
        dir = 1;
        total = left;
      } else {
        dir = 2;
        krem -= left;
        total = s.total - left;
      }
      RSel ns = s;
      ns.dir = dir;
      ns.krem = krem;
      ns.total = total;
      ns.arrive = 0;
      ns.iter = s.iter + 1;
      if (total == krem) {
        ns.done = 1;
      } else {
        // u-th key (0-based) of the new windows, in sequence order
        const uint64_t st = stream_state(lv.seed, RLM_STREAM + lv.level, c, ns.iter);
        uint32_t u = draw_pos(st, 0, total);
        const uint32_t *part = dir == 1 ? w.bl : w.br;
        // block holding it: a sequential walk over the block totals (at
        // most a few hundred)
        uint32_t bsel = 0;
        if (tid == 0) {
          uint32_t acc = 0;
          for (bsel = 0; bsel < nblk; ++bsel) {
            const uint32_t v = ((volatile uint32_t *)part)[C.blkBase + bsel];
            if (u < acc + v) break;
            acc += v;
          }
          sh[1] = bsel < nblk ? bsel : nblk - 1;
          sh[2] = u - acc;
        }
        __syncthreads();
        bsel = sh[1];
        u = sh[2];
        // sequence holding it inside that block
        const uint32_t i = bsel * RLM_NT + tid;
        uint32_t wlo = 0, wsz = 0;
        if (i < S) {
          const uint32_t e = C.cutBase + i;
          const uint32_t lo = ((volatile uint32_t *)w.lo)[e], hi = ((volatile uint32_t *)w.hi)[e];
          const uint32_t cc = ((volatile uint32_t *)w.cc)[e];
          wlo = dir == 1 ? lo : cc;
          wsz = dir == 1 ? cc - lo : hi - cc;
        }
        const uint32_t incl = wave_incl_scan(wsz);
        if (lane == 63) red[wave] = incl;
        __syncthreads();
        uint32_t off = 0;
        for (uint32_t q = 0; q < wave; ++q) off += red[q];
        const uint32_t first = off + incl - wsz;
        if (tid == 0) sh[3] = 0xFFFFFFFFu;
        __syncthreads();
        if (wsz && u >= first && u < first + wsz) {
          sh[3] = i;
          sh[1] = wlo + (u - first);
        }
        __syncthreads();
        if (sh[3] == 0xFFFFFFFFu) {  // cannot happen: the partials cover u
          ns.done = 1;
          if (tid == 0) rlm_error(w, AMS_DEVERR_RANGE);
        } else {
          ns.q = sh[3];
          ns.t = sh[1];
          ns.pivot = (uint64_t)Key<KT>::enc(src[P.start + (size_t)ns.q * lv.T + ns.t]);
        }
      }
      if (tid == 0) {
        w.sel[c] = ns;
        __threadfence();
      }
      __syncthreads();
    }
  }
}

// Cut positions: the windows' upper ends once the last decision is applied.
__global__ void __launch_bounds__(RLM_NT) k_rlm_cut(RWs w, RLev lv) {
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    const RSel s = w.sel[c];
    if (threadIdx.x == 0 && !s.done) rlm_error(w, AMS_DEVERR_RANGE);
    for (uint32_t i = threadIdx.x; i < S; i += RLM_NT) {
      const uint32_t e = C.cutBase + i;
      uint32_t v;
      if (C.j == 0) v = 0;
      else v = s.dir == 1 ? w.cc[e] : w.hi[e];
      w.cut[e] = v;
    }
  }
}

// Piece offsets of every part: Q[i] = keys of the part in sequences < i.
__global__ void __launch_bounds__(RLM_NT) k_rlm_pieces(RWs w, RLev lv) {
  __shared__ uint32_t tmp[RLM_NT / 64];
  const uint32_t nc = w.hdr->nChildren;
  for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const RGroup C = w.children[c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + lv.T - 1) / lv.T;
    uint32_t *Q = w.q + C.qBase;
    for (uint32_t i = threadIdx.x; i < S; i += RLM_NT) {
      const uint32_t a = w.cut[C.cutBase + i];
      // the next part's cut row follows this one (same parent, same S)
      const uint32_t b = C.last ? seq_len(P, i, lv.T) : w.cut[C.cutBase + S + i];
      Q[i] = b >= a ? b - a : 0u;
    }
    __syncthreads();
    const uint32_t tot = block_exscan<RLM_NT>(Q, S, tmp);
    if (threadIdx.x == 0) {
      Q[S] = tot;
      if (tot != C.size) rlm_error(w, AMS_DEVERR_RANGE);
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

template <int KT>
__global__ void __launch_bounds__(RLM_MT) k_rlm_merge(RWs w, RLev lv, const void *src_,
                                                      void *dst_) {
  typedef typename Key<KT>::T K;
  const GMem<K> *src = (const GMem<K> *)src_;
  GMem<K> *dst = (GMem<K> *)dst_;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t T = lv.T;
  K *bufA = (K *)smem_raw;
  K *bufB = bufA + T;
  uint32_t *seg = (uint32_t *)(bufB + T);  // T + 1 entries
  __shared__ uint32_t tmp[RLM_MT / 64];
  __shared__ uint32_t shv[4];
  const uint32_t tid = threadIdx.x;
  const uint32_t nc = w.hdr->nChildren, ns = w.hdr->cnt[3];
  for (uint32_t item = blockIdx.x; item < ns; item += gridDim.x) {
    uint32_t lo_c = 0, hi_c = nc;
    while (hi_c - lo_c > 1) {
      const uint32_t mid = (lo_c + hi_c) >> 1;
      if (w.children[mid].sliceBase <= item) lo_c = mid; else hi_c = mid;
    }
    const RGroup C = w.children[lo_c];
    const RGroup P = w.groups[C.parent];
    const uint32_t S = (P.size + T - 1) / T;
    const uint32_t *Q = w.q + C.qBase;
    const uint32_t *cut = w.cut + C.cutBase;
    if (Q[S] != C.size) continue;  // the piece offsets raised an error already
    const uint32_t a = (item - C.sliceBase) * T;
    const uint32_t len = C.size - a < T ? C.size - a : T;
    // pieces overlapping [a, a + len): i0 = last i with Q[i] <= a,
    // i1 = first i with Q[i] >= a + len
    if (tid == 0) {
      uint32_t l = 0, h = S + 1;
      while (h - l > 1) {
        const uint32_t m = (l + h) >> 1;
        if (Q[m] <= a) l = m; else h = m;
      }
      uint32_t l2 = l, h2 = S;
      while (l2 < h2) {
        const uint32_t m = (l2 + h2) >> 1;
        if (Q[m] >= a + len) h2 = m; else l2 = m + 1;
      }
      shv[0] = l;
      shv[1] = l2 > l ? l2 : l + 1;
    }
    __syncthreads();
    const uint32_t i0 = shv[0], i1 = shv[1];
    const uint32_t np = i1 - i0;
    const bool cached = np <= T;
    if (cached)
      for (uint32_t k = tid; k <= np; k += RLM_MT) seg[k] = Q[i0 + k];
    __syncthreads();
    // gather: element x of the slice comes from the piece holding a + x
    uint32_t *flag = (uint32_t *)bufB;
    for (uint32_t x = tid; x < len; x += RLM_MT) {
      const uint32_t g = a + x;
      const uint32_t k = cached ? upper_le<K>(seg, np, g) : upper_le<K>(Q + i0, np, g);
      const uint32_t i = i0 + k;
      const uint32_t qi = cached ? seg[k] : Q[i];
      const uint32_t pos = cut[i] + (g - qi);
      if (pos < seq_len(P, i, T)) {
        bufA[x] = Key<KT>::enc(src[P.start + (size_t)i * T + pos]);
      } else {  // cannot happen when the cuts and offsets agree
        bufA[x] = 0;
        rlm_error(w, AMS_DEVERR_RANGE);
      }
      flag[x] = (x == 0 || qi == g) ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t nseg = block_exscan<RLM_MT>(flag, len, tmp);
    // flag[] now holds ranks; a start is where the rank steps
    for (uint32_t x = tid; x < len; x += RLM_MT) {
      const uint32_t rk = flag[x];
      const uint32_t nx = x + 1 < len ? flag[x + 1] : nseg;
      if (nx != rk) seg[rk] = x;
    }
    if (tid == 0) seg[nseg] = len;
    __syncthreads();
    // pairwise merge rounds: segments (2m, 2m+1) -> m, A first on ties
    uint32_t nsg = nseg;
    K *in = bufA, *out = bufB;
    const uint32_t per = (len + RLM_MT - 1) / RLM_MT;
    while (nsg > 1) {
      const uint32_t x0 = tid * per < len ? tid * per : len;
      const uint32_t x1 = x0 + per < len ? x0 + per : len;
      uint32_t x = x0;
      while (x < x1) {
        // pair m holding output x: segments 2m, 2m+1
        uint32_t l = 0, h = (nsg + 1) / 2;  // pairs
        while (h - l > 1) {
          const uint32_t m = (l + h) >> 1;
          if (seg[2 * m] <= x) l = m; else h = m;
        }
        const uint32_t m = l;
        const uint32_t as = seg[2 * m];
        const uint32_t ae = 2 * m + 1 <= nsg ? seg[2 * m + 1] : len;
        const uint32_t be = 2 * m + 2 <= nsg ? seg[2 * m + 2] : ae;
        const uint32_t na = ae - as, nb = be - ae;
        const K *A = in + as, *B = in + ae;
        const uint32_t rho = x - as;
        uint32_t clo = rho > nb ? rho - nb : 0, chi = rho < na ? rho : na;
        while (clo < chi) {
          const uint32_t mid = (clo + chi) >> 1;
          if (A[mid] <= B[rho - mid - 1]) clo = mid + 1; else chi = mid;
        }
        uint32_t ia = clo, ib = rho - clo;
        const uint32_t stop = x1 < be ? x1 : be;
        for (; x < stop; ++x) {
          const bool takeA = ib >= nb || (ia < na && A[ia] <= B[ib]);
          out[x] = takeA ? A[ia] : B[ib];
          ia += takeA ? 1u : 0u;
          ib += takeA ? 0u : 1u;
        }
      }
      __syncthreads();
      // segments of the next round: every other boundary
      const uint32_t nn = (nsg + 1) / 2;
      uint32_t v[8];
      uint32_t cntv = 0;
      for (uint32_t k = tid; k < nn && cntv < 8; k += RLM_MT) v[cntv++] = seg[2 * k];
      __syncthreads();
      cntv = 0;
      for (uint32_t k = tid; k < nn && cntv < 8; k += RLM_MT) seg[k] = v[cntv++];
      if (tid == 0) seg[nn] = len;
      __syncthreads();
      nsg = nn;
      K *t = in;
      in = out;
      out = t;
    }
    // keys leave LDS as raw bits at every level (the next level encodes
    // them again on load, as it does the tile sort's output)
    for (uint32_t x = tid; x < len; x += RLM_MT) dst[C.start + a + x] = Key<KT>::dec(in[x]);
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
  bool multiblock[RLM_MAXLEV];
  size_t o_hdr, o_tmp, o_tile, o_g0, o_g1, o_sel, o_lo, o_hi, o_cc, o_cut, o_bl, o_br, o_q,
      o_scr, bytes;
};

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
    pl.multiblock[L] = maxS > RLM_NT;
    pl.itmax[L] = 3 * (64 - __builtin_clzll(mx)) + 16;
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
  pl.o_cc = take((size_t)pl.maxCut * 4);
  pl.o_cut = take((size_t)pl.maxCut * 4);
  pl.o_bl = take((size_t)pl.maxBlk * 4);
  pl.o_br = take((size_t)pl.maxBlk * 4);
  pl.o_q = take((size_t)pl.maxQ * 4);
  pl.o_scr = take((ng + 1) * 4);
  pl.bytes = o;
  return AMS_OK;
}

uint32_t grid_cap(uint64_t items, uint32_t cap) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(items, cap));
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
  w.br = (uint32_t *)(base + pl.o_br);
  w.q = (uint32_t *)(base + pl.o_q);
  w.scratch = (uint32_t *)(base + pl.o_scr);
  void *tmp = base + pl.o_tmp;
  // buffer of level l's output: the last level writes `out`
  auto buf = [&](uint32_t l) -> void * { return ((pl.L - l) & 1u) ? tmp : out; };
  hipLaunchKernelGGL(k_rlm_root, dim3(1), dim3(64), 0, s, w, (uint32_t)pl.n);
  ams_status st = run_tile_sort(KT, false, in, nullptr, buf(0), nullptr, pl.n, pl.T,
                                base + pl.o_tile, s);
  if (st) return st;
  const size_t ldsM = 2 * (size_t)pl.T * sizeof(K) + ((size_t)pl.T + 1) * 4;
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
    }
    {
      TraceScope ts("rlm_select", l, s);
      hipLaunchKernelGGL(k_rlm_sel_init<KT>, dim3(grid_cap(pl.maxChildren, 2048)), dim3(RLM_NT), 0,
                         s, w, lv, src);
      const uint32_t steps = pl.multiblock[l] ? pl.itmax[l] : 1u;
      for (uint32_t it = 0; it < steps; ++it)
        hipLaunchKernelGGL(k_rlm_select<KT>, dim3(grid_cap(pl.maxBlk, 4096)), dim3(RLM_NT), 0, s,
                           w, lv, src);
      hipLaunchKernelGGL(k_rlm_cut, dim3(grid_cap(pl.maxChildren, 2048)), dim3(RLM_NT), 0, s, w,
                         lv);
    }
    {
      TraceScope ts("rlm_pieces", l, s);
      hipLaunchKernelGGL(k_rlm_pieces, dim3(grid_cap(pl.maxChildren, 2048)), dim3(RLM_NT), 0, s,
                         w, lv);
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
  pl.o_cc = take(cut * 4);
  pl.o_bl = take(blk * 4);
  pl.o_br = take(blk * 4);
  pl.o_scr = take((parts + 2) * 4);
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
  w.br = (uint32_t *)(base + pl.o_br);
  w.scratch = (uint32_t *)(base + pl.o_scr);
  RLev lv;
  memset(&lv, 0, sizeof lv);
  lv.T = T;
  lv.r = parts;
  lv.force = parts;
  lv.itmax = 3 * (64 - __builtin_clzll(n)) + 16;
  lv.capChildren = parts;
  lv.capCut = (uint32_t)cut;
  lv.capBlk = (uint32_t)blk;
  lv.capQ = (uint32_t)(cut + parts);
  lv.capSlice = (uint32_t)(S + parts);
  lv.seed = seed ? seed : 14106754ull;
  hipLaunchKernelGGL(k_rlm_root, dim3(1), dim3(64), 0, s, w, (uint32_t)n);
  hipLaunchKernelGGL(k_rlm_children, dim3(1), dim3(1024), 0, s, w, lv);
  hipLaunchKernelGGL(k_rlm_sel_init<KT>, dim3(grid_cap(parts, 2048)), dim3(RLM_NT), 0, s, w, lv,
                     d_runs);
  const uint32_t steps = S > RLM_NT ? lv.itmax : 1u;
  for (uint32_t it = 0; it < steps; ++it)
    hipLaunchKernelGGL(k_rlm_select<KT>, dim3(grid_cap(blk, 4096)), dim3(RLM_NT), 0, s, w, lv,
                       d_runs);
  hipLaunchKernelGGL(k_rlm_cut, dim3(grid_cap(parts, 2048)), dim3(RLM_NT), 0, s, w, lv);
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
