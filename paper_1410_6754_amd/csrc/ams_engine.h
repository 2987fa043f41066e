// Host-side view of the sort engine: planning and launching the level
// kernels for a set of independent roots.  Shared by the C ABI entry points
// and the serving loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "ams.h"
#include "ams_device.h"

namespace ams {

constexpr uint32_t MAXLEV = 4;         // partition levels at most
constexpr uint32_t CMAX = 8192;        // keys one base-case workgroup sorts in LDS
constexpr uint32_t FIN_THREADS = 512;  // base-case workgroup size
constexpr uint32_t FMAX = 256;         // largest in-LDS fan-out of the base case
// bytes of the fixed per-device workspace of ams_sort_keys_noalloc
constexpr size_t NOALLOC_SCRATCH_BYTES = AMS_NOALLOC_SCRATCH_BYTES;
constexpr uint32_t MAX_DEVICES = 64;
// internal plan flag: the caller runs only level steps, never the base case
constexpr uint32_t FLAG_NO_BASE_CASE = 1u << 31;

struct LevelShape {
  uint32_t rmax;     // groups per subproblem (paper's r)
  uint32_t b;        // overpartitioning factor
  uint32_t a;        // oversampling factor
  uint32_t mmax;     // largest bucket count at this level
  uint32_t Smax;     // largest sample
  uint32_t TC;       // keys per tile
  uint32_t TB;       // tiles per tile block
  uint32_t HS;       // histogram stride (2 * mmax)
  uint32_t CH;       // child table stride (3 * rmax)
  uint32_t rankG;    // sample blocks ranked per workgroup item
  uint32_t P;        // active subproblems (upper bound)
  uint32_t tiles;    // tiles (upper bound)
  uint32_t blocks;   // tile blocks (upper bound)
  uint32_t sblocks;  // sample blocks of 256 (upper bound)
};

struct Plan {
  int kt;
  bool pay;
  uint32_t kw;       // key bytes
  uint64_t ntotal;   // elements over all roots
  uint32_t nroots;
  uint64_t maxroot;
  uint32_t nbig;     // roots larger than C
  uint32_t C;        // leaf capacity
  uint32_t L;        // partition levels
  uint32_t cutoff;   // base-case bucket cutoff
  uint64_t seed;
  uint32_t flags;
  LevelShape lev[MAXLEV];
  uint32_t capLeaf;
  uint32_t capBig;  // oversized-leaf list
  // workspace layout (byte offsets)
  size_t o_tmpK, o_tmpV, o_roots, o_ctr, o_act[MAXLEV + 1], o_leaves, o_big, o_sink, o_tileStart, o_blkStart,
      o_sampStart, o_samp, o_spl, o_tree, o_eq, o_hist, o_blkHist, o_tileOff,
      o_i2c, o_cfirst, o_cstart, o_cdst, o_nch, o_dbg, o_totals, o_strata;
  uint32_t capActMax, capTile, capBlk, capSBlk, maxHS, maxCH, maxM, maxS;
  size_t bytes;
};

// Build the plan for roots of the given sizes (sizes == NULL: one root of n).
ams_status make_plan(Plan &pl, int kt, bool pay, const uint64_t *sizes, uint32_t nroots,
                     uint64_t n_single, const ams_params *p);

// Enqueue the whole sort.  Roots come from one of: a single root (R), a batch
// of contiguous segments (base pointers + device offsets), or a root table
// already in the workspace (prebuilt).
struct RootSource {
  int mode;  // 0 single, 1 offsets, 2 prebuilt
  Root single;
  const char *kin;
  const uint32_t *vin;
  char *kout;
  uint32_t *vout;
  const uint64_t *d_offsets;
};

ams_status run_plan(const Plan &pl, void *ws, const RootSource &src, hipStream_t s,
                    uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                    const void *given_splitters);

void set_error(const char *fmt, ...);

// Kernel tracing: when ams_trace_start is on for the calling thread, a
// TraceScope brackets the launches made in its lifetime with a pair of
// events on the stream (name, or name.L<level>).
struct TraceRec {
  char name[32];
  hipEvent_t e0, e1;
};
struct TraceScope {
  TraceRec rec;
  bool on;
  hipStream_t s;
  TraceScope(const char *name, uint32_t level, hipStream_t st);
  ~TraceScope();
};

// RLM-sort's local sort: tiles of T keys of one array sorted in LDS by the
// base case (ams_engine.hip); workspace of tile_sort_ws_bytes(n, T).
size_t tile_sort_ws_bytes(uint64_t n, uint32_t T);
ams_status run_tile_sort(int kt, bool pay, const void *in, const uint32_t *vin, void *out,
                         uint32_t *vout, uint64_t n, uint32_t T, void *ws, hipStream_t s);
uint32_t base_case_capacity(uint32_t kw, bool pay);

// Parameters the autotuner chose for this shape class, if any (ams_tune.hip).
bool tuned_lookup(int kt, bool pay, uint64_t total, uint64_t mx, uint64_t nroots,
                  ams_params *out);

}  // namespace ams
