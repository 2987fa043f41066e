// Autotuner: picks the number of levels, the group count k, the
// overpartitioning factor b, the base-case cutoff and the tile size for a
// sort of a given shape by timing candidates on the device, and remembers the
// choice for the process.  Every candidate sorts the same input; a candidate
// whose output differs from the first one's is rejected (the sorted output is
// unique, so this never happens unless something is broken).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ams.h"
#include "ams_engine.h"

namespace ams {

ams_status run_plan_ex(const Plan &pl, void *ws, const RootSource &src, hipStream_t s,
                       uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                       const void *given_splitters, bool shrink_last);

namespace {

// Shape class: key type, payload, floor(log2) of the total, of the largest
// segment and of the segment count.
typedef std::tuple<int, int, int, int, int> ShapeKey;

int flog2(uint64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    ++l;
  }
  return l;
}

ShapeKey shape_key(int kt, bool pay, uint64_t total, uint64_t mx, uint64_t nroots) {
  return ShapeKey(kt, pay ? 1 : 0, flog2(total), flog2(mx), flog2(nroots));
}

std::mutex g_mu;
std::map<ShapeKey, ams_params> g_tuned;

__global__ void k_count_diff(const uint32_t *a, const uint32_t *b, size_t nw, uint32_t *diff) {
  uint32_t local = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (size_t)gridDim.x * blockDim.x)
    local += a[i] != b[i] ? 1u : 0u;
  if (local) atomicAdd(diff, local);
}

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ams_status ensure(size_t need) {
    if (need <= bytes) return AMS_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, need ? need : 1) != hipSuccess) {
      set_error("autotune: hipMalloc(%zu) failed", need);
      return AMS_ENOMEM;
    }
    bytes = need;
    return AMS_OK;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

bool tuned_lookup(int kt, bool pay, uint64_t total, uint64_t mx, uint64_t nroots,
                  ams_params *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_tuned.empty()) return false;
  auto it = g_tuned.find(shape_key(kt, pay, total, mx, nroots));
  if (it == g_tuned.end()) return false;
  *out = it->second;
  return true;
}

}  // namespace ams

using namespace ams;

extern "C" ams_status ams_autotune(ams_key_t t, const void *d_kin, const uint32_t *d_vin,
                                   const uint64_t *h_offsets, size_t num, void *stream,
                                   uint32_t max_trials, ams_params *best, double *best_ms) {
  set_error("");
  if ((t != AMS_U32 && t != AMS_U64 && t != AMS_F32) || !d_kin || !h_offsets || !best ||
      num == 0 || h_offsets[0] != 0) {
    set_error("autotune: bad arguments");
    return AMS_EINVAL;
  }
  if (num >= (1ull << 31)) {
    set_error("autotune: too many segments");
    return AMS_EUNSUPPORTED;
  }
  std::vector<uint64_t> sizes(num);
  uint64_t mx = 0;
  for (size_t i = 0; i < num; ++i) {
    if (h_offsets[i + 1] < h_offsets[i]) {
      set_error("autotune: h_offsets must be non-decreasing (index %zu)", i);
      return AMS_EINVAL;
    }
    sizes[i] = h_offsets[i + 1] - h_offsets[i];
    mx = std::max(mx, sizes[i]);
  }
  const uint64_t total = h_offsets[num];
  if (total == 0) {
    set_error("autotune: nothing to sort");
    return AMS_EINVAL;
  }
  const bool pay = d_vin != nullptr;
  const size_t kw = t == AMS_U64 ? 8 : 4;
  hipStream_t s = (hipStream_t)stream;
  if (max_trials == 0) max_trials = 24;
  {  // this shape's earlier choice must not steer the candidates
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned.erase(shape_key((int)t, pay, total, mx, num));
  }

  DevBuf out, ref, ws, offs, diff;
  const size_t kbytes = (size_t)total * kw, vbytes = pay ? (size_t)total * 4 : 0;
  ams_status st;
  if ((st = out.ensure(kbytes + vbytes)) || (st = ref.ensure(kbytes + vbytes)) ||
      (st = offs.ensure((num + 1) * 8)) || (st = diff.ensure(4)))
    return st;
  if (hipMemcpyAsync(offs.p, h_offsets, (num + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
    set_error("autotune: offset upload failed");
    return AMS_EHIP;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("autotune: hipEventCreate failed");
    return AMS_EHIP;
  }
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};

  bool have_ref = false;
  uint32_t trials = 0;
  // one candidate: plan, warm run, two timed runs (the faster counts), and
  // the output compared with the reference; < 0 when it cannot run
  auto evaluate = [&](const ams_params &p, double &ms) -> ams_status {
    Plan pl;
    ams_status r = make_plan(pl, (int)t, pay, sizes.data(), (uint32_t)num, 0, &p);
    if (r) return r;
    if ((r = ws.ensure(pl.bytes))) return r;
    char *dst = have_ref ? (char *)out.p : (char *)ref.p;
    RootSource rs;
    memset(&rs, 0, sizeof rs);
    rs.mode = 1;
    rs.kin = (const char *)d_kin;
    rs.vin = pay ? d_vin : nullptr;
    rs.kout = dst;
    rs.vout = pay ? (uint32_t *)(dst + kbytes) : nullptr;
    rs.d_offsets = (const uint64_t *)offs.p;
    float best_run = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) return AMS_EHIP;
      if ((r = run_plan_ex(pl, ws.p, rs, s, nullptr, nullptr, nullptr, nullptr, true))) return r;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        set_error("autotune: device error while timing a candidate");
        return AMS_EHIP;
      }
      float msr = 0;
      (void)hipEventElapsedTime(&msr, e0, e1);
      if (rep > 0) best_run = std::min(best_run, msr);
    }
    ++trials;
    if (have_ref) {
      uint32_t nd = 0;
      const size_t nw = (kbytes + vbytes) / 4;
      if (hipMemsetAsync(diff.p, 0, 4, s) != hipSuccess) return AMS_EHIP;
      hipLaunchKernelGGL(k_count_diff, dim3(2048), dim3(256), 0, s, (const uint32_t *)out.p,
                         (const uint32_t *)ref.p, nw, (uint32_t *)diff.p);
      if (hipMemcpyAsync(&nd, diff.p, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return AMS_EHIP;
      if (nd) {
        set_error("autotune: a candidate's output differs from the reference in %u words", nd);
        return AMS_EHIP;
      }
    }
    have_ref = true;
    ms = best_run;
    return AMS_OK;
  };

  // start from the built-in defaults, then improve one parameter at a time;
  // b stays 0 (the plan's own choice per level) until a value is tried
  ams_params cur;
  memset(&cur, 0, sizeof cur);
  cur.base_cutoff = 32;
  double cur_ms = 0;
  if ((st = evaluate(cur, cur_ms))) return st;
  {  // the levels, group count and tile size the plan picked by itself
    Plan pl;
    if (make_plan(pl, (int)t, pay, sizes.data(), (uint32_t)num, 0, &cur) == AMS_OK) {
      cur.levels = pl.L;
      cur.k = pl.L ? pl.lev[0].rmax : 256;
      cur.tile_keys = pl.L ? pl.lev[0].TC : 32768;
    }
  }
  const uint32_t Lauto = cur.levels;
  struct Dim {
    uint32_t ams_params::*field;
    std::vector<uint32_t> values;
  };
  const std::vector<Dim> dims = {
      {&ams_params::k, {128, 256, 512, 1024}},
      {&ams_params::overpartition_b, {2, 4, 8}},
      {&ams_params::base_cutoff, {16, 24, 48}},
      {&ams_params::tile_keys, {16384, 32768, 65536}},
      {&ams_params::levels, {Lauto + 1, Lauto > 1 ? Lauto - 1 : Lauto + 2}},
  };
  for (const Dim &d : dims) {
    for (uint32_t v : d.values) {
      if (trials >= max_trials) break;
      if (cur.*(d.field) == v) continue;
      ams_params cand = cur;
      cand.*(d.field) = v;
      if ((uint64_t)cand.k * cand.overpartition_b > 2048 || cand.levels > MAXLEV) continue;
      if (cand.levels == 0 && Lauto > 0) continue;
      double ms = 0;
      ams_status r = evaluate(cand, ms);
      if (r == AMS_EHIP) return r;  // a device error or a wrong result: stop
      if (r) continue;              // not a valid plan for this shape: skip
      if (ms < cur_ms) {
        cur = cand;
        cur_ms = ms;
      }
    }
  }
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[shape_key((int)t, pay, total, mx, num)] = cur;
  }
  return AMS_OK;
}

extern "C" void ams_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tuned.clear();
}
