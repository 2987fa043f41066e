// C ABI of the sort library: argument checks, workspace handling and the
// step entry points.  Every sort call only enqueues work on the caller's
// stream.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ams.h"
#include "ams_engine.h"

namespace ams {
const char *last_error();
ams_status run_plan_ex(const Plan &pl, void *ws, const RootSource &src, hipStream_t s,
                       uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                       const void *given_splitters, bool shrink_last);
ams_status run_pack_only(const uint32_t *d_w, uint32_t nb, uint32_t r, uint32_t *d_out,
                         hipStream_t s);
ams_status copy_splitters(const Plan &pl, void *ws, void *d_out, uint32_t m, hipStream_t s);
ams_status run_sample_only(const Plan &pl, void *wsv, const RootSource &rs, hipStream_t s);
ams_status trace_start();
int trace_stop(ams_trace_entry *out, int max);
ams_status device_errors(hipStream_t s, uint32_t *bits, bool clear);
ams_status run_errors(const void *ws, hipStream_t s, uint32_t *bits);
ams_status run_stats(const void *ws, hipStream_t s, ams_run_stats *out);
ams_status device_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
ams_status noalloc_scratch(void **ptr);
}  // namespace ams

using namespace ams;

namespace {

bool valid_type(ams_key_t t) { return t == AMS_U32 || t == AMS_U64 || t == AMS_F32; }

size_t key_bytes(ams_key_t t) { return t == AMS_U64 ? 8 : 4; }

// Workspace provided by the caller, or allocated and freed in stream order.
struct WsGuard {
  void *ptr = nullptr;
  bool owned = false;
  hipStream_t s = nullptr;
  ams_status acquire(void *given, size_t given_bytes, size_t need, hipStream_t st) {
    s = st;
    if (given) {
      if (given_bytes < need) {
        set_error("workspace of %zu bytes is smaller than the %zu needed", given_bytes, need);
        return AMS_ENOMEM;
      }
      ptr = given;
      return AMS_OK;
    }
    if (need == 0) return AMS_OK;
    hipError_t e = hipMallocAsync(&ptr, need, st);
    if (e != hipSuccess) {
      set_error("hipMallocAsync(%zu): %s", need, hipGetErrorString(e));
      ptr = nullptr;
      return AMS_ENOMEM;
    }
    owned = true;
    return AMS_OK;
  }
  ~WsGuard() {
    if (owned && ptr) (void)hipFreeAsync(ptr, s);
  }
};

// With AMS_FLAG_CHECK: wait for the run and turn a device error it raised
// into AMS_EDEVICE.
ams_status checked(const Plan &pl, ams_status st, const void *ws, hipStream_t s) {
  if (st || !(pl.flags & AMS_FLAG_CHECK)) return st;
  uint32_t bits = 0;
  st = run_errors(ws, s, &bits);
  if (st) return st;
  if (bits) {
    set_error("the device raised error bits 0x%x (a table bound was exceeded)", bits);
    return AMS_EDEVICE;
  }
  return AMS_OK;
}

ams_status sort_single(ams_key_t t, const void *d_kin, const uint32_t *d_vin, void *d_kout,
                       uint32_t *d_vout, size_t n, void *d_ws, size_t ws_bytes, void *stream,
                       const ams_params *p, bool pay) {
  set_error("");
  if (!valid_type(t)) {
    set_error("unknown key type %d", (int)t);
    return AMS_EINVAL;
  }
  if (n == 0) return AMS_OK;
  if (!d_kin || !d_kout || (pay && (!d_vin || !d_vout))) {
    set_error("NULL device pointer with n = %zu", n);
    return AMS_EINVAL;
  }
  Plan pl;
  ams_status st = make_plan(pl, (int)t, pay, nullptr, 1, n, p);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  WsGuard ws;
  st = ws.acquire(d_ws, ws_bytes, pl.bytes, s);
  if (st) return st;
  RootSource rs;
  memset(&rs, 0, sizeof rs);
  rs.mode = 0;
  rs.single.kin = d_kin;
  rs.single.vin = pay ? d_vin : nullptr;
  rs.single.kout = d_kout;
  rs.single.vout = pay ? d_vout : nullptr;
  rs.single.n = n;
  rs.single.tmp_off = 0;
  st = run_plan_ex(pl, ws.ptr, rs, s, nullptr, nullptr, nullptr, nullptr, true);
  return checked(pl, st, ws.ptr, s);
}

}  // namespace

extern "C" {

const char *ams_last_error(void) { return ams::last_error(); }

const char *ams_version(void) { return "ams-mi355x 0.2 (gfx950)"; }

ams_status ams_device_errors(void *stream, uint32_t *bits, int clear) {
  set_error("");
  if (!bits) {
    set_error("bits is NULL");
    return AMS_EINVAL;
  }
  return device_errors((hipStream_t)stream, bits, clear != 0);
}

ams_status ams_device_copy(const void *d_src, void *d_dst, size_t bytes, void *stream) {
  set_error("");
  if (!bytes) return AMS_OK;
  if (!d_src || !d_dst || (((uintptr_t)d_src | (uintptr_t)d_dst) & 15)) {
    set_error("copy needs 16-byte aligned, non-NULL buffers");
    return AMS_EINVAL;
  }
  return device_copy(d_src, d_dst, bytes, (hipStream_t)stream);
}

ams_status ams_workspace_stats(const void *d_ws, void *stream, ams_run_stats *out) {
  set_error("");
  if (!d_ws || !out) {
    set_error("NULL workspace or output");
    return AMS_EINVAL;
  }
  return run_stats(d_ws, (hipStream_t)stream, out);
}

ams_status ams_trace_start(void) { return ams::trace_start(); }

int ams_trace_stop(ams_trace_entry *out, int max) { return ams::trace_stop(out, max); }

size_t ams_workspace_bytes(ams_key_t t, size_t n, int with_vals, const ams_params *p) {
  if (!valid_type(t)) return 0;
  Plan pl;
  if (make_plan(pl, (int)t, with_vals != 0, nullptr, 1, n, p)) return 0;
  return pl.bytes;
}

size_t ams_batch_workspace_bytes(ams_key_t t, const uint64_t *h_offsets, size_t num,
                                 int with_vals, const ams_params *p) {
  if (!valid_type(t) || (num && !h_offsets)) return 0;
  std::vector<uint64_t> sizes(num);
  for (size_t i = 0; i < num; ++i) {
    if (h_offsets[i + 1] < h_offsets[i]) return 0;
    sizes[i] = h_offsets[i + 1] - h_offsets[i];
  }
  Plan pl;
  if (make_plan(pl, (int)t, with_vals != 0, sizes.data(), (uint32_t)num, 0, p)) return 0;
  return pl.bytes;
}

ams_status ams_sort_keys(ams_key_t t, const void *d_in, void *d_out, size_t n, void *d_ws,
                         size_t ws_bytes, void *stream, const ams_params *p) {
  return sort_single(t, d_in, nullptr, d_out, nullptr, n, d_ws, ws_bytes, stream, p, false);
}

ams_status ams_sort_keys_noalloc(ams_key_t t, const void *d_in, void *d_out, size_t n,
                                 void *stream, const ams_params *p) {
  set_error("");
  if (!valid_type(t)) {
    set_error("unknown key type %d", (int)t);
    return AMS_EINVAL;
  }
  if (n == 0) return AMS_OK;
  Plan pl;
  ams_status st = make_plan(pl, (int)t, false, nullptr, 1, n, p);
  if (st) return st;
  if (pl.bytes > NOALLOC_SCRATCH_BYTES) {
    set_error("%zu keys need %zu bytes of workspace, more than the %zu-byte fixed array", n,
              pl.bytes, (size_t)NOALLOC_SCRATCH_BYTES);
    return AMS_EUNSUPPORTED;
  }
  void *ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st) return st;
  // the same path as ams_sort_keys with a caller workspace: nothing below
  // allocates
  return sort_single(t, d_in, nullptr, d_out, nullptr, n, ws, NOALLOC_SCRATCH_BYTES, stream, p,
                     false);
}

ams_status ams_sort_pairs(ams_key_t t, const void *d_kin, const uint32_t *d_vin, void *d_kout,
                          uint32_t *d_vout, size_t n, void *d_ws, size_t ws_bytes, void *stream,
                          const ams_params *p) {
  return sort_single(t, d_kin, d_vin, d_kout, d_vout, n, d_ws, ws_bytes, stream, p, true);
}

ams_status ams_sort_batch(ams_key_t t, const void *d_kin, const uint32_t *d_vin, void *d_kout,
                          uint32_t *d_vout, const uint64_t *h_offsets, const uint64_t *d_offsets,
                          size_t num, void *d_ws, size_t ws_bytes, void *stream,
                          const ams_params *p) {
  set_error("");
  if (!valid_type(t)) {
    set_error("unknown key type %d", (int)t);
    return AMS_EINVAL;
  }
  if (num == 0) return AMS_OK;
  if (!h_offsets) {
    set_error("h_offsets is required");
    return AMS_EINVAL;
  }
  if (num >= (1ull << 31)) {
    set_error("too many segments");
    return AMS_EUNSUPPORTED;
  }
  if (h_offsets[0] != 0) {
    set_error("h_offsets[0] must be 0");
    return AMS_EINVAL;
  }
  std::vector<uint64_t> sizes(num);
  for (size_t i = 0; i < num; ++i) {
    if (h_offsets[i + 1] < h_offsets[i]) {
      set_error("h_offsets must be non-decreasing (index %zu)", i);
      return AMS_EINVAL;
    }
    sizes[i] = h_offsets[i + 1] - h_offsets[i];
  }
  const uint64_t total = h_offsets[num];
  const bool pay = d_vin != nullptr || d_vout != nullptr;
  if (total == 0) return AMS_OK;
  if (!d_kin || !d_kout || (pay && (!d_vin || !d_vout))) {
    set_error("NULL device pointer with %llu elements", (unsigned long long)total);
    return AMS_EINVAL;
  }
  Plan pl;
  ams_status st = make_plan(pl, (int)t, pay, sizes.data(), (uint32_t)num, 0, p);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  WsGuard ws;
  st = ws.acquire(d_ws, ws_bytes, pl.bytes, s);
  if (st) return st;
  const uint64_t *offs = d_offsets;
  if (!offs) {
    uint64_t *dst = (uint64_t *)((char *)ws.ptr + pl.o_dbg);
    hipError_t e = hipMemcpyAsync(dst, h_offsets, (num + 1) * sizeof(uint64_t),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      set_error("offset upload: %s", hipGetErrorString(e));
      return AMS_EHIP;
    }
    offs = dst;
  }
  RootSource rs;
  memset(&rs, 0, sizeof rs);
  rs.mode = 1;
  rs.kin = (const char *)d_kin;
  rs.vin = pay ? d_vin : nullptr;
  rs.kout = (char *)d_kout;
  rs.vout = pay ? d_vout : nullptr;
  rs.d_offsets = offs;
  st = run_plan_ex(pl, ws.ptr, rs, s, nullptr, nullptr, nullptr, nullptr, true);
  return checked(pl, st, ws.ptr, s);
}

// ---------------------------------------------------------------------------
// step entry points
// ---------------------------------------------------------------------------
ams_status ams_step_splitters(ams_key_t t, const void *d_keys, size_t n, uint32_t m, uint32_t a,
                              uint64_t seed, void *d_splitters, void *stream) {
  set_error("");
  if (!valid_type(t) || !d_keys || !d_splitters || n == 0) {
    set_error("bad arguments");
    return AMS_EINVAL;
  }
  const uint32_t Scap = 65536 / (uint32_t)key_bytes(t);
  if (m < 2 || m > 2048 || (m & (m - 1)) || a == 0 || ((uint64_t)a * m) % 256 ||
      (uint64_t)a * m > Scap) {
    set_error("need m a power of two in 2..2048 and a*m a multiple of 256, at most %u", Scap);
    return AMS_EINVAL;
  }
  ams_params p;
  memset(&p, 0, sizeof p);
  p.levels = 1;
  p.k = m;
  p.overpartition_b = 1;
  p.samples_per_bucket = a;
  p.seed = seed ? seed : 14106754ull;
  p.leaf_capacity = 64;
  p.flags = FLAG_NO_BASE_CASE;
  if (m > 1024) {  // k is limited to 1024: use b = 2
    p.k = m / 2;
    p.overpartition_b = 2;
  }
  if (n < 65) {
    set_error("step_splitters needs n >= 65");
    return AMS_EINVAL;
  }
  Plan pl;
  ams_status st = make_plan(pl, (int)t, false, nullptr, 1, n, &p);
  if (st) return st;
  pl.seed = seed;  // exact seed, 0 included
  hipStream_t s = (hipStream_t)stream;
  WsGuard ws;
  st = ws.acquire(nullptr, 0, pl.bytes, s);
  if (st) return st;
  RootSource rs;
  memset(&rs, 0, sizeof rs);
  rs.single.kin = d_keys;
  rs.single.kout = (void *)d_keys;  // never written: only sampling runs
  rs.single.n = n;
  st = run_sample_only(pl, ws.ptr, rs, s);
  if (st) return st;
  return copy_splitters(pl, ws.ptr, d_splitters, m, s);
}

ams_status ams_step_level(ams_key_t t, const void *d_in, void *d_out, size_t n,
                          const void *d_splitters, uint32_t m, uint32_t r, uint32_t flags,
                          uint32_t *d_hist, uint32_t *d_children, uint32_t *n_children,
                          void *stream) {
  set_error("");
  if (t != AMS_U32 && t != AMS_U64) {
    set_error("step_level is defined for integer keys");
    return AMS_EUNSUPPORTED;
  }
  if (!d_in || !d_out || !d_splitters || !d_hist || !d_children || !n_children || n < 65 ||
      d_in == d_out) {
    set_error("bad arguments (n >= 65, distinct in/out)");
    return AMS_EINVAL;
  }
  if (m < 2 || m > 2048 || (m & (m - 1)) || r < 2 || (r & (r - 1)) || r > m || r > 1024) {
    set_error("m and r must be powers of two, 2 <= r <= m <= 2048, r <= 1024");
    return AMS_EINVAL;
  }
  ams_params p;
  memset(&p, 0, sizeof p);
  p.levels = 1;
  p.k = r;
  p.overpartition_b = m / r;
  p.samples_per_bucket = 1;
  p.leaf_capacity = 64;
  p.flags = flags | FLAG_NO_BASE_CASE;
  Plan pl;
  ams_status st = make_plan(pl, (int)t, false, nullptr, 1, n, &p);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  WsGuard ws;
  st = ws.acquire(nullptr, 0, pl.bytes + 256, s);
  if (st) return st;
  uint32_t *d_nch = (uint32_t *)((char *)ws.ptr + pl.bytes);
  RootSource rs;
  memset(&rs, 0, sizeof rs);
  rs.single.kin = d_in;
  rs.single.kout = d_out;
  rs.single.n = n;
  st = run_plan_ex(pl, ws.ptr, rs, s, d_hist, d_children, d_nch, d_splitters, false);
  if (st) return st;
  hipError_t e = hipMemcpyAsync(n_children, d_nch, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("step_level: %s", hipGetErrorString(e));
    return AMS_EHIP;
  }
  pl.flags |= AMS_FLAG_CHECK;
  return checked(pl, AMS_OK, ws.ptr, s);
}

ams_status ams_step_pack(const uint32_t *d_w, uint32_t nb, uint32_t r, uint32_t *d_out,
                         void *stream) {
  set_error("");
  if (!d_w || !d_out || nb == 0 || nb > 4095 || r == 0) {
    set_error("bad arguments");
    return AMS_EINVAL;
  }
  return run_pack_only(d_w, nb, r, d_out, (hipStream_t)stream);
}

ams_status ams_step_base_case(ams_key_t t, const void *d_kin, const uint32_t *d_vin,
                              void *d_kout, uint32_t *d_vout, size_t n, uint32_t base_cutoff,
                              void *stream) {
  if (n > CMAX) {
    set_error("base case holds at most %u keys", CMAX);
    return AMS_EINVAL;
  }
  ams_params p;
  memset(&p, 0, sizeof p);
  p.base_cutoff = base_cutoff;
  bool pay = d_vin != nullptr;
  return sort_single(t, d_kin, d_vin, d_kout, d_vout, n, nullptr, 0, stream, &p, pay);
}

}  // extern "C"
