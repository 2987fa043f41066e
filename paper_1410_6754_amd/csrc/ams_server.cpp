// Serving loop: continuous batching of independent sort requests.
//
// Requests (keys already in device memory) wait in a FIFO queue.  A scheduler
// thread forms a batch from the oldest requests of one key type whenever a
// worker stream is free, admitting each request only while the bytes it needs
// (its result buffers plus its share of the batch workspace) fit the memory
// budget; the batch runs through the same level kernels as ams_sort_batch,
// with a root table that points at every request's own buffers.  Batches on
// different streams overlap on the device.  Completion is observed through
// events; results stay in server-owned device buffers until released.
//
// Per batch the host does one plan, one result allocation (carved into every
// request's buffers, freed when the last of them is released), one workspace
// allocation and one copy of the root table from a pinned buffer that each
// stream keeps; the device's default memory pool is set to keep freed memory,
// so these allocations are served from the pool after the first batches.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "ams.h"
#include "ams_engine.h"

namespace ams {
ams_status run_plan_ex(const Plan &pl, void *ws, const RootSource &src, hipStream_t s,
                       uint32_t *dbg_hist, uint32_t *dbg_children, uint32_t *dbg_nchild,
                       const void *given_splitters, bool shrink_last);
size_t run_error_offset();
}

using namespace ams;

namespace {

enum ReqState { PENDING = 0, RUNNING = 1, DONE = 2 };

struct Request {
  uint64_t ticket;
  ams_key_t type;
  const void *keys;
  const uint32_t *vals;
  uint64_t n;
  void *out_k = nullptr;
  uint32_t *out_v = nullptr;
  size_t result_bytes = 0;
  ReqState state = PENDING;
  ams_req_stats st{};
};

struct Batch {
  uint64_t id;
  int stream;
  std::vector<uint64_t> tickets;
  void *ws = nullptr;
  size_t ws_bytes = 0;
};

// One allocation holding the results of a batch's requests.
struct ResultBlock {
  void *ptr = nullptr;
  uint32_t live = 0;  // requests of the batch not yet released
};

// What each worker stream keeps between batches (one batch per stream at a
// time, so reuse never races with a copy still in flight).
struct StreamState {
  hipStream_t s = nullptr;
  bool busy = false;
  Root *h_roots = nullptr;  // pinned staging of the root table
  size_t cap_roots = 0;
  uint32_t *h_err = nullptr;  // pinned copy of the running batch's device error bits
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

double now_us(const std::chrono::steady_clock::time_point &t0) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

size_t kbytes(ams_key_t t) { return t == AMS_U64 ? 8 : 4; }

}  // namespace

struct ams_server {
  int device = 0;
  size_t budget = 0;
  size_t reserved = 0;  // results of unreleased requests + workspaces of running batches
  uint32_t max_pending = 4096;
  std::vector<StreamState> streams;
  std::unordered_map<uint64_t, ResultBlock> blocks;  // by batch id
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;  // pending tickets, FIFO
  std::unordered_map<uint64_t, Request> reqs;
  std::vector<Batch> running;
  uint64_t next_ticket = 1, next_batch = 1;
  uint32_t outstanding = 0;  // pending + running
  bool stop = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  uint64_t max_batch_keys = 1ull << 28;
  uint32_t max_batch_reqs = 1024;
  uint32_t inject_alloc_failures = 0;  // test hook: batches left to fail

  size_t workspace_for(ams_key_t t, bool pay, const std::vector<uint64_t> &sizes) {
    Plan pl;
    if (make_plan(pl, (int)t, pay, sizes.data(), (uint32_t)sizes.size(), 0, nullptr)) return 0;
    return pl.bytes;
  }

  size_t alone_need(const Request &r) {
    std::vector<uint64_t> one{r.n};
    return r.result_bytes + workspace_for(r.type, r.vals != nullptr, one);
  }

  // Result bytes of a request as carved from its batch's block.
  static size_t carved(const Request &r) {
    return align256(r.n * kbytes(r.type)) + (r.vals ? align256(r.n * 4) : 0);
  }

  // Called with mu held through lk (released while a batch is launched).
  // Forms and launches batches while a stream is free.
  // A batch takes the oldest pending requests of the head's key type and
  // payload, in FIFO order, while the result bytes plus a bound on the
  // workspace fit the budget; the exact plan is made once for the batch and
  // requests are dropped from its end if it does not fit.
  void schedule(std::unique_lock<std::mutex> &lk) {
    for (;;) {
      int free_s = -1;
      for (size_t i = 0; i < streams.size(); ++i)
        if (!streams[i].busy) {
          free_s = (int)i;
          break;
        }
      if (free_s < 0 || queue.empty()) return;
      const Request &head = reqs[queue.front()];
      const ams_key_t type = head.type;
      const bool pay = head.vals != nullptr;
      const size_t ew = kbytes(type) + (pay ? 4 : 0);
      std::vector<uint64_t> pick, sizes;
      size_t results = 0;
      uint64_t keys = 0;
      for (auto it = queue.begin(); it != queue.end(); ++it) {
        Request &r = reqs[*it];
        if (r.type != type || (r.vals != nullptr) != pay) continue;
        if (!pick.empty() && (keys + r.n > max_batch_keys || pick.size() >= max_batch_reqs)) break;
        // workspace bound: the keys once more plus tables (well under the keys
        // again) and a fixed part per request
        const size_t bound = 2 * (keys + r.n) * ew + (pick.size() + 1) * 4096 + (64u << 20);
        if (!pick.empty() && reserved + results + carved(r) + bound > budget) break;
        pick.push_back(*it);
        sizes.push_back(r.n);
        results += carved(r);
        keys += r.n;
      }
      size_t ws = 0;
      while (!pick.empty()) {
        ws = workspace_for(type, pay, sizes);
        if (ws && reserved + results + ws <= budget) break;
        results -= carved(reqs[pick.back()]);
        pick.pop_back();
        sizes.pop_back();
      }
      if (pick.empty()) return;  // not enough memory yet; retry when some frees
      launch(lk, free_s, type, pay, pick, sizes, ws, results);
    }
  }

  // Called with mu released (launch): consumes one injected failure.
  bool take_injected_failure() {
    std::lock_guard<std::mutex> g(mu);
    if (!inject_alloc_failures) return false;
    --inject_alloc_failures;
    return true;
  }

  void fail(Request &r, ams_status st) {
    r.state = DONE;
    r.st.status = st;
    r.st.t_done_us = now_us(t0);
    --outstanding;
  }

  // Called with mu held through lk.  The requests leave the queue and are
  // marked running under the lock; the plan, the allocations and the
  // launches run with the lock released, so that submits, polls and
  // releases of other requests do not wait for them.
  void launch(std::unique_lock<std::mutex> &lk, int si, ams_key_t type, bool pay,
              const std::vector<uint64_t> &pick, const std::vector<uint64_t> &sizes,
              size_t ws_bytes, size_t results) {
    StreamState &ss = streams[si];
    hipStream_t s = ss.s;
    Batch b;
    b.id = next_batch++;
    b.stream = si;
    b.tickets = pick;
    b.ws_bytes = ws_bytes;
    const double ta = now_us(t0);
    {
      const std::unordered_set<uint64_t> taken(pick.begin(), pick.end());
      size_t k = 0;
      for (auto it = queue.begin(); it != queue.end() && k < pick.size();) {
        if (taken.count(*it)) {
          it = queue.erase(it);
          ++k;
        } else {
          ++it;
        }
      }
    }
    struct In {
      const void *keys;
      const uint32_t *vals;
      uint64_t n;
      void *out_k;
      uint32_t *out_v;
    };
    std::vector<In> in(pick.size());
    for (size_t i = 0; i < pick.size(); ++i) {
      Request &r = reqs[pick[i]];
      r.state = RUNNING;
      r.st.t_admit_us = ta;
      in[i] = In{r.keys, r.vals, r.n, nullptr, nullptr};
    }
    reserved += results + ws_bytes;
    ss.busy = true;
    lk.unlock();

    ams_status st = AMS_OK;
    ResultBlock blk;
    Plan pl;
    st = make_plan(pl, (int)type, pay, sizes.data(), (uint32_t)sizes.size(), 0, nullptr);
    if (!st && take_injected_failure()) st = AMS_ENOMEM;
    if (!st && hipMallocAsync(&blk.ptr, results ? results : 256, s) != hipSuccess) st = AMS_ENOMEM;
    if (!st && hipMallocAsync(&b.ws, pl.bytes, s) != hipSuccess) st = AMS_ENOMEM;
    if (!st && ss.cap_roots < pick.size()) {
      if (ss.h_roots) (void)hipHostFree(ss.h_roots);
      ss.h_roots = nullptr;
      ss.cap_roots = 0;
      size_t cap = std::max<size_t>(pick.size(), 1024);
      if (hipHostMalloc((void **)&ss.h_roots, sizeof(Root) * cap, 0) != hipSuccess) st = AMS_ENOMEM;
      else ss.cap_roots = cap;
    }
    if (!st) {
      uint64_t off = 0;
      char *cur = (char *)blk.ptr;
      for (size_t i = 0; i < pick.size(); ++i) {
        In &r = in[i];
        r.out_k = cur;
        cur += align256(r.n * kbytes(type));
        if (pay) {
          r.out_v = (uint32_t *)cur;
          cur += align256(r.n * 4);
        }
        Root R;
        R.kin = r.keys;
        R.vin = pay ? r.vals : nullptr;
        R.kout = r.out_k;
        R.vout = r.out_v;
        R.n = r.n;
        R.tmp_off = off;
        off += r.n;
        ss.h_roots[i] = R;
      }
      if (hipMemcpyAsync((char *)b.ws + pl.o_roots, ss.h_roots, sizeof(Root) * pick.size(),
                         hipMemcpyHostToDevice, s) != hipSuccess)
        st = AMS_EHIP;
    }
    if (!st) {
      (void)hipEventRecord(ss.ev0, s);
      RootSource rs;
      memset(&rs, 0, sizeof rs);
      rs.mode = 2;
      st = run_plan_ex(pl, b.ws, rs, s, nullptr, nullptr, nullptr, nullptr, true);
      // the batch's device error bits (counters at the start of the
      // workspace), read back with the batch
      if (!st && hipMemcpyAsync(ss.h_err, (char *)b.ws + run_error_offset(), 4,
                                hipMemcpyDeviceToHost, s) != hipSuccess)
        st = AMS_EHIP;
      (void)hipEventRecord(ss.ev1, s);
    }
    const double tl = now_us(t0);

    lk.lock();
    blk.live = (uint32_t)pick.size();
    if (blk.ptr) blocks[b.id] = blk;
    for (size_t i = 0; i < pick.size(); ++i) {
      Request &r = reqs[pick[i]];
      r.out_k = in[i].out_k;
      r.out_v = in[i].out_v;
      r.st.t_launch_us = tl;
      r.st.batch_id = b.id;
      r.st.batch_size = (uint32_t)pick.size();
      r.result_bytes = carved(r);
      if (st) fail(r, st);
    }
    if (st) {
      (void)hipStreamSynchronize(s);
      finish_batch(b, false);
      reserved -= ws_bytes;
      ss.busy = false;
      cv_done.notify_all();
      return;
    }
    running.push_back(b);
  }

  void finish_batch(Batch &b, bool ok) {
    StreamState &ss = streams[b.stream];
    if (ok) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, ss.ev0, ss.ev1);
      const double td = now_us(t0);
      // a device error of the batch invalidates every result in it
      const ams_status bst = *ss.h_err ? AMS_EDEVICE : AMS_OK;
      for (uint64_t t : b.tickets) {
        Request &r = reqs[t];
        if (r.state == DONE) continue;
        r.state = DONE;
        r.st.status = bst;
        r.st.t_done_us = td;
        r.st.gpu_ms = ms;
        --outstanding;
      }
    }
    if (b.ws) (void)hipFreeAsync(b.ws, ss.s);
    b.ws = nullptr;
  }

  // One request's results are no longer needed: drop it from its block and
  // free the block after the last one.
  void drop_result(Request &r) {
    auto it = blocks.find(r.st.batch_id);
    if (it != blocks.end() && --it->second.live == 0) {
      (void)hipFreeAsync(it->second.ptr, streams[0].s);
      blocks.erase(it);
    }
    r.out_k = nullptr;
    r.out_v = nullptr;
  }

  // Called with mu held: retire finished batches.
  bool reap() {
    bool any = false;
    for (size_t i = 0; i < running.size();) {
      Batch &b = running[i];
      hipError_t q = hipEventQuery(streams[b.stream].ev1);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) {
        for (uint64_t t : b.tickets) {
          Request &r = reqs[t];
          if (r.state != DONE) fail(r, AMS_EHIP);
        }
      }
      finish_batch(b, q == hipSuccess);
      reserved -= b.ws_bytes;
      streams[b.stream].busy = false;
      running.erase(running.begin() + i);
      any = true;
    }
    return any;
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop || !running.empty()) {
      if (reap()) cv_done.notify_all();
      if (!stop) schedule(lk);
      if (running.empty() && (queue.empty() || stop)) {
        cv_work.wait_for(lk, std::chrono::milliseconds(5));
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
  }
};

extern "C" {

ams_server *ams_server_create(int device, size_t hbm_budget, uint32_t max_pending,
                              uint32_t n_streams, ams_status *st) {
  if (st) *st = AMS_OK;
  if (hipSetDevice(device) != hipSuccess) {
    set_error("hipSetDevice(%d) failed", device);
    if (st) *st = AMS_EHIP;
    return nullptr;
  }
  ams_server *s = new ams_server();
  s->device = device;
  if (!hbm_budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      set_error("hipMemGetInfo failed");
      if (st) *st = AMS_EHIP;
      return nullptr;
    }
    hbm_budget = fr / 10 * 8;
  }
  s->budget = hbm_budget;
  s->max_pending = max_pending ? max_pending : 4096;
  uint32_t ns = n_streams ? n_streams : 2;
  // keep freed memory in the device's default pool (result blocks and
  // workspaces come and go with every batch)
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  for (uint32_t i = 0; i < ns; ++i) {
    StreamState ss;
    if (hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&ss.ev0) != hipSuccess || hipEventCreate(&ss.ev1) != hipSuccess ||
        hipHostMalloc((void **)&ss.h_err, 4, 0) != hipSuccess) {
      set_error("hipStreamCreate / hipEventCreate / hipHostMalloc failed");
      if (st) *st = AMS_EHIP;
      s->streams.push_back(ss);
      for (StreamState &x : s->streams) {
        if (x.s) (void)hipStreamDestroy(x.s);
        if (x.ev0) (void)hipEventDestroy(x.ev0);
        if (x.ev1) (void)hipEventDestroy(x.ev1);
        if (x.h_err) (void)hipHostFree(x.h_err);
      }
      delete s;
      return nullptr;
    }
    *ss.h_err = 0;
    s->streams.push_back(ss);
  }
  s->worker = std::thread([s] { s->loop(); });
  return s;
}

ams_status ams_submit(ams_server *srv, ams_key_t t, const void *d_keys, const uint32_t *d_vals,
                      size_t n, uint64_t *ticket) {
  if (!srv || !ticket || (t != AMS_U32 && t != AMS_U64 && t != AMS_F32) || (n && !d_keys)) {
    set_error("bad arguments");
    return AMS_EINVAL;
  }
  if (n > AMS_MAX_SEGMENT) {
    set_error("request of %zu keys: at most %llu are supported", n,
              (unsigned long long)AMS_MAX_SEGMENT);
    return AMS_EUNSUPPORTED;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->outstanding >= srv->max_pending) {
    set_error("%u requests already pending or running", srv->outstanding);
    return AMS_EAGAIN;
  }
  Request r;
  r.ticket = srv->next_ticket++;
  r.type = t;
  r.keys = d_keys;
  r.vals = d_vals;
  r.n = n;
  r.result_bytes = n * kbytes(t) + (d_vals ? n * 4 : 0);
  r.st.n = n;
  r.st.key_type = (int32_t)t;
  r.st.t_submit_us = now_us(srv->t0);
  if (srv->alone_need(r) > srv->budget) {
    set_error("request needs %zu bytes, more than the %zu-byte budget", srv->alone_need(r),
              srv->budget);
    return AMS_ENOMEM;
  }
  *ticket = r.ticket;
  if (n == 0) {
    r.state = DONE;
    r.st.t_admit_us = r.st.t_launch_us = r.st.t_done_us = r.st.t_submit_us;
    srv->reqs[r.ticket] = r;
    return AMS_OK;
  }
  srv->reqs[r.ticket] = r;
  srv->queue.push_back(r.ticket);
  ++srv->outstanding;
  lk.unlock();
  srv->cv_work.notify_one();
  return AMS_OK;
}

ams_status ams_poll(ams_server *srv, uint64_t ticket, int *done, ams_req_stats *stats) {
  if (!srv || !done) return AMS_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return AMS_ENOTFOUND;
  *done = it->second.state == DONE;
  if (stats) *stats = it->second.st;
  return AMS_OK;
}

ams_status ams_wait(ams_server *srv, uint64_t ticket, ams_req_stats *stats) {
  if (!srv) return AMS_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return AMS_ENOTFOUND;
    if (it->second.state == DONE) {
      if (stats) *stats = it->second.st;
      return it->second.st.status;
    }
    srv->cv_done.wait_for(lk, std::chrono::milliseconds(2));
  }
}

ams_status ams_result(ams_server *srv, uint64_t ticket, void **d_keys, uint32_t **d_vals) {
  if (!srv) return AMS_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return AMS_ENOTFOUND;
  if (it->second.state != DONE) {
    set_error("request %llu has not finished", (unsigned long long)ticket);
    return AMS_EAGAIN;
  }
  if (d_keys) *d_keys = it->second.out_k;
  if (d_vals) *d_vals = it->second.out_v;
  return it->second.st.status;
}

ams_status ams_release(ams_server *srv, uint64_t ticket) {
  if (!srv) return AMS_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return AMS_ENOTFOUND;
  Request &r = it->second;
  if (r.state != DONE) {
    set_error("request %llu has not finished", (unsigned long long)ticket);
    return AMS_EAGAIN;
  }
  if (r.st.batch_id) {
    srv->drop_result(r);
    srv->reserved -= r.result_bytes;
  }
  srv->reqs.erase(it);
  srv->cv_work.notify_one();
  return AMS_OK;
}

void ams_server_destroy(ams_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    // requests never launched end with AMS_EAGAIN
    for (uint64_t t : srv->queue) srv->fail(srv->reqs[t], AMS_EAGAIN);
    srv->queue.clear();
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (auto &kv : srv->blocks) (void)hipFreeAsync(kv.second.ptr, srv->streams[0].s);
  srv->blocks.clear();
  for (StreamState &x : srv->streams) {
    (void)hipStreamSynchronize(x.s);
    (void)hipStreamDestroy(x.s);
    if (x.h_roots) (void)hipHostFree(x.h_roots);
    if (x.h_err) (void)hipHostFree(x.h_err);
    (void)hipEventDestroy(x.ev0);
    (void)hipEventDestroy(x.ev1);
  }
  delete srv;
}

ams_status ams_result_copy(ams_server *srv, uint64_t ticket, void *d_keys, uint32_t *d_vals,
                           void *stream) {
  if (!srv) return AMS_EINVAL;
  void *k = nullptr;
  uint32_t *v = nullptr;
  uint64_t n = 0;
  size_t kb = 0;
  {
    // one lookup under the lock: a concurrent release cannot slip in between
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return AMS_ENOTFOUND;
    const Request &r = it->second;
    if (r.state != DONE) {
      set_error("request %llu has not finished", (unsigned long long)ticket);
      return AMS_EAGAIN;
    }
    if (r.st.status) return r.st.status;
    k = r.out_k;
    v = r.out_v;
    n = r.n;
    kb = kbytes(r.type);
    if (!n) return AMS_OK;
    hipStream_t s = (hipStream_t)stream;
    // the copies are enqueued under the lock, so the ticket cannot be
    // released between the lookup and the copies
    if (d_keys && hipMemcpyAsync(d_keys, k, n * kb, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return AMS_EHIP;
    if (d_vals && v && hipMemcpyAsync(d_vals, v, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return AMS_EHIP;
  }
  return AMS_OK;
}

ams_status ams_server_inject_alloc_failures(ams_server *srv, uint32_t count) {
  if (!srv) return AMS_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->inject_alloc_failures = count;
  return AMS_OK;
}

}  // extern "C"
