// Served form: continuous batching of walk requests on one GPU.
//
// The graph stays resident in HBM.  Requests (algorithm, parameters, start
// vertices, length, seed) are submitted from any host thread and queued.  A
// scheduler thread admits queued requests in arrival order while their
// device memory (start vertices + result rows) fits the budget (the memory
// admission rule of Eq. 5, section 5.2, applied per request), groups the
// admitted requests of one round into a batch, and launches the batch on one
// of a few streams: per algorithm, one multi-request persistent launch whose
// global task pool is the concatenation of the batch's queries.  Batches on
// different streams run concurrently, so requests that arrive while others
// are on the GPU are admitted as memory and streams free up, and their
// workgroups start as the earlier launches' workgroups retire.  Results are
// copied back on the batch's stream into pinned memory.
//
// Every walk depends only on (graph, algorithm, parameters, request seed,
// index in the request, start), so a request's result is the same alone and
// in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fw_runtime.h"

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) with coalescing (host bookkeeping of the
// device arena and of the pinned host staging arena).
class Arena {
 public:
  explicit Arena(uint64_t size) : size_(size) { free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = (bytes + 255) & ~255ull;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_[*off] = bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    uint64_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  uint64_t size() const { return size_; }

 private:
  uint64_t size_;
  std::map<uint64_t, uint64_t> free_, used_;
};

enum ReqState { kQueued, kRunning, kDone, kFailed };

struct Request {
  uint64_t ticket;
  int algo;
  fw::DevParams prm;
  std::vector<uint32_t> starts;
  uint64_t n;
  uint32_t length;
  uint64_t seed;
  uint64_t bytes = 0;
  uint64_t off = 0, hoff = 0;   // device region and its pinned host staging region
  bool has_region = false;      // device region held (until the rows are copied back)
  bool has_host = false;        // host region held (until the request is collected)
  ReqState state = kQueued;
  int status = FW_OK;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  bool small = false;  // runs in its batch's first phase
  bool claimed = false;  // a wait has taken the ticket
  // A finished request whose host region was reclaimed before it was waited
  // for keeps its rows and hop count here.
  bool spilled = false;
  std::vector<uint32_t> spill;
  uint64_t spill_steps = 0;
};

constexpr int kMaxAlgos = 4;  // DeepWalk, node2vec, MetaPath, PPR

// A batch may run in two phases on its stream: first one launch per
// algorithm over its small requests (n <= small_max_queries, when that is
// non-zero) and their copies back, then the same for the others.  Each phase
// ends with an event, so small requests complete without waiting for the
// large ones of their batch.
constexpr int kPhases = 2;

// Workgroups per CU reserved for the express lane (fw_server_opts).
constexpr uint32_t kExpressWgs = 2;

struct Batch {
  bool express = false;  // the express lane: small requests, a reserved share of the CUs
  std::vector<std::shared_ptr<Request>> reqs;
  hipEvent_t done = nullptr;        // end of the last phase
  hipEvent_t small_done = nullptr;  // end of the small-request phase
  bool small_pending = false;       // small_done recorded, not yet observed
  bool busy = false;
  // Per (phase, algorithm): descriptor table + prefix (device and pinned
  // staging).
  fw::ReqDesc* d_desc[kPhases * kMaxAlgos] = {};
  uint64_t* d_prefix[kPhases * kMaxAlgos] = {};
  fw::ReqDesc* h_desc[kPhases * kMaxAlgos] = {};
  uint64_t* h_prefix[kPhases * kMaxAlgos] = {};
  uint64_t* d_head = nullptr;  // kMaxAlgos counters, 128 B apart
  hipStream_t stream = nullptr;
};

}  // namespace

struct fw_server {
  const fw_graph* g = nullptr;
  fw_server_opts opts{};
  fw::TuneCfg cfg[kMaxAlgos];
  uint8_t* d_arena = nullptr;
  uint8_t* h_arena = nullptr;  // pinned host staging, twice the device budget
  std::unique_ptr<Arena> arena, host_arena;
  std::vector<Batch> batches;
  uint32_t* d_status = nullptr;

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  int waiters = 0;
  bool stop = false;
  std::thread thread;
  std::string fatal;
};

namespace {

int fail(int code, const char* msg) { return fw::set_error(code, msg); }

// A request's arena region: its realised-hop counter (in a 256-byte cell),
// its start vertices (rounded up to 256 bytes), then its rows.
constexpr uint64_t kCounterBytes = 256;

uint64_t starts_bytes(uint64_t n) { return (n * 4 + 255) & ~255ull; }

uint64_t request_bytes(uint64_t n, uint32_t length) {
  return kCounterBytes + starts_bytes(n) + n * ((uint64_t)length + 1) * 4;
}

// Launches one batch (scheduler thread, lock not held).
hipError_t launch_batch(fw_server* s, Batch& b) {
  hipError_t e = hipSuccess;
  for (auto& r : b.reqs) {
    // The counter starts at zero and goes over with the start vertices.
    uint8_t* h = s->h_arena + r->hoff;
    std::memset(h, 0, kCounterBytes);
    std::memcpy(h + kCounterBytes, r->starts.data(), r->n * 4);
    e = hipMemcpyAsync(s->d_arena + r->off, h, kCounterBytes + r->n * 4, hipMemcpyHostToDevice,
                       b.stream);
    if (e != hipSuccess) return e;
  }
  const fw::DevGraph dg = fw::dev_graph(s->g);
  b.small_pending = false;
  for (int ph = 0; ph < kPhases; ++ph) {
    const bool small = ph == 0;
    bool any = false;
    for (int a = 0; a < kMaxAlgos; ++a) {
      const int ta = ph * kMaxAlgos + a;
      uint32_t k = 0;
      uint64_t total = 0;
      for (auto& r : b.reqs) {
        if (r->algo != a || r->small != small) continue;
        fw::ReqDesc& d = b.h_desc[ta][k];
        d.steps = reinterpret_cast<unsigned long long*>(s->d_arena + r->off);
        d.starts = reinterpret_cast<const uint32_t*>(s->d_arena + r->off + kCounterBytes);
        d.out = reinterpret_cast<uint32_t*>(s->d_arena + r->off + kCounterBytes +
                                            starts_bytes(r->n));
        d.n = r->n;
        d.seed = r->seed;
        d.qid_base = 0;
        d.length = r->length;
        d.pad = 0;
        d.prm = r->prm;
        b.h_prefix[ta][k] = total;
        total += r->n;
        ++k;
      }
      if (!k) continue;
      any = true;
      b.h_prefix[ta][k] = total;
      e = hipMemcpyAsync(b.d_desc[ta], b.h_desc[ta], k * sizeof(fw::ReqDesc),
                         hipMemcpyHostToDevice, b.stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(b.d_prefix[ta], b.h_prefix[ta], (k + 1) * sizeof(uint64_t),
                           hipMemcpyHostToDevice, b.stream);
      if (e != hipSuccess) return e;
      fw::ReqTable t{b.d_desc[ta], b.d_prefix[ta], k, total};
      fw::TuneCfg cfg = s->cfg[a];
      if (s->opts.express_max_queries) {
        // The express lane keeps kExpressWgs workgroups per CU for itself;
        // the bulk streams share the rest, so an express launch always finds
        // room instead of waiting for persistent launches to drain.
        const uint32_t bulk = s->opts.max_inflight - 1;
        const uint32_t w = b.express ? kExpressWgs
                                     : std::max<uint32_t>(1, (cfg.wgs_per_cu - kExpressWgs) / bulk);
        cfg.wgs_per_cu = std::min(cfg.wgs_per_cu, w);
      }
      cfg.narrow = 1;
      for (uint32_t i = 0; i < k; ++i)
        cfg.narrow &= fw::narrow_products(s->g->max_w, b.h_desc[ta][i].prm);
      // The phases of one algorithm run one after the other on this stream
      // and share its head counter.
      e = fw::launch_persistent_multi(a, dg, t, s->d_status, b.d_head + 16 * a, s->g->num_cus,
                                      cfg, b.stream);
      if (e != hipSuccess) return e;
    }
    if (!any) continue;
    for (auto& r : b.reqs) {
      if (r->small != small) continue;
      const uint64_t so = kCounterBytes + starts_bytes(r->n);
      e = hipMemcpyAsync(s->h_arena + r->hoff + so, s->d_arena + r->off + so,
                         r->n * ((uint64_t)r->length + 1) * 4, hipMemcpyDeviceToHost, b.stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_arena + r->hoff, s->d_arena + r->off, sizeof(uint64_t),
                           hipMemcpyDeviceToHost, b.stream);
      if (e != hipSuccess) return e;
    }
    if (small) {
      e = hipEventRecord(b.small_done, b.stream);
      if (e != hipSuccess) return e;
      b.small_pending = true;
    }
  }
  return hipEventRecord(b.done, b.stream);
}

// Marks the still-running requests of a batch (all of them, or the small
// ones) finished, by the status of the event that covered them.  (Lock held.)
void finish(fw_server* s, Batch& b, hipError_t q, bool small_only) {
  const uint64_t t = now_ns();
  for (auto& r : b.reqs) {
    if (r->state != kRunning || (small_only && !r->small)) continue;
    r->state = (q == hipSuccess) ? kDone : kFailed;
    if (q != hipSuccess) r->status = FW_EHIP;
    r->t_done = t;
    // The event covered the copy back: the device region is free again.
    if (r->has_region) {
      s->arena->release(r->off);
      r->has_region = false;
    }
  }
  s->cv_done.notify_all();
}

// A finished request gives its device region back at once (its rows are in
// its host region by then) and keeps its host region until it is waited
// for.  Admission is in arrival order; when the next request finds no host
// region, finished requests nobody has collected yet move their rows to
// ordinary host memory and give their host regions back, so that the order
// of the client's waits cannot stall admission.  Returns whether any region
// was freed.  (Lock held.)
bool spill_finished(fw_server* s) {
  bool freed = false;
  for (auto& kv : s->reqs) {
    auto& r = kv.second;
    if (!r->has_host || (r->state != kDone && r->state != kFailed)) continue;
    if (r->state == kDone) {
      const uint64_t so = kCounterBytes + starts_bytes(r->n);
      const uint64_t cells = r->n * ((uint64_t)r->length + 1);
      r->spill.resize(cells);
      std::memcpy(r->spill.data(), s->h_arena + r->hoff + so, cells * 4);
      std::memcpy(&r->spill_steps, s->h_arena + r->hoff, sizeof(uint64_t));
      r->spilled = true;
    }
    s->host_arena->release(r->hoff);
    r->has_host = false;
    freed = true;
  }
  return freed;
}

void scheduler(fw_server* s) {
  (void)hipSetDevice(s->g->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // Completions.
    bool any_busy = false;
    for (auto& b : s->batches) {
      if (!b.busy) continue;
      if (b.small_pending) {
        const hipError_t qs = hipEventQuery(b.small_done);
        if (qs != hipErrorNotReady) {
          finish(s, b, qs, true);
          b.small_pending = false;
        }
      }
      const hipError_t q = hipEventQuery(b.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      finish(s, b, q, false);
      b.small_pending = false;
      b.reqs.clear();
      b.busy = false;
    }
    if (s->stop && s->queue.empty() && !any_busy) break;
    // Admission: one batch per free stream, requests in arrival order (the
    // express lane takes the small requests among them, wherever they are
    // in the queue).
    for (auto& b : s->batches) {
      if (b.busy || s->queue.empty() || s->stop) continue;
      auto it = s->queue.begin();
      while (it != s->queue.end() && b.reqs.size() < s->opts.max_batch_requests) {
        auto r = *it;
        if (b.express && r->n > s->opts.express_max_queries) {
          ++it;
          continue;
        }
        if (!s->arena->alloc(r->bytes, &r->off)) break;  // wait for completions
        if (!s->host_arena->alloc(r->bytes, &r->hoff)) {
          s->arena->release(r->off);
          if (spill_finished(s)) continue;
          break;
        }
        r->has_region = true;
        r->has_host = true;
        r->small = r->n <= s->opts.small_max_queries;
        r->state = kRunning;
        r->t_admit = now_ns();
        b.reqs.push_back(r);
        it = s->queue.erase(it);
      }
      if (b.reqs.empty()) continue;
      b.busy = true;
      lk.unlock();
      const hipError_t e = launch_batch(s, b);
      lk.lock();
      if (e != hipSuccess) {
        for (auto& r : b.reqs) {
          r->state = kFailed;
          r->status = FW_EHIP;
          r->t_done = now_ns();
        }
        (void)hipStreamSynchronize(b.stream);
        b.reqs.clear();
        b.busy = false;
        s->cv_done.notify_all();
      }
      any_busy = true;
    }
    if (s->stop) {
      for (auto& r : s->queue) {
        r->state = kFailed;
        r->status = FW_ECANCELED;
      }
      s->queue.clear();
      s->cv_done.notify_all();
    }
    if (any_busy)
      s->cv_sched.wait_for(lk, std::chrono::microseconds(20));
    else
      s->cv_sched.wait(lk, [s] { return s->stop || !s->queue.empty(); });
  }
}

void release_request(fw_server* s, const std::shared_ptr<Request>& r) {
  if (r->has_region) {
    s->arena->release(r->off);
    r->has_region = false;
  }
  if (r->has_host) {
    s->host_arena->release(r->hoff);
    r->has_host = false;
  }
  s->reqs.erase(r->ticket);
  s->cv_sched.notify_one();
}

}  // namespace

extern "C" {

int fw_server_create(const fw_graph* g, const fw_server_opts* opts, fw_server** out) {
  if (!g || !out) return fail(FW_EINVAL, "NULL argument");
  *out = nullptr;
  auto s = std::make_unique<fw_server>();
  s->g = g;
  if (opts) s->opts = *opts;
  if (!s->opts.mem_budget_bytes) s->opts.mem_budget_bytes = 1ull << 30;
  if (!s->opts.max_inflight) s->opts.max_inflight = 3;
  if (!s->opts.max_batch_requests) s->opts.max_batch_requests = 256;
  if (s->opts.max_inflight > 16 || s->opts.max_batch_requests > 4096)
    return fail(FW_EINVAL, "max_inflight <= 16 and max_batch_requests <= 4096");
  if (s->opts.express_max_queries && s->opts.max_inflight < 2)
    return fail(FW_EINVAL, "an express lane needs max_inflight >= 2");
  for (int a = 0; a < kMaxAlgos; ++a) {
    bool staged = false;
    const int rc = fw::resolve_tune(g, a, FW_MODE_PERSISTENT, nullptr, &s->cfg[a], &staged);
    if (rc) return rc;
  }
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess) e = hipMalloc((void**)&s->d_arena, s->opts.mem_budget_bytes);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_arena, 2 * s->opts.mem_budget_bytes, 0);
  if (e == hipSuccess) e = hipMalloc((void**)&s->d_status, 256);
  if (e == hipSuccess) e = hipMemset(s->d_status, 0, 256);
  s->batches.resize(s->opts.max_inflight);
  if (s->opts.express_max_queries) s->batches[0].express = true;
  const size_t nd = s->opts.max_batch_requests;
  for (auto& b : s->batches) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.small_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void**)&b.d_head, kMaxAlgos * 16 * sizeof(uint64_t));
    for (int a = 0; a < kPhases * kMaxAlgos && e == hipSuccess; ++a) {
      e = hipMalloc((void**)&b.d_desc[a], nd * sizeof(fw::ReqDesc));
      if (e == hipSuccess) e = hipMalloc((void**)&b.d_prefix[a], (nd + 1) * sizeof(uint64_t));
      if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_desc[a], nd * sizeof(fw::ReqDesc), 0);
      if (e == hipSuccess)
        e = hipHostMalloc((void**)&b.h_prefix[a], (nd + 1) * sizeof(uint64_t), 0);
    }
  }
  if (e != hipSuccess) {
    fw_server* raw = s.release();
    fw_server_destroy(raw);
    return fail(e == hipErrorOutOfMemory ? FW_ENOMEM : FW_EHIP, "creating the server");
  }
  s->arena = std::make_unique<Arena>(s->opts.mem_budget_bytes);
  s->host_arena = std::make_unique<Arena>(2 * s->opts.mem_budget_bytes);
  fw_server* raw = s.release();
  raw->thread = std::thread(scheduler, raw);
  *out = raw;
  return FW_OK;
}

int fw_server_submit(fw_server* s, fw_algo algo, const fw_params* params,
                     const uint32_t* starts_host, uint64_t n, uint32_t length, uint64_t seed,
                     uint64_t* ticket) {
  if (!s || !ticket) return fail(FW_EINVAL, "NULL argument");
  fw::DevParams dp;
  const int rc = fw::check_walk_args(s->g, (int)algo, params, n, length, starts_host,
                                     starts_host, &dp);
  if (rc) return rc;
  if (n == 0) return fail(FW_EINVAL, "empty request");
  for (uint64_t i = 0; i < n; ++i)
    if (starts_host[i] >= s->g->nv) return fail(FW_EINVAL, "a start vertex is >= n_vertices");
  auto r = std::make_shared<Request>();
  r->algo = (int)algo;
  r->prm = dp;
  r->starts.assign(starts_host, starts_host + n);
  r->n = n;
  r->length = length;
  r->seed = seed;
  r->bytes = request_bytes(n, length);
  if (r->bytes > s->arena->size()) return fail(FW_ENOMEM, "request larger than the memory budget");
  r->t_submit = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(FW_ECANCELED, "server is shutting down");
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_sched.notify_one();
  return FW_OK;
}

int fw_server_poll(fw_server* s, uint64_t ticket) {
  if (!s) return fail(FW_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FW_EINVAL, "unknown ticket");
  return (it->second->state == kDone || it->second->state == kFailed) ? 1 : 0;
}

int fw_server_wait(fw_server* s, uint64_t ticket, uint32_t* out_host, fw_req_stats* stats) {
  if (!s) return fail(FW_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FW_EINVAL, "unknown ticket");
  std::shared_ptr<Request> r = it->second;
  // One wait per ticket: a second one would read rows whose memory the
  // first gives back.
  if (r->claimed) return fail(FW_EINVAL, "ticket is already being waited for");
  r->claimed = true;
  ++s->waiters;
  s->cv_done.wait(lk, [&] { return r->state == kDone || r->state == kFailed; });
  --s->waiters;
  s->cv_done.notify_all();
  if (stats) {
    stats->submit_ns = r->t_submit;
    stats->admit_ns = r->t_admit;
    stats->done_ns = r->t_done;
    stats->n = r->n;
    stats->length = r->length;
    stats->status = r->status;
    stats->steps = 0;
    if (r->status == FW_OK && r->spilled)
      stats->steps = r->spill_steps;
    else if (r->status == FW_OK && r->has_host)
      std::memcpy(&stats->steps, s->h_arena + r->hoff, sizeof(uint64_t));
  }
  int rc = r->status;
  if (rc == FW_OK && out_host) {
    const uint64_t cells = r->n * ((uint64_t)r->length + 1);
    if (r->spilled)
      std::memcpy(out_host, r->spill.data(), cells * 4);
    else
      std::memcpy(out_host, s->h_arena + r->hoff + kCounterBytes + starts_bytes(r->n), cells * 4);
  }
  release_request(s, r);
  if (rc != FW_OK) return fail(rc, rc == FW_ECANCELED ? "request cancelled" : "request failed");
  return FW_OK;
}

int fw_server_destroy(fw_server* s) {
  if (!s) return FW_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
  }
  if (s->thread.joinable()) s->thread.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& kv : s->reqs) {
      if (kv.second->state == kQueued || kv.second->state == kRunning) {
        kv.second->state = kFailed;
        kv.second->status = FW_ECANCELED;
      }
    }
    s->cv_done.notify_all();
  }
  {
    // Let threads blocked in fw_server_wait return before the memory goes.
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->waiters == 0; });
  }
  for (auto& b : s->batches) {
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.small_done) (void)hipEventDestroy(b.small_done);
    (void)hipFree(b.d_head);
    for (int a = 0; a < kPhases * kMaxAlgos; ++a) {
      (void)hipFree(b.d_desc[a]);
      (void)hipFree(b.d_prefix[a]);
      if (b.h_desc[a]) (void)hipHostFree(b.h_desc[a]);
      if (b.h_prefix[a]) (void)hipHostFree(b.h_prefix[a]);
    }
  }
  (void)hipFree(s->d_arena);
  if (s->h_arena) (void)hipHostFree(s->h_arena);
  (void)hipFree(s->d_status);
  delete s;
  return FW_OK;
}

}  // extern "C"
