// Host side of the persistent form: launch configuration (defaults, the
// tuned per-algorithm configuration, user overrides, validation) and the
// launch itself, optionally replayed from a captured hipGraph.
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "fw_runtime.h"

namespace fw {

namespace {

// Static LDS of the persistent kernel (the slot pool), bytes; the hash-set
// region comes on top of it.
constexpr size_t kPoolLdsBytes = 16 * 1024;

struct GraphKey {
  int algo;
  int staged;
  TuneCfg cfg;
  DevParams prm;
  const uint32_t* starts;
  uint32_t* out;
  uint64_t n, seed, qid_base;
  uint32_t length;
  hipStream_t stream;
  bool operator<(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(*this)) < 0; }
};

// A captured launch: its executable graph, the task-pool head counter it
// owns (captured into the graph, so no other launch ever uses it), and an
// event recorded after its latest replay (the caller's stream may be gone
// by the time the entry is dropped; the event is ours).
struct CachedExec {
  hipGraphExec_t exec = nullptr;
  uint64_t* head = nullptr;
  hipEvent_t done = nullptr;
  uint64_t last_use = 0;
};

// Captured launches of one graph handle, at most kMaxCachedExecs of them; the
// least recently replayed one is dropped first (after its stream drains).
constexpr size_t kMaxCachedExecs = 16;

struct GraphCache {
  std::map<GraphKey, CachedExec> execs;
  uint64_t clock = 0;
};

void drop_exec(CachedExec& c) {
  if (c.done) {
    (void)hipEventSynchronize(c.done);  // the latest replay may still be running
    (void)hipEventDestroy(c.done);
  }
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  (void)hipFree(c.head);
  c.exec = nullptr;
  c.head = nullptr;
  c.done = nullptr;
}

// Tuned configurations of both forms, per (graph fingerprint, device,
// algorithm), for the life of the process.
struct Tuned {
  TuneCfg persistent, staged;
  bool have_persistent = false, have_staged = false;
  bool auto_staged = false;  // FW_MODE_AUTO runs the staged form
};

std::mutex g_tuned_mu;
std::map<std::tuple<uint64_t, int, int>, Tuned> g_tuned;

bool find_tuned(const fw_graph* g, int algo, Tuned* out) {
  std::lock_guard<std::mutex> lk(g_tuned_mu);
  auto it = g_tuned.find(std::make_tuple(g->fingerprint, g->device, algo));
  if (it == g_tuned.end()) return false;
  *out = it->second;
  return true;
}

uint64_t mix64(uint64_t x) {  // SplitMix64's finaliser
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

}  // namespace

uint64_t graph_fingerprint(const fw_graph* g, const uint64_t* off, const uint32_t* adj,
                           const uint32_t* w, const uint8_t* lab) {
  uint64_t h = mix64(g->nv) ^ mix64(g->ne + 1) * 3 ^ mix64(g->max_deg + 2) * 5 ^
               mix64(g->max_w + 3) * 7 ^ (w ? 11 : 0) ^ (lab ? 13 : 0);
  constexpr uint64_t kSamples = 4096;
  for (uint64_t k = 0; k < kSamples; ++k) {
    const uint64_t v = g->nv ? k * (g->nv + 1) / kSamples : 0;
    h = mix64(h ^ off[v]);
    if (g->ne) {
      const uint64_t e = k * g->ne / kSamples;
      h = mix64(h ^ adj[e] ^ ((uint64_t)(w ? w[e] : 0) << 32) ^ ((uint64_t)(lab ? lab[e] : 0) << 24));
    }
  }
  return h;
}

TuneCfg default_tune(const fw_graph* g, int algo, bool staged) {
  (void)g;
  TuneCfg c;
  std::memset(&c, 0, sizeof(c));
  if (staged) {
    c.wg_size = 512;
    c.slots = 64;
    c.tiny_max = 16;
    c.hub_min = 2048;
    c.wgs_per_cu = 2;
    c.hash_cells = (algo == 1) ? 8192 : 512;
  } else {
    c.wg_size = 256;
    c.slots = 4;
    c.tiny_max = 16;
    c.hub_min = 17;
    c.wgs_per_cu = 8;  // the kernel is built for 8 wavefronts per SIMD
    c.hash_cells = (algo == 1) ? 1024 : 64;
    c.sparse_ratio = (algo == 1) ? 128 : 0;
  }
  return c;
}

int validate_tune(const fw_graph* g, const TuneCfg& c, bool staged) {
  if (c.tiny_max > 16) return set_error(FW_EINVAL, "tiny_max must be <= 16");
  if (c.wgs_per_cu < 1 || c.wgs_per_cu > 32)
    return set_error(FW_EINVAL, "wgs_per_cu must be in 1..32");
  if (c.hash_cells & (c.hash_cells - 1)) return set_error(FW_EINVAL, "hash_cells must be a power of two");
  if (!staged) {
    if (c.hash_cells < 64) return set_error(FW_EINVAL, "hash_cells must be >= 64");
    if ((size_t)c.hash_cells * 4 * 4 > g->lds_per_block)
      return set_error(FW_EINVAL, "hash_cells exceeds the LDS of a workgroup");
    return FW_OK;
  }
  if (c.wg_size != 256 && c.wg_size != 512 && c.wg_size != 1024)
    return set_error(FW_EINVAL, "wg_size must be 256, 512 or 1024");
  if (c.slots < 1 || c.slots > 128) return set_error(FW_EINVAL, "slots must be in 1..128");
  if (c.hub_min <= c.tiny_max) return set_error(FW_EINVAL, "hub_min must exceed tiny_max");
  if (c.hash_cells < 64 * (c.wg_size / 64))
    return set_error(FW_EINVAL, "hash_cells must be >= 64 per wavefront");
  if (kPoolLdsBytes + (size_t)c.hash_cells * 4 > g->lds_per_block)
    return set_error(FW_EINVAL, "hash_cells exceeds the LDS of a workgroup");
  return FW_OK;
}

int resolve_tune(const fw_graph* g, int algo, int mode, const fw_tune* user, TuneCfg* cfg,
                 bool* staged) {
  Tuned t;
  const bool have = find_tuned(g, algo, &t);
  const bool st = mode == FW_MODE_STAGED || (mode == FW_MODE_AUTO && have && t.auto_staged);
  TuneCfg c = default_tune(g, algo, st);
  if (have && st && t.have_staged) c = t.staged;
  if (have && !st && t.have_persistent) c = t.persistent;
  if (user) {
    if (user->wg_size) c.wg_size = user->wg_size;
    if (user->slots) c.slots = user->slots;
    if (user->tiny_max) c.tiny_max = user->tiny_max;
    if (user->hub_min) c.hub_min = user->hub_min;
    if (user->wgs_per_cu) c.wgs_per_cu = user->wgs_per_cu;
    if (user->hash_cells) c.hash_cells = user->hash_cells;
    if (user->sparse_ratio) c.sparse_ratio = user->sparse_ratio == 0xFFFFFFFFu ? 0 : user->sparse_ratio;
  }
  const int rc = validate_tune(g, c, st);
  if (rc) return rc;
  *cfg = c;
  *staged = st;
  return FW_OK;
}

hipError_t launch_persistent_checked(const fw_graph* g, const LaunchArgs& a, hipStream_t stream,
                                     bool use_graph, bool staged) {
  auto launch = [staged](const LaunchArgs& x, hipStream_t st) {
    return staged ? launch_staged(x, st) : launch_persistent(x, st);
  };
  if (!use_graph || stream == nullptr) return launch(a, stream);
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.algo = a.algo;
  key.staged = staged;
  key.cfg = a.cfg;
  key.prm = a.prm;
  key.starts = a.starts;
  key.out = a.out;
  key.n = a.n;
  key.seed = a.seed;
  key.qid_base = a.qid_base;
  key.length = a.length;
  key.stream = stream;
  std::lock_guard<std::mutex> lk(g->mu);
  if (!g->graph_cache) g->graph_cache = new GraphCache();
  auto* cache = static_cast<GraphCache*>(g->graph_cache);
  auto it = cache->execs.find(key);
  if (it == cache->execs.end()) {
    if (cache->execs.size() >= kMaxCachedExecs) {
      auto lru = cache->execs.begin();
      for (auto j = cache->execs.begin(); j != cache->execs.end(); ++j)
        if (j->second.last_use < lru->second.last_use) lru = j;
      drop_exec(lru->second);
      cache->execs.erase(lru);
    }
    // The captured launch resets and claims from a counter of its own: a
    // rotated head slot could be handed to an eager launch running on another
    // stream at the same time as a replay.
    CachedExec c;
    hipError_t e = hipMalloc((void**)&c.head, kHeadStride * sizeof(uint64_t));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      drop_exec(c);
      return e;
    }
    LaunchArgs x = a;
    x.head = c.head;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t le = launch(x, stream);
      e = hipStreamEndCapture(stream, &graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      drop_exec(c);
      return e;
    }
    it = cache->execs.emplace(key, c).first;
  }
  it->second.last_use = ++cache->clock;
  hipError_t e = hipGraphLaunch(it->second.exec, stream);
  if (e == hipSuccess) e = hipEventRecord(it->second.done, stream);
  return e;
}

// Times cfg on the sample: a warm-up launch, then the faster of two timed
// launches (hipEvents on stream; one launch alone left the choice between
// close configurations to noise).
static int time_config(const fw_graph* g, LaunchArgs a, const TuneCfg& cfg, bool staged,
                       hipStream_t stream, hipEvent_t e0, hipEvent_t e1, float* ms) {
  a.cfg = cfg;
  a.cfg.narrow = narrow_products(g->max_w, a.prm);
  auto launch = [&]() { return staged ? launch_staged(a, stream) : launch_persistent(a, stream); };
  hipError_t e = launch();  // warm-up
  *ms = 1e30f;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
    float t = 0;
    e = hipEventRecord(e0, stream);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess && t < *ms) *ms = t;
  }
  if (e != hipSuccess) return set_error(FW_EHIP, hipGetErrorString(e));
  return FW_OK;
}

int autotune(fw_graph* g, int algo, const DevParams& dp, const uint32_t* starts, uint64_t n,
             uint32_t length, uint64_t seed, hipStream_t stream, TuneCfg* best,
             bool* best_staged) {
  uint32_t* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&out, n * ((uint64_t)length + 1) * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = FW_OK;
  if (e != hipSuccess) rc = set_error(e == hipErrorOutOfMemory ? FW_ENOMEM : FW_EHIP,
                                      "autotune allocation");
  LaunchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.algo = algo;
  a.g = dev_graph(g);
  a.prm = dp;
  a.starts = starts;
  a.n = n;
  a.length = length;
  a.seed = seed;
  a.out = out;
  a.status = g->d_status;
  a.head = g->d_head + kHeadStride * (g->launches.fetch_add(1) % kHeadSlots);
  a.num_cus = g->num_cus;
  const uint64_t lds_cu = 160 * 1024;  // LDS of a compute unit
  // Persistent form.  Coordinate search: occupancy x membership-table size,
  // then the tiny threshold.  Configurations that do not fit the LDS are
  // skipped.
  TuneCfg c = default_tune(g, algo, false), best_p = c;
  float best_p_ms = 1e30f;
  const uint32_t cells[] = {256, 512, 1024, 2048, 4096};
  const uint32_t wgs[] = {3, 4, 5, 6, 7, 8};
  for (uint32_t hc : cells) {
    if (algo != 1 && hc != 256) continue;  // only node2vec uses the tables
    for (uint32_t w : wgs) {
      if (rc) break;
      TuneCfg t = c;
      t.hash_cells = (algo == 1) ? hc : 64;
      t.wgs_per_cu = w;
      if (validate_tune(g, t, false)) continue;
      if ((uint64_t)t.hash_cells * 16 * w > lds_cu) continue;  // would not be resident
      float ms = 0;
      rc = time_config(g, a, t, false, stream, e0, e1, &ms);
      if (!rc && ms < best_p_ms) {
        best_p_ms = ms;
        best_p = t;
      }
    }
  }
  for (uint32_t tm : {0u, 8u, 16u}) {
    if (rc) break;
    TuneCfg t = best_p;
    t.tiny_max = tm;
    float ms = 0;
    rc = time_config(g, a, t, false, stream, e0, e1, &ms);
    if (!rc && ms < best_p_ms) {
      best_p_ms = ms;
      best_p = t;
    }
  }
  // node2vec: how much shorter N(prev) must be than N(cur) for the hop to
  // look N(prev)'s keys up in N(cur) (0: never).
  for (uint32_t sr : {0u, 16u, 32u, 64u, 128u, 256u}) {
    if (rc || algo != 1) break;
    TuneCfg t = best_p;
    t.sparse_ratio = sr;
    float ms = 0;
    rc = time_config(g, a, t, false, stream, e0, e1, &ms);
    if (!rc && ms < best_p_ms) {
      best_p_ms = ms;
      best_p = t;
    }
  }
  // Staged form (section 5.1's block design): workgroup size x hub
  // threshold d_t x local pool size |P_L| (Appendix C.2's two parameters).
  TuneCfg best_s = default_tune(g, algo, true);
  float best_s_ms = 1e30f;
  const uint32_t wg_sizes[] = {256, 512, 1024};
  const uint32_t hub_mins[] = {1024, 4096, 16384};
  const uint32_t pools[] = {32, 64};
  for (uint32_t wg : wg_sizes) {
    for (uint32_t hm : hub_mins) {
      for (uint32_t sl : pools) {
        if (rc) break;
        TuneCfg t = default_tune(g, algo, true);
        t.wg_size = wg;
        t.hub_min = hm;
        t.slots = sl;
        const uint32_t waves = wg / 64;
        if (t.hash_cells < 64 * waves) t.hash_cells = 64 * waves;
        const uint64_t lds_wg = 16 * 1024 + (uint64_t)t.hash_cells * 4;
        t.wgs_per_cu = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(32 / waves, lds_cu / lds_wg));
        if (validate_tune(g, t, true)) continue;
        float ms = 0;
        rc = time_config(g, a, t, true, stream, e0, e1, &ms);
        if (!rc && ms < best_s_ms) {
          best_s_ms = ms;
          best_s = t;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(stream);
  (void)hipFree(out);
  uint32_t st = 0;
  (void)hipMemcpy(&st, g->d_status, sizeof(st), hipMemcpyDeviceToHost);
  if (st) {
    (void)hipMemset(g->d_status, 0, sizeof(st));
    if (!rc) rc = set_error(FW_EINVAL, "a start vertex is >= n_vertices");
  }
  if (rc) return rc;
  Tuned t;
  t.persistent = best_p;
  t.staged = best_s;
  t.have_persistent = t.have_staged = true;
  t.auto_staged = best_s_ms < best_p_ms;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[std::make_tuple(g->fingerprint, g->device, algo)] = t;
  }
  *best = t.auto_staged ? best_s : best_p;
  *best_staged = t.auto_staged;
  return FW_OK;
}

void release_graph_state(fw_graph* g) {
  auto* cache = static_cast<GraphCache*>(g->graph_cache);
  if (!cache) return;
  for (auto& kv : cache->execs) drop_exec(kv.second);
  delete cache;
  g->graph_cache = nullptr;
}

}  // namespace fw
