// Host side of the persistent form: launch configuration (defaults, the
// tuned per-algorithm configuration, user overrides, validation) and the
// launch itself, optionally replayed from a captured hipGraph.
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

struct GraphCache {
  std::map<GraphKey, std::pair<hipGraphExec_t, uint64_t*>> execs;
};

}  // namespace

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
    c.wgs_per_cu = 4;
    c.hash_cells = (algo == 1) ? 1024 : 64;
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

int resolve_tune(const fw_graph* g, int algo, bool staged, const fw_tune* user, TuneCfg* cfg) {
  TuneCfg c = default_tune(g, algo, staged);
  if (!staged) {
    std::lock_guard<std::mutex> lk(g->mu);
    auto it = g->tuned.find(algo);
    if (it != g->tuned.end()) c = it->second;
  }
  if (user) {
    if (user->wg_size) c.wg_size = user->wg_size;
    if (user->slots) c.slots = user->slots;
    if (user->tiny_max) c.tiny_max = user->tiny_max;
    if (user->hub_min) c.hub_min = user->hub_min;
    if (user->wgs_per_cu) c.wgs_per_cu = user->wgs_per_cu;
    if (user->hash_cells) c.hash_cells = user->hash_cells;
  }
  const int rc = validate_tune(g, c, staged);
  if (rc) return rc;
  *cfg = c;
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
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = launch(a, stream);
    e = hipStreamEndCapture(stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    it = cache->execs.emplace(key, std::make_pair(exec, a.head)).first;
  }
  return hipGraphLaunch(it->second.first, stream);
}

void release_graph_state(fw_graph* g) {
  auto* cache = static_cast<GraphCache*>(g->graph_cache);
  if (!cache) return;
  for (auto& kv : cache->execs) (void)hipGraphExecDestroy(kv.second.first);
  delete cache;
  g->graph_cache = nullptr;
}

}  // namespace fw
