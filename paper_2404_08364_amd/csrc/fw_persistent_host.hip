// Host side of the persistent form: configuration defaults and launch.
#include "fw_runtime.h"

namespace fw {

int resolve_tune(const fw_graph* g, int algo, const fw_tune* user, TuneCfg* cfg) {
  TuneCfg c{256, 64, 16, 4096, 4, 8};
  {
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
    if (user->fetch) c.fetch = user->fetch;
  }
  *cfg = c;
  return FW_OK;
}

hipError_t launch_persistent_checked(const fw_graph* g, const LaunchArgs& a, hipStream_t stream,
                                     bool use_graph) {
  (void)g;
  (void)use_graph;
  return launch_plain(a, stream);
}

void release_graph_state(fw_graph* g) { (void)g; }

}  // namespace fw
