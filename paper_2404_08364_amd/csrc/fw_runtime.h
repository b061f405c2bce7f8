// Internal host-side state shared by the runtime's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <mutex>

#include "flowwalk.h"
#include "fw_kernels.h"

struct fw_graph {
  uint64_t nv = 0, ne = 0, max_deg = 0, max_w = 1;
  uint64_t* d_off = nullptr;
  uint32_t* d_adj = nullptr;
  uint32_t* d_w = nullptr;
  uint8_t* d_lab = nullptr;
  uint32_t* d_status = nullptr;  // sticky error bits written by kernels
  uint64_t* d_head = nullptr;    // kHeadSlots task-pool heads, one per in-flight launch
  int device = 0;
  int num_cus = 0;
  size_t lds_per_block = 0;                        // device limit, bytes
  uint64_t bytes = 0;
  uint64_t fingerprint = 0;                        // keys the tuned configurations
  mutable std::atomic<uint64_t> launches{0};       // rotates the head counters
  mutable std::mutex mu;                           // guards the cache below
  mutable void* graph_cache = nullptr;             // captured launch graphs
};

namespace fw {

// Head counters (128 B apart) rotated over launches so that up to this many
// persistent launches on one graph may be in flight on different streams.
constexpr int kHeadSlots = 64;
constexpr int kHeadStride = 16;

int set_error(int code, const char* msg);
int check_walk_args(const fw_graph* g, int algo, const fw_params* params, uint64_t n,
                    uint32_t length, const void* starts, const void* out, DevParams* dp);
DevGraph dev_graph(const fw_graph* g);
int read_status(const fw_graph* g, hipStream_t stream);

// Persistent form: configuration and launch (fw_persistent_host.hip).
// mode: FW_MODE_PERSISTENT, FW_MODE_STAGED or FW_MODE_AUTO (the tuned form);
// *staged tells which kernel the configuration is for.
int resolve_tune(const fw_graph* g, int algo, int mode, const fw_tune* user, TuneCfg* cfg,
                 bool* staged);
uint64_t graph_fingerprint(const fw_graph* g, const uint64_t* off, const uint32_t* adj,
                           const uint32_t* w, const uint8_t* lab);
hipError_t launch_persistent_checked(const fw_graph* g, const LaunchArgs& a, hipStream_t stream,
                                     bool use_graph, bool staged);
void release_graph_state(fw_graph* g);
TuneCfg default_tune(const fw_graph* g, int algo, bool staged);
int validate_tune(const fw_graph* g, const TuneCfg& c, bool staged);
int autotune(fw_graph* g, int algo, const DevParams& dp, const uint32_t* starts, uint64_t n,
             uint32_t length, uint64_t seed, hipStream_t stream, TuneCfg* best,
             bool* best_staged);

}  // namespace fw
