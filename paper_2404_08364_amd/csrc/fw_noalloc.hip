// fw_walk_noalloc: the persistent walk for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).  Its only
// scratch, the task-pool head counter the wavefronts claim queries from,
// lives in a static device array of this library instead of the graph's
// rotated head slots; nothing is allocated, on the device or the host.
#include <cstring>
#include <mutex>

#include "fw_runtime.h"

namespace {

// 256 bytes per GPU, held until the process ends: word 0 is the head counter
// (the rest keeps it alone on its cache lines).
constexpr size_t kScratchWords = 32;
static __device__ __align__(256) uint64_t scratch[kScratchWords];

// Device address of `scratch` on each GPU (each holds its own copy), taken
// once per device with that device current.  In host code the array's name
// is not a device address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[kMaxDevices] = {};

int scratch_on(int dev, uint64_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fw::set_error(FW_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fw::set_error(FW_EHIP, e != hipSuccess ? hipGetErrorString(e)
                                                    : "no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FW_OK;
}

}  // namespace

extern "C" int fw_walk_noalloc(const fw_graph* g, fw_algo algo, const fw_params* params,
                               const uint32_t* starts, uint64_t n, uint32_t length,
                               uint64_t seed, uint32_t* out_paths, void* stream) {
  fw::DevParams dp;
  int rc = fw::check_walk_args(g, (int)algo, params, n, length, starts, out_paths, &dp);
  if (rc) return rc;
  if (n == 0) return FW_OK;
  int dev = -1;
  const hipError_t de = hipGetDevice(&dev);
  if (de != hipSuccess) return fw::set_error(FW_EHIP, hipGetErrorString(de));
  if (dev != g->device) return fw::set_error(FW_EINVAL, "the graph lives on another device");
  uint64_t* head = nullptr;
  rc = scratch_on(dev, &head);
  if (rc) return rc;
  fw::LaunchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.algo = (int)algo;
  a.g = fw::dev_graph(g);
  a.prm = dp;
  a.starts = starts;
  a.n = n;
  a.length = length;
  a.seed = seed;
  a.qid_base = 0;
  a.out = out_paths;
  a.status = g->d_status;
  a.head = head;
  a.num_cus = g->num_cus;
  bool staged = false;
  rc = fw::resolve_tune(g, (int)algo, FW_MODE_PERSISTENT, nullptr, &a.cfg, &staged);
  if (rc) return rc;
  a.cfg.narrow = fw::narrow_products(g->max_w, dp);
  // The counter is reset by a one-thread kernel ahead of the walk (no memset
  // node when the caller captures the stream).
  const hipError_t e = fw::launch_persistent(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fw::set_error(FW_EHIP, hipGetErrorString(e));
  return FW_OK;
}
