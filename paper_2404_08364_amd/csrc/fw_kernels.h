// Launch interface between the host runtime and the walker kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fw_device.h"

namespace fw {

struct TuneCfg {
  uint32_t wg_size;     // 256, 512 or 1024
  uint32_t slots;       // local pool slots per workgroup
  uint32_t tiny_max;    // degree <= tiny_max: sub-wave sampler
  uint32_t hub_min;     // degree >= hub_min: workgroup sampler
  uint32_t wgs_per_cu;  // persistent workgroups per CU
  uint32_t fetch;       // reserved (refills claim every empty slot at once)
  uint32_t hash_cells;  // LDS hash-set cells per workgroup (power of two)
  uint32_t narrow;      // set per launch: max weight * max factor < 2^24, so a
                        // weight times a factor is one 24-bit multiply
  uint32_t sparse_ratio;  // persistent node2vec: a hop with d(cur) >= ratio *
                          // d(prev) looks N(prev)'s keys up in N(cur) (0: never)
};

// max_w * max_f < 2^24: the product of a weight and a factor fits 32 bits
// and 256 of them fit 32 bits.
inline uint32_t narrow_products(uint64_t max_w, const DevParams& p) {
  uint64_t f = p.f_ret;
  if (p.f_in > f) f = p.f_in;
  if (p.f_out > f) f = p.f_out;
  if (f == 0) f = 1;
  return (max_w < (1ull << 24) && f < (1ull << 24) && max_w * f < (1ull << 24)) ? 1u : 0u;
}

struct LaunchArgs {
  int algo;
  DevGraph g;
  DevParams prm;
  const uint32_t* starts;
  uint64_t n;
  uint32_t length;
  uint64_t seed;
  uint64_t qid_base;
  uint32_t* out;
  uint32_t* status;     // device: bit 0 set when a start vertex is >= V
  uint64_t* head;       // device: global task-pool head (persistent form)
  int num_cus;
  TuneCfg cfg;
};

// One walk request of a multi-request launch (the served form): query i of
// the request has id qid_base + i, starts at starts[i] and writes row i of
// out (length + 1 entries); the realised hops of its retired queries are
// added to *steps (may be null).
struct ReqDesc {
  const uint32_t* starts;
  uint32_t* out;
  unsigned long long* steps;
  uint64_t n, seed, qid_base;
  uint32_t length, pad;
  DevParams prm;
};

// Requests of one launch: prefix[r] = queries before request r, prefix[nreq]
// = total.  All requests of a launch share the algorithm.
struct ReqTable {
  const ReqDesc* reqs;
  const uint64_t* prefix;
  uint32_t nreq;
  uint64_t total;
};

hipError_t launch_plain(const LaunchArgs& a, hipStream_t stream);
// Reservoir-sampling walkers: sampler 1 = DPRS, 2 = ZPRS (plain assignment).
hipError_t launch_reservoir(const LaunchArgs& a, int sampler, hipStream_t stream);
// Multi-request persistent launch on `stream` (resets `head` first).
hipError_t launch_persistent_multi(int algo, const DevGraph& g, const ReqTable& t,
                                   uint32_t* status, uint64_t* head, int num_cus,
                                   const TuneCfg& cfg, hipStream_t stream);
hipError_t launch_persistent(const LaunchArgs& a, hipStream_t stream);
hipError_t launch_staged(const LaunchArgs& a, hipStream_t stream);

}  // namespace fw
