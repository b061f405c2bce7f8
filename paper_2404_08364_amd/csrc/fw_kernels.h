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
};

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

hipError_t launch_plain(const LaunchArgs& a, hipStream_t stream);
hipError_t launch_persistent(const LaunchArgs& a, hipStream_t stream);

}  // namespace fw
