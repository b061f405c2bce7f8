// One-wavefront sampler for a hop of any degree.
//
// It computes the pick of the exact inverse CDF without any buffer: the
// neighbour slice is split into at most 64 contiguous groups; one streaming
// pass (coalesced, lane j reads element j of each 64-wide chunk) leaves the
// total of group g in lane g; a wave prefix scan of those totals gives T, the
// draw r, and the group holding r; the same step then repeats inside that
// group until at most 64 elements remain, where an inclusive scan and a
// ballot give the index.  Each level re-reads 1/64 of the previous one, so a
// hop of degree d evaluates about d * 64/63 transition weights.
#pragma once

#include "fw_device.h"

namespace fw {

// Returns the index (relative to the slice) of the picked neighbour, or -1
// when the slice's total weight is 0.  d and u are wave-uniform.
template <class E>
__device__ __forceinline__ int64_t wave_pick(const E& ev, uint64_t d, uint64_t u) {
  const int lane = lane_id();
  uint64_t lo = 0, len = d, r = 0;
  bool have_r = false;
  while (len > kWave) {
    const uint64_t chunks = (len + kWave - 1) / kWave;
    const uint64_t per_group = (chunks + kWave - 1) / kWave;  // chunks per group
    const uint64_t gsz = per_group * kWave;
    const uint64_t groups = (len + gsz - 1) / gsz;
    uint64_t mine = 0;  // lane g: total of group g
    for (uint64_t g = 0; g < groups; ++g) {
      const uint64_t gb = lo + g * gsz;
      const uint64_t ge = min(gb + gsz, lo + len);
      uint64_t acc = 0;
      for (uint64_t i = gb + lane; i < ge; i += kWave) acc += ev(i);
      const uint64_t tot = wave_sum(acc);
      if ((uint64_t)lane == g) mine = tot;
    }
    const uint64_t incl = wave_incl_scan(mine);
    if (!have_r) {
      const uint64_t total = readlane64(incl, kWave - 1);
      if (total == 0) return -1;
      r = scale_draw(u, total);
      have_r = true;
    }
    // incl(63) > r always holds; the fallback only keeps indices in range.
    const uint64_t m = ballot(incl > r);
    const int gs = m ? first_lane(m) : (int)groups - 1;
    r -= readlane64(incl - mine, gs);
    lo += (uint64_t)gs * gsz;
    len = min(gsz, len - (uint64_t)gs * gsz);
  }
  const uint64_t v = (uint64_t)lane < len ? ev(lo + lane) : 0ull;
  const uint64_t incl = wave_incl_scan(v);
  if (!have_r) {
    const uint64_t total = readlane64(incl, kWave - 1);
    if (total == 0) return -1;
    r = scale_draw(u, total);
  }
  const uint64_t m = ballot(incl > r);
  return (int64_t)(lo + (m ? (uint64_t)first_lane(m) : len - 1));
}

}  // namespace fw
