// The two parallel reservoir samplers of section 4 for one wavefront (see
// fw_reservoir.hip for the definition of the per-entry words and of the
// visiting orders).  E provides operator()(i): the weight of entry i of the
// sequence.
#pragma once

#include "fw_device.h"

namespace fw {


// Weights and words of quad q (relative entries 4q .. 4q + 3; 0 past d).
template <class E>
__device__ __forceinline__ void quad_entries(const E& ev, uint64_t d, uint64_t q, uint64_t seed,
                                             uint64_t qid, uint32_t t, uint64_t w[4],
                                             uint64_t u[4], bool draw) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t i = 4 * q + j;
    w[j] = i < d ? ev(i) : 0ull;
  }
  if (draw) philox4x64_10(qid, t, q, 1, seed, u);
}

// Last selection among the four entries of a quad, given the running total
// before it; updates the running total.  Returns -1 when none is selected.
__device__ __forceinline__ int64_t quad_select(const uint64_t w[4], const uint64_t u[4],
                                               uint64_t q, uint64_t& running) {
  int64_t sel = -1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    running += w[j];
    if (w[j] != 0 && __umul64hi(u[j], running) < w[j]) sel = (int64_t)(4 * q + j);
  }
  return sel;
}

// The selection of the highest lane that holds one (every lane calls it).
__device__ __forceinline__ int64_t last_selection(int64_t sel) {
  const uint64_t m = ballot(sel >= 0);
  if (!m) return -1;
  const int src = 63 - __builtin_clzll(m);
  return (int64_t)readlane64((uint64_t)sel, src);
}

template <class E>
__device__ __forceinline__ int64_t dprs_pick(const E& ev, uint64_t d, uint64_t seed,
                                             uint64_t qid, uint32_t t) {
  const int lane = lane_id();
  const uint64_t quads = (d + 3) / 4;
  uint64_t base = 0;  // total of the chunks before
  int64_t pick = -1;
  for (uint64_t c = 0; c * kWave < quads; ++c) {
    const uint64_t q = c * kWave + lane;
    uint64_t w[4] = {0, 0, 0, 0}, u[4] = {0, 0, 0, 0};
    if (q < quads) quad_entries(ev, d, q, seed, qid, t, w, u, true);
    const uint64_t s = (w[0] + w[1]) + (w[2] + w[3]);
    const uint64_t incl = wave_incl_scan(s);
    uint64_t running = base + incl - s;
    const int64_t sel = last_selection(quad_select(w, u, q, running));
    if (sel >= 0) pick = sel;
    base += readlane64(incl, kWave - 1);
  }
  return pick;
}

template <class E>
__device__ __forceinline__ int64_t zprs_pick(const E& ev, uint64_t d, uint64_t seed,
                                             uint64_t qid, uint32_t t) {
  const int lane = lane_id();
  const uint64_t quads = (d + 3) / 4;
  uint64_t mine = 0;
  for (uint64_t q = lane; q < quads; q += kWave) {
    uint64_t w[4], u[4];
    quad_entries(ev, d, q, seed, qid, t, w, u, false);
    mine += (w[0] + w[1]) + (w[2] + w[3]);
  }
  uint64_t running = wave_incl_scan(mine) - mine;
  int64_t sel = -1;
  for (uint64_t q = lane; q < quads; q += kWave) {
    uint64_t w[4], u[4];
    quad_entries(ev, d, q, seed, qid, t, w, u, true);
    const int64_t s = quad_select(w, u, q, running);
    if (s >= 0) sel = s;
  }
  return last_selection(sel);
}


}  // namespace fw
