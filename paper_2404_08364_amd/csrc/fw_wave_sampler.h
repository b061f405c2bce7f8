// One-wavefront sampler for a hop of any degree, over 16-byte quads.
//
// The neighbour slice [o, o + d) of the CSR arrays is read as aligned quads of
// four entries (one dwordx4 load per array per lane): quad q covers absolute
// positions [A + 4q, A + 4q + 4) with A = o rounded down to a multiple of 4;
// positions outside the slice weigh 0.  The pick of the exact inverse CDF is
// found without any buffer: the quads are split into at most 64 contiguous
// groups; one streaming pass (lane j reads quad j of each 64-quad chunk)
// leaves the total of group g in lane g; a wave prefix scan of those totals
// gives T, the draw r and the group holding r; the same step repeats inside
// that group until at most 64 quads remain, where a scan over the lanes and a
// ballot give the quad and a scan inside the quad gives the entry.  Each
// level re-reads 1/64 of the previous one.
//
// The transition-weight evaluator is inlined at exactly two places (the
// streaming loop and the last level): the walkers' instruction footprint has
// to stay inside the instruction cache.
#pragma once

#include "fw_device.h"

namespace fw {

// Absolute-position view of a slice.
struct QuadSlice {
  uint64_t o, d;   // first entry, degree
  uint64_t a;      // o rounded down to a multiple of 4
  uint64_t nq;     // quads covering [o, o + d)
  __device__ __forceinline__ QuadSlice(uint64_t o_, uint64_t d_) : o(o_), d(d_) {
    a = o_ & ~3ull;
    nq = d_ ? (o_ + d_ - a + 3) / 4 : 0;
  }
};

// The four transition weights of quad q (0 outside the slice).
template <class E>
__device__ __forceinline__ void quad_weights(const E& ev, const QuadSlice& s, uint64_t q,
                                             uint64_t w[4]) {
  const uint64_t p = s.a + 4 * q;
  ev.quad(p, w);
  if (p < s.o || p + 4 > s.o + s.d) {  // only the first and last quads
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (p + j < s.o || p + j >= s.o + s.d) w[j] = 0;
  }
}

// Group layout of `len` quads: at most 64 groups of per_group 64-quad chunks.
struct GroupSplit {
  uint64_t gsz, groups;
  __device__ __forceinline__ explicit GroupSplit(uint64_t len) {
    const uint64_t chunks = (len + kWave - 1) / kWave;
    const uint64_t per_group = (chunks + kWave - 1) / kWave;
    gsz = (per_group ? per_group : 1) * kWave;
    groups = (len + gsz - 1) / gsz;
  }
};

// Lane g returns the total of group g of quads [lo, lo + len).
template <class E>
__device__ __forceinline__ uint64_t wave_group_totals(const E& ev, const QuadSlice& s,
                                                      uint64_t lo, uint64_t len,
                                                      const GroupSplit& sp) {
  const int lane = lane_id();
  uint64_t mine = 0;
  for (uint64_t g = 0; g < sp.groups; ++g) {
    const uint64_t gb = lo + g * sp.gsz;
    const uint64_t ge = min(gb + sp.gsz, lo + len);
    uint64_t acc = 0;
    // Not unrolled: at eight wavefronts per SIMD occupancy hides the load
    // latency, and the second copy of the evaluator would spill registers.
#pragma unroll 1
    for (uint64_t q = gb + lane; q < ge; q += kWave) {
      uint64_t w[4];
      quad_weights(ev, s, q, w);
      acc += (w[0] + w[1]) + (w[2] + w[3]);
    }
    const uint64_t tot = wave_sum(acc);
    if ((uint64_t)lane == g) mine = tot;
  }
  return mine;
}

// Descends from quads [lo, lo + len) to the picked entry.  With have_r the
// draw r (below the range's total) is given; otherwise the first level's
// total T yields r = floor(u * T / 2^64).  Returns the index relative to s.o,
// or -1 when the total is 0.
template <class E>
__device__ __forceinline__ int64_t wave_descend(const E& ev, const QuadSlice& s, uint64_t lo,
                                                uint64_t len, uint64_t r, bool have_r,
                                                uint64_t u) {
  const int lane = lane_id();
  while (len > (uint64_t)kWave) {
    const GroupSplit sp(len);
    const uint64_t mine = wave_group_totals(ev, s, lo, len, sp);
    const uint64_t incl = wave_incl_scan(mine);
    if (!have_r) {
      const uint64_t total = readlane64(incl, kWave - 1);
      if (total == 0) return -1;
      r = scale_draw(u, total);
      have_r = true;
    }
    // incl(63) > r always holds; the fallback only keeps indices in range.
    const uint64_t m = ballot(incl > r);
    const int gs = m ? first_lane(m) : (int)sp.groups - 1;
    r -= readlane64(incl - mine, gs);
    lo += (uint64_t)gs * sp.gsz;
    len = min(sp.gsz, len - (uint64_t)gs * sp.gsz);
  }
  uint64_t w[4] = {0, 0, 0, 0};
  if ((uint64_t)lane < len) quad_weights(ev, s, lo + lane, w);
  const uint64_t c0 = w[0], c1 = c0 + w[1], c2 = c1 + w[2], tot = c2 + w[3];
  const uint64_t incl = wave_incl_scan(tot);
  if (!have_r) {
    const uint64_t total = readlane64(incl, kWave - 1);
    if (total == 0) return -1;
    r = scale_draw(u, total);
  }
  const uint64_t m = ballot(incl > r);
  const int L = m ? first_lane(m) : (int)(len ? len : 1) - 1;
  const uint64_t rr = r - (incl - tot);  // meaningful in lane L
  const uint32_t j = rr < c0 ? 0u : rr < c1 ? 1u : rr < c2 ? 2u : 3u;
  const uint32_t jl = readlane32(j, L);
  return (int64_t)(s.a + 4 * (lo + (uint64_t)L) + jl - s.o);
}

// Given r below the total of quads [lo, lo + len), returns the relative index
// (from s.o) of the first entry whose inclusive prefix (from quad lo) exceeds r.
template <class E>
__device__ __forceinline__ uint64_t wave_locate(const E& ev, const QuadSlice& s, uint64_t lo,
                                                uint64_t len, uint64_t r) {
  return (uint64_t)wave_descend(ev, s, lo, len, r, true, 0);
}

// Returns the index (relative to the slice) of the picked neighbour, or -1
// when the slice's total weight is 0.  o, d and u are wave-uniform.
template <class E>
__device__ __forceinline__ int64_t wave_pick(const E& ev, uint64_t o, uint64_t d, uint64_t u) {
  const QuadSlice s(o, d);
  return wave_descend(ev, s, 0, s.nq, 0, false, u);
}

}  // namespace fw
