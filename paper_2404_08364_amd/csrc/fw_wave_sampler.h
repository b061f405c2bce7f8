// One-wavefront sampler for a hop of any degree, over 16-byte quads.
//
// The neighbour slice [o, o + d) of the CSR arrays is read as aligned quads of
// four entries (one dwordx4 load per array per lane): quad q covers absolute
// positions [a + 4q, a + 4q + 4) with a = o rounded down to a multiple of 4;
// positions outside the slice weigh 0.  The pick of the exact inverse CDF is
// found without any buffer: the quads are split into at most 64 contiguous
// groups; one streaming pass (lane j reads quad j of each 64-quad chunk)
// leaves the total of group g in lane g; a wave prefix scan of those totals
// gives T, the draw r and the group holding r; the same step repeats inside
// that group until at most 64 quads remain, where a scan over the lanes and a
// ballot give the quad and a scan inside the quad gives the entry.  Each
// level re-reads 1/64 of the previous one.
//
// Quad indices are 32-bit (slices are shorter than 2^28 entries) and every
// load is addressed from the slice's uniform base.  The transition-weight
// evaluator is inlined at exactly two places (the streaming loop and the last
// level): the walkers' instruction footprint has to stay inside the
// instruction cache.
#pragma once

#include "fw_device.h"

namespace fw {

// A slice as a run of quads.
struct QuadSlice {
  uint64_t o;     // first entry
  uint64_t a;     // o rounded down to a multiple of 4
  uint32_t d;     // degree
  uint32_t lead;  // o - a: entries of quad 0 before the slice
  uint32_t nq;    // quads covering [o, o + d)
  __device__ __forceinline__ QuadSlice(uint64_t o_, uint64_t d_) : o(o_) {
    a = o_ & ~3ull;
    d = (uint32_t)d_;
    lead = (uint32_t)(o_ - a);
    nq = d ? (lead + d + 3) / 4 : 0;
  }
  // Entry j of quad q lies in the slice (the subtraction wraps below lead).
  __device__ __forceinline__ bool inside(uint32_t q, int j) const {
    return 4 * q + j - lead < d;
  }
};

// The evaluator bound to a slice's quad run.
template <class E>
__device__ __forceinline__ E bind_quads(const E& ev, const QuadSlice& s) {
  E b = ev;
  b.qa = s.a;
  return b;
}

// The four transition weights of quad q (0 outside the slice).
template <class E>
__device__ __forceinline__ void quad_weights(const E& ev, const QuadSlice& s, uint32_t q,
                                             uint64_t w[4]) {
  ev.quad(q, w);
  if (q == 0 || q + 1 == s.nq) {  // only the first and the last quad are partial
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (!s.inside(q, j)) w[j] = 0;
  }
}

// Group layout of `len` quads: at most 64 groups of per_group 64-quad chunks.
struct GroupSplit {
  uint32_t gsz, groups;
  __device__ __forceinline__ explicit GroupSplit(uint32_t len) {
    const uint32_t chunks = (len + kWave - 1) / kWave;
    const uint32_t per_group = (chunks + kWave - 1) / kWave;
    gsz = (per_group ? per_group : 1) * kWave;
    groups = (len + gsz - 1) / gsz;
  }
};

// Lane g returns the total of group g of quads [lo, lo + len).  ev is bound.
template <class E>
__device__ __forceinline__ uint64_t wave_group_totals(const E& ev, const QuadSlice& s,
                                                      uint32_t lo, uint32_t len,
                                                      const GroupSplit& sp) {
  const int lane = lane_id();
  uint64_t mine = 0;
  for (uint32_t g = 0; g < sp.groups; ++g) {
    const uint32_t gb = lo + g * sp.gsz;
    const uint32_t ge = min(gb + sp.gsz, lo + len);
    uint64_t acc = 0;
    if constexpr (E::kCheapTotal) {
      // The slice's first and last quads need the masked weights; every
      // other quad takes the evaluator's own total, a few bit operations on
      // one small load.  Those loads are short, so eight (then four) quads
      // per lane are loaded at once to keep enough bytes in flight (sixteen
      // were slower again).
      const uint32_t ib = gb > 1u ? gb : 1u;
      const uint32_t ie = ge < s.nq - 1 ? ge : s.nq - 1;
      uint32_t q = ib + (uint32_t)lane;
#pragma unroll 1
      for (; q + 7 * kWave < ie; q += 8 * kWave) {
        uint64_t t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = ev.quad_total4(q + k * kWave);
        acc += ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
      }
      if (q + 3 * kWave < ie) {
        const uint64_t t0 = ev.quad_total4(q), t1 = ev.quad_total4(q + kWave),
                       t2 = ev.quad_total4(q + 2 * kWave), t3 = ev.quad_total4(q + 3 * kWave);
        acc += (t0 + t1) + (t2 + t3);
        q += 4 * kWave;
      }
#pragma unroll 1
      for (; q < ie; q += kWave) acc += ev.quad_total4(q);
      const bool first = gb == 0 && ge > 0 && lane == 0;
      const bool last = ge == s.nq && s.nq > 1 && gb < ge && lane == 1;
      if (first || last) {
        uint64_t w[4];
        quad_weights(ev, s, first ? 0u : s.nq - 1, w);
        acc += (w[0] + w[1]) + (w[2] + w[3]);
      }
    } else {
      // Not unrolled: at eight wavefronts per SIMD occupancy hides the load
      // latency, and a second copy of the evaluator would spill registers.
#pragma unroll 1
      for (uint32_t q = gb + lane; q < ge; q += kWave) {
        uint64_t w[4];
        quad_weights(ev, s, q, w);
        acc += (w[0] + w[1]) + (w[2] + w[3]);
      }
    }
    const uint64_t tot = wave_sum(acc);
    if ((uint32_t)lane == g) mine = tot;
  }
  return mine;
}

// Last level: lane i holds the weights of quad lo + i (0 for i >= len,
// len <= 64).  With have_r the draw r is below their total; otherwise
// r = floor(u * T / 2^64) from the total T.  Returns the picked index
// relative to s.o, or -1 when the total is 0.
__device__ __forceinline__ int64_t pick_in_quads(const uint64_t w[4], const QuadSlice& s,
                                                 uint32_t lo, uint32_t len, uint64_t r,
                                                 bool have_r, uint64_t u) {
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
  return (int64_t)(4 * (lo + (uint32_t)L) + jl) - (int64_t)s.lead;
}

// Descends from quads [lo, lo + len) to the picked entry.  With have_r the
// draw r (below the range's total) is given; otherwise the first level's
// total T yields r = floor(u * T / 2^64).  Returns the index relative to s.o,
// or -1 when the total is 0.  ev is bound.
template <class E>
__device__ __forceinline__ int64_t wave_descend(const E& ev, const QuadSlice& s, uint32_t lo,
                                                uint32_t len, uint64_t r, bool have_r,
                                                uint64_t u) {
  const int lane = lane_id();
  while (len > (uint32_t)kWave) {
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
    lo += (uint32_t)gs * sp.gsz;
    len = min(sp.gsz, len - (uint32_t)gs * sp.gsz);
  }
  uint64_t w[4] = {0, 0, 0, 0};
  if ((uint32_t)lane < len) quad_weights(ev, s, lo + lane, w);
  return pick_in_quads(w, s, lo, len, r, have_r, u);
}

// Given r below the total of quads [lo, lo + len), returns the relative index
// (from s.o) of the first entry whose inclusive prefix (from quad lo) exceeds r.
template <class E>
__device__ __forceinline__ uint64_t wave_locate(const E& ev, const QuadSlice& s, uint32_t lo,
                                                uint32_t len, uint64_t r) {
  return (uint64_t)wave_descend(bind_quads(ev, s), s, lo, len, r, true, 0);
}

// Returns the index (relative to the slice) of the picked neighbour, or -1
// when the slice's total weight is 0.  o, d and u are wave-uniform.
template <class E>
__device__ __forceinline__ int64_t wave_pick(const E& ev, uint64_t o, uint64_t d, uint64_t u) {
  const QuadSlice s(o, d);
  return wave_descend(bind_quads(ev, s), s, 0, s.nq, 0, false, u);
}

}  // namespace fw
