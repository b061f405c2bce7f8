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
// load is addressed from the slice's uniform base.  The full transition-weight
// evaluator is inlined at most twice (the streaming pass and the last level;
// the streaming passes of unweighted MetaPath and of weighted DeepWalk / PPR
// use small dedicated forms instead): the walkers' instruction footprint has
// to stay inside the instruction cache.  Where a streaming pass issues
// several loads per lane, a scheduling barrier keeps them together: near the
// register limit of eight wavefronts per SIMD the compiler otherwise waits on
// each load before issuing the next.
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

// Bit 7 of byte j is set for the entries j of quad q inside the slice.
__device__ __forceinline__ uint32_t inside_bytes(const QuadSlice& s, uint32_t q) {
  uint32_t m = 0x80808080u;
  if (q == 0) m &= 0xFFFFFFFFu << (8 * s.lead);
  if (q + 1 == s.nq) m &= 0xFFFFFFFFu >> (8 * (3 - ((s.lead + s.d - 1) & 3u)));
  return m;
}

// Sum of a quad's raw weights, entries outside the slice left out.
__device__ __forceinline__ uint64_t raw_quad_sum(const QuadSlice& s, uint32_t q, uint4 v) {
  uint32_t x[4] = {v.x, v.y, v.z, v.w};
  if (q == 0 || q + 1 == s.nq) {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = s.inside(q, j) ? x[j] : 0u;
  }
  return ((uint64_t)x[0] + x[1]) + ((uint64_t)x[2] + x[3]);
}

// wave_group_totals for an evaluator with a cheap quad total (unweighted
// MetaPath: one 4-byte load of labels and a few bit operations per quad).
// A load that short keeps few bytes in flight, so every lane loads several
// quads before counting.  With eight or more 64-quad chunks per group a lane
// sums eight quads of a group at a time and one wave sum gives the group's
// total; with fewer, four consecutive chunks are counted at once and their
// totals (each at most 256) come from two wave sums of two 16-bit fields.
template <class E>
__device__ __forceinline__ uint64_t cheap_group_totals(const E& ev, const QuadSlice& s,
                                                       uint32_t lo, uint32_t len,
                                                       const GroupSplit& sp) {
  const int lane = lane_id();
  const uint32_t P = sp.gsz / kWave;  // chunks per group
  const uint32_t end = lo + len;
  uint64_t mine = 0;
  if (P >= 8) {
    for (uint32_t g = 0; g < sp.groups; ++g) {
      const uint32_t gb = lo + g * sp.gsz;
      const uint32_t ge = min(gb + sp.gsz, end);
      // The slice's first and last quads are counted with their masks.
      const uint32_t ib = gb > 1u ? gb : 1u;
      const uint32_t ie = ge < s.nq - 1 ? ge : s.nq - 1;
      uint64_t acc = 0;
      uint32_t q = ib + (uint32_t)lane;
#pragma unroll 1
      for (; q + 7 * kWave < ie; q += 8 * kWave) {
        uint64_t t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = ev.quad_total4(q + k * kWave);
        acc += ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
      }
#pragma unroll 1
      for (; q < ie; q += kWave) acc += ev.quad_total4(q);
      const bool first = gb == 0 && lane == 0;
      const bool last = ge == s.nq && lane == 1;
      if (first || last) {
        uint64_t w[4];
        quad_weights(ev, s, first ? 0u : s.nq - 1, w);
        acc += (w[0] + w[1]) + (w[2] + w[3]);
      }
      const uint64_t tot = wave_sum(acc);
      if ((uint32_t)lane == g) mine = tot;
    }
    return mine;
  }
  uint32_t g = 0, r = 0;  // group of the next chunk, and its place in the group
#pragma unroll 1
  for (uint32_t c = lo; c < end; c += 4 * kWave) {
    // Every lane loads (past the range it re-reads the range's last quad
    // and counts nothing); the four loads are issued before any is used
    // (the scheduler would otherwise wait on each in turn).
    uint32_t l[4], n[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      l[k] = ev.quad_labels(min(c + (uint32_t)k * kWave + (uint32_t)lane, end - 1));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t q = c + (uint32_t)k * kWave + (uint32_t)lane;
      const uint32_t m = q < end ? inside_bytes(s, q) : 0u;
      n[k] = (uint32_t)__builtin_popcount(ev.match_bits(l[k]) & m);
    }
    uint32_t t[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const uint32_t x = wave_incl_scan32(n[2 * k] | (n[2 * k + 1] << 16));
      t[k] = (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t tot = (t[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
      if ((uint32_t)lane == g) mine += tot;
      if (++r == P) {
        r = 0;
        ++g;
      }
    }
  }
  return mine;
}

// Lane g returns the total of group g of quads [lo, lo + len).  ev is bound.
template <class E>
__device__ __forceinline__ uint64_t wave_group_totals(const E& ev, const QuadSlice& s,
                                                      uint32_t lo, uint32_t len,
                                                      const GroupSplit& sp) {
  if constexpr (E::kCheapTotal) {
    return cheap_group_totals(ev, s, lo, len, sp);
  } else if constexpr (E::kRawWeights) {
    // Four 16-byte loads per lane issued together (the scheduler, near the
    // register limit, would otherwise wait on each in turn): rows read from
    // cache, such as a hub every walk starts from, are bound by load latency.
    const int lane = lane_id();
    uint64_t mine = 0;
    for (uint32_t g = 0; g < sp.groups; ++g) {
      const uint32_t gb = lo + g * sp.gsz;
      const uint32_t ge = min(gb + sp.gsz, lo + len);
      uint64_t acc = 0;
      uint32_t q = gb + lane;
#pragma unroll 1
      for (; q + 3 * kWave < ge; q += 4 * kWave) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = ev.quad_raw(q + k * kWave);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += raw_quad_sum(s, q + k * kWave, v[k]);
      }
      if (q + kWave < ge) {
        const uint4 a = ev.quad_raw(q), b = ev.quad_raw(q + kWave);
        __builtin_amdgcn_sched_barrier(0);
        acc += raw_quad_sum(s, q, a) + raw_quad_sum(s, q + kWave, b);
        q += 2 * kWave;
      }
      if (q < ge) acc += raw_quad_sum(s, q, ev.quad_raw(q));
      const uint64_t tot = wave_sum(acc);
      if ((uint32_t)lane == g) mine = tot;
    }
    return mine;
  } else {
    const int lane = lane_id();
    uint64_t mine = 0;
    for (uint32_t g = 0; g < sp.groups; ++g) {
      const uint32_t gb = lo + g * sp.gsz;
      const uint32_t ge = min(gb + sp.gsz, lo + len);
      uint64_t acc = 0;
      // Not unrolled: at eight wavefronts per SIMD occupancy hides the load
      // latency, and a second copy of the evaluator would spill registers.
#pragma unroll 1
      for (uint32_t q = gb + lane; q < ge; q += kWave) {
        uint64_t w[4];
        quad_weights(ev, s, q, w);
        acc += (w[0] + w[1]) + (w[2] + w[3]);
      }
      const uint64_t tot = wave_sum(acc);
      if ((uint32_t)lane == g) mine = tot;
    }
    return mine;
  }
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
