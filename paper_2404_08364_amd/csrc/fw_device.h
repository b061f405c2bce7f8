// Device primitives for the gfx950 walkers: the step draw (Philox4x64-10),
// 64-bit scaling, wave64 integer scans and ballots, and the per-neighbour
// transition-weight evaluators.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

constexpr uint32_t kEnd = 0xFFFFFFFFu;
constexpr int kWave = 64;
// Degrees (and sampler task sizes) stay below 2^28, so that quad offsets
// within a neighbour slice fit in 32 bits.
constexpr uint64_t kMaxDegree = 1ull << 28;

enum Algo : int { kDeepWalk = 0, kNode2Vec = 1, kMetaPath = 2, kPPR = 3 };

struct DevGraph {
  const uint64_t* __restrict__ off;
  const uint32_t* __restrict__ adj;
  const uint32_t* __restrict__ w;    // nullptr: every weight is 1
  const uint8_t* __restrict__ lab;   // nullptr: no labels
  uint64_t nv;
};

struct DevParams {
  uint32_t f_ret, f_in, f_out;
  uint32_t schema_len;
  uint8_t schema[16];
  uint32_t stop_num, stop_den;  // PPR: stop chance per hop
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC 2011): the four words of the block at
// counter (c0, c1, c2, c3), key (seed, 0).  The step draw is word 0 of the
// block at (qid, t, 0, 0), one per hop, no generator state; word 1 of the
// same block is PPR's stop coin; the reservoir samplers draw entry i's word
// from the block at (qid, t, i / 4, 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t seed, uint64_t out[4]) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t h0 = __umul64hi(kM0, c0), l0 = kM0 * c0;
    const uint64_t h1 = __umul64hi(kM1, c2), l1 = kM1 * c2;
    c0 = h1 ^ c1 ^ k0;
    c1 = l1;
    c2 = h0 ^ c3 ^ k1;
    c3 = l0;
    k0 += kW0;
    k1 += kW1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ __forceinline__ uint64_t philox_draw2(uint64_t seed, uint64_t qid, uint64_t t,
                                                 uint64_t& word1) {
  uint64_t w[4];
  philox4x64_10(qid, t, 0, 0, seed, w);
  word1 = w[1];
  return w[0];
}

__device__ __forceinline__ uint64_t philox_draw(uint64_t seed, uint64_t qid, uint64_t t) {
  uint64_t unused;
  return philox_draw2(seed, qid, t, unused);
}

// PPR: does the query stop before hop t?  True with chance stop_num /
// stop_den: floor(word1 * stop_den / 2^64) < stop_num.
__device__ __forceinline__ bool ppr_stops(const DevParams& p, uint64_t seed, uint64_t qid,
                                          uint64_t t) {
  uint64_t word1;
  philox_draw2(seed, qid, t, word1);
  return __umul64hi(word1, (uint64_t)p.stop_den) < (uint64_t)p.stop_num;
}

// floor(u * total / 2^64) in [0, total).
__device__ __forceinline__ uint64_t scale_draw(uint64_t u, uint64_t total) {
  return __umul64hi(u, total);
}

// ---------------------------------------------------------------------------
// wave64 collectives built from DPP row shifts and row broadcasts.  They must
// be called with every lane of the wavefront active.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  // Lanes whose source is outside the row, or whose row is masked off, read 0.
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = dpp32<CTRL, ROWS>((uint32_t)v);
  const uint32_t hi = dpp32<CTRL, ROWS>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum over the 64 lanes (Hillis-Steele inside each 16-lane
// row, then row 0/2 totals into rows 1/3, then the rows 0-1 total into 2-3).
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
  x += dpp64<0x111, 0xF>(x);  // row_shr:1
  x += dpp64<0x112, 0xF>(x);  // row_shr:2
  x += dpp64<0x114, 0xF>(x);  // row_shr:4
  x += dpp64<0x118, 0xF>(x);  // row_shr:8
  x += dpp64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t x) {
  x += dpp32<0x111, 0xF>(x);
  x += dpp32<0x112, 0xF>(x);
  x += dpp32<0x114, 0xF>(x);
  x += dpp32<0x118, 0xF>(x);
  x += dpp32<0x142, 0xA>(x);
  x += dpp32<0x143, 0xC>(x);
  return x;
}

// Maximum over the 64 lanes (returned in every lane).
__device__ __forceinline__ uint32_t wave_max32(uint32_t x) {
  x = max(x, dpp32<0x111, 0xF>(x));
  x = max(x, dpp32<0x112, 0xF>(x));
  x = max(x, dpp32<0x114, 0xF>(x));
  x = max(x, dpp32<0x118, 0xF>(x));
  x = max(x, dpp32<0x142, 0xA>(x));
  x = max(x, dpp32<0x143, 0xC>(x));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t readlane32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t uniform32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) { return readlane64(wave_incl_scan(x), 63); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int first_lane(uint64_t mask) { return (int)__builtin_ctzll(mask); }

// ---------------------------------------------------------------------------
// Transition weights (section 2.1).  One evaluator per hop; element i is the
// i-th neighbour of the current vertex in CSR order.
// ---------------------------------------------------------------------------
// Entry i of a row, addressed by a 32-bit byte offset from the row's start
// (rows are shorter than 2^28 entries; with a wave-uniform row this is one
// load with a scalar base and no 64-bit address arithmetic).
__device__ __forceinline__ uint32_t row_at(const uint32_t* __restrict__ row, uint32_t i) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(row) + i * 4u);
}

// Lower-bound search of u in the sorted row adj[b, b + n).
__device__ __forceinline__ bool row_contains(const uint32_t* __restrict__ adj, uint64_t b,
                                             uint64_t n, uint32_t u) {
  const uint32_t* __restrict__ row = adj + b;
  uint32_t lo = 0, hi = (uint32_t)n;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (row_at(row, mid) < u)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < (uint32_t)n && row_at(row, lo) == u;
}

// Label of schema entry t mod schema_len, without dynamic register indexing
// (which would spill the parameter block to scratch).
__device__ __forceinline__ uint32_t schema_label(const DevParams& p, uint32_t t) {
  const uint32_t i = t % p.schema_len;
  uint32_t w[4];
  __builtin_memcpy(w, p.schema, 16);
  const uint32_t word = i < 4 ? w[0] : i < 8 ? w[1] : i < 12 ? w[2] : w[3];
  return (word >> (8 * (i & 3))) & 0xFFu;
}

// Four lower-bound searches in the sorted row adj[b, b + n) with one trip
// count for all of them (n is wave-uniform at the callers): no divergence,
// and the four probes of a step, and the two reads of the last step, are
// issued together.
__device__ __forceinline__ void row_contains4(const uint32_t* __restrict__ adj, uint64_t b,
                                              uint64_t n, const uint32_t u[4], bool hit[4]) {
  if (n == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) hit[j] = false;
    return;
  }
  const uint32_t* __restrict__ row = adj + b;
  const uint32_t n32 = (uint32_t)n;  // rows are shorter than 2^28
  uint32_t base[4] = {0, 0, 0, 0};
  uint32_t len = n32;
  while (len > 1) {  // invariant: the lower bound of u[j] is in [base[j], base[j] + len]
    const uint32_t half = len >> 1;
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = row_at(row, base[j] + half);
#pragma unroll
    for (int j = 0; j < 4; ++j) base[j] = (x[j] < u[j]) ? base[j] + half : base[j];
    len -= half;
  }
  const uint32_t last = n32 - 1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t x0 = row_at(row, base[j]);
    const uint32_t x1 = row_at(row, min(base[j] + 1, last));
    hit[j] = (x0 == u[j]) | ((x0 < u[j]) & (base[j] < last) & (x1 == u[j]));
  }
}

// Membership in N(prev) by binary search of its sorted row in global memory.
struct MemberGlobal {
  const uint32_t* __restrict__ adj;
  uint64_t po, pd;
  __device__ __forceinline__ bool contains(uint32_t u) const { return row_contains(adj, po, pd, u); }
  // f[j] = fin if u[j] is in the row, else fout.
  __device__ __forceinline__ void factors4(const uint32_t u[4], uint32_t fin, uint32_t fout,
                                           uint32_t f[4]) const {
    bool hit[4];
    row_contains4(adj, po, pd, u, hit);
#pragma unroll
    for (int j = 0; j < 4; ++j) f[j] = hit[j] ? fin : fout;
  }
};

template <int ALGO, bool WEIGHTED, class MEM = MemberGlobal>
struct Eval {
  const uint32_t* __restrict__ adj;
  const uint32_t* __restrict__ w;
  const uint8_t* __restrict__ lab;
  uint64_t o;  // first CSR entry of the current vertex
  // node2vec: previous vertex, membership in its row, the factors; the
  // first hop uses w alone.
  uint32_t prev;
  MEM mem;
  uint32_t f_ret, f_in, f_out;
  bool first;
  // MetaPath: label this hop must carry.
  uint32_t want;
  // First entry of the current slice's quad run (a multiple of 4): quad q
  // of the run holds the absolute entries qa + 4q .. qa + 4q + 3.
  uint64_t qa = 0;
  // Weight times factor is exact as a 24-bit multiply (bound checked per
  // launch on the host).
  bool narrow = false;

  __device__ __forceinline__ uint64_t operator()(uint64_t i) const {
    const uint64_t e = o + i;
    const uint64_t wt = WEIGHTED ? (uint64_t)w[e] : 1ull;
    if (ALGO == kNode2Vec) {
      if (first) return wt;
      const uint32_t u = adj[e];
      const uint32_t is_ret = (u == prev) ? 1u : 0u;
      const uint32_t is_in = (!is_ret && mem.contains(u)) ? 1u : 0u;
      const uint32_t f = f_out + is_in * (f_in - f_out) + is_ret * (f_ret - f_out);
      return wt * f;
    } else if (ALGO == kMetaPath) {
      return lab[e] == want ? wt : 0ull;
    } else {
      return wt;
    }
  }

  // Total transition weight of quad q (all four entries, so interior quads
  // only).  Unweighted MetaPath counts the matching labels of the quad's
  // word in a few bit operations (kCheapTotal: the streaming pass then takes
  // several quads per lane at once); everything else sums quad().
  static constexpr bool kCheapTotal = ALGO == kMetaPath && !WEIGHTED;
  // Weighted DeepWalk and PPR: a quad's transition weights are its raw
  // weights (one 16-byte load, quad_raw).
  static constexpr bool kRawWeights = (ALGO == kDeepWalk || ALGO == kPPR) && WEIGHTED;
  __device__ __forceinline__ uint4 quad_raw(uint32_t q) const {
    return *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(w + qa) + q * 16u);
  }
  __device__ __forceinline__ uint64_t quad_total4(uint32_t q) const {
    if (ALGO == kMetaPath && !WEIGHTED) return (uint64_t)__builtin_popcount(quad_match(q));
    uint64_t o[4];
    quad(q, o);
    return (o[0] + o[1]) + (o[2] + o[3]);
  }

  // Unweighted MetaPath: bit 7 of byte j is set iff entry j of quad q
  // carries the wanted label (a zero byte of labels ^ want, found without
  // carries between bytes).
  __device__ __forceinline__ uint32_t quad_match(uint32_t q) const {
    return match_bits(quad_labels(q));
  }
  // The four labels of quad q, entry j in byte j.
  __device__ __forceinline__ uint32_t quad_labels(uint32_t q) const {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(lab + qa) + q * 4u);
  }
  __device__ __forceinline__ uint32_t match_bits(uint32_t l) const {
    const uint32_t x = l ^ (want * 0x01010101u);
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
  }

  // Weights of quad q of the run at qa (the arrays are padded so that a
  // quad never ends past the allocation), entries outside the slice
  // included: the caller masks them.  The offset from the uniform base qa is
  // 32-bit (slices are < 2^28 entries), so each load is one scalar base plus
  // one vector offset.
  __device__ __forceinline__ void quad(uint32_t q, uint64_t out[4]) const {
    uint32_t wq[4] = {1u, 1u, 1u, 1u};
    if (WEIGHTED) {
      const uint4 v = *reinterpret_cast<const uint4*>(
          reinterpret_cast<const char*>(w + qa) + q * 16u);
      wq[0] = v.x; wq[1] = v.y; wq[2] = v.z; wq[3] = v.w;
    }
    if (ALGO == kNode2Vec) {
      if (first) {
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j] = wq[j];
        return;
      }
      const uint4 a = *reinterpret_cast<const uint4*>(
          reinterpret_cast<const char*>(adj + qa) + q * 16u);
      const uint32_t u[4] = {a.x, a.y, a.z, a.w};
      // f_in for a neighbour of prev, f_out otherwise, then f_ret for prev.
      uint32_t f[4];
      mem.factors4(u, f_in, f_out, f);
      const uint32_t fr = f_ret;
#pragma unroll
      for (int j = 0; j < 4; ++j) f[j] = u[j] == prev ? fr : f[j];
      if (narrow) {
        // (HIP's __umul24 returns a signed int: go through uint32_t.)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j] = (uint64_t)(uint32_t)__umul24(wq[j], f[j]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) out[j] = (uint64_t)wq[j] * f[j];
      }
    } else if (ALGO == kMetaPath) {
      const uint32_t l = *reinterpret_cast<const uint32_t*>(
          reinterpret_cast<const char*>(lab + qa) + q * 4u);
#pragma unroll
      for (int j = 0; j < 4; ++j) out[j] = (((l >> (8 * j)) & 0xFFu) == want) ? wq[j] : 0ull;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) out[j] = wq[j];
    }
  }
};

}  // namespace fw
