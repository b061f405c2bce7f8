// Persistent, dynamically scheduled walker (sections 5.1 and 5.2, re-derived
// for wave64).
//
// A fixed grid of wavefronts stays resident.  Each wavefront keeps a local
// task pool of four live queries, one per 16-lane group (query id, current
// and previous vertex, hop index, cached CSR range; every lane of a group
// holds a copy), and refills empty entries from the global task pool with one
// 64-bit atomicAdd on a head counter.  Every round advances each live query
// by one hop:
//   * tiny hops (degree <= tiny_max <= 16) run together, one per 16-lane
//     group: a row-wide DPP scan, a draw per group, a ballot;
//   * every other hop runs on the whole wavefront, one query after the
//     other, with the quad-streaming sampler of fw_wave_sampler.h.
// There are no workgroup barriers: wavefronts never wait for each other, so
// every resident wavefront keeps its loads in flight.
//
// Node2vec membership in N(prev) for non-tiny hops uses the wavefront's LDS
// region: an exact 4-cell-bucket hash set of N(prev) when it fits; otherwise,
// while N(prev) is at most 64x N(cur), a merge of the two sorted rows (each
// 256-entry chunk of N(cur) stages the window of N(prev) that holds its value
// range into LDS and searches it there); when N(prev) is much larger than
// N(cur), binary search of the sorted row in global memory.  No global memory
// beyond the inputs, the output paths and one head counter is used.
#include <cstring>

#include "fw_kernels.h"
#include "fw_wave_sampler.h"

namespace fw {

extern __shared__ __attribute__((aligned(16))) uint32_t fw_dyn_lds[];

constexpr uint32_t kFib24 = 0x9E3779u;  // 2^24 / golden ratio

// Bucket of key u in a table of 2^(32 - shift) buckets (Fibonacci hashing:
// the top bits of the low word of u times 2^24 / golden ratio).  The 24-bit
// multiply runs at the full VALU rate (a 32-bit one at a quarter); ids from
// 2^24 on hash by their low 24 bits, which costs probes, never exactness.
// (HIP's __umul24 returns a signed int: go through uint32_t.)
__device__ __forceinline__ uint32_t bucket_of(uint32_t u, uint32_t shift) {
  return (uint32_t)__umul24(u, kFib24) >> shift;
}
constexpr int kGroups = 4;  // queries per wavefront
// Node2vec hops from vertices of at least this degree may take the
// sparse-N(prev) pass (sparse_prev_group_totals).
constexpr uint64_t kSparseMinDegree = 2048;
// A node2vec hop whose N(prev) is more than this many times longer than
// N(cur) looks each of N(cur)'s keys up by binary search of N(prev) in global
// memory (few keys; the top levels of a hub's row stay in cache); a shorter
// N(prev) goes to the hash set or the merge.  Full passes on one MI355X for
// ratios 16, 32, 64 and 128: R-MAT-22 node2vec 1308, 1272, 1275 and
// 1330 ms; Chung-Lu 227M node2vec, 1M queries, 7157, 7084, 7021 and 6992 ms.
constexpr uint64_t kSearchRatio = 64;
constexpr int kGroupLanes = 16;
constexpr int kBlock = 256;  // threads per workgroup (4 wavefronts)

__device__ __forceinline__ uint32_t log2_ceil(uint64_t x) {
  uint32_t b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// u is one of the four cells: the smallest XOR with u is 0.
__device__ __forceinline__ bool has4(uint4 v, uint32_t u) {
  return min(min(v.x ^ u, v.y ^ u), min(v.z ^ u, v.w ^ u)) == 0u;
}

// The bucket has a free cell.  Cells fill in order (an insert takes the first
// free one), so that is the last cell being free.
__device__ __forceinline__ bool open4(uint4 v) { return v.w == kEnd; }

// Membership in N(prev) for one node2vec hop, by a wave-uniform mode:
//   0  binary search of the sorted row in global memory;
//   1  exact hash set in LDS: nb buckets of 4 cells (16 bytes) at
//      fw_dyn_lds[base, base + 4 nb), kEnd marks an empty cell; a key lives
//      in the first bucket, in probe order from its hash, that had a free cell
//      when it was inserted, so a lookup stops at a hit or at a bucket with a
//      free cell.
// (Mode 2, the merge of sorted rows, has its own code: merge_chunk.)
// One type for all modes keeps a single copy of the sampler in the kernel.
struct MemberAny {
  int mode;
  uint32_t base, bmask, shift;
  const uint32_t* __restrict__ adj;
  uint64_t po, pd;

  // base is a multiple of 4 cells, so a bucket is one aligned 16-byte read.
  __device__ __forceinline__ uint4 bucket(uint32_t b) const {
    return reinterpret_cast<const uint4*>(fw_dyn_lds)[(base >> 2) + b];
  }
  __device__ __forceinline__ bool probe_rest(uint32_t u, uint32_t b) const {
    for (;;) {
      b = (b + 1) & bmask;
      const uint4 v = bucket(b);
      if (has4(v, u)) return true;
      if (open4(v)) return false;
    }
  }
  // f[j] = fin if u[j] is in N(prev), else fout.  Choosing the factor inside
  // the lookup keeps the hits in lane masks on the common path; only the
  // rare longer probes update a factor under a lane mask.
  __device__ __forceinline__ void factors4(const uint32_t u[4], uint32_t fin, uint32_t fout,
                                           uint32_t f[4]) const {
    if (mode == 1) {
      uint32_t b[4];
      uint4 v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        b[j] = bucket_of(u[j], shift);
        v[j] = bucket(b[j]);
      }
      bool more = false;
      bool done[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool hit = has4(v[j], u[j]);
        f[j] = hit ? fin : fout;
        done[j] = hit | open4(v[j]);
        more |= !done[j];
      }
      if (more) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (!done[j]) f[j] = probe_rest(u[j], b[j]) ? fin : fout;
      }
      return;
    }
    bool hit[4];
    row_contains4(adj, po, pd, u, hit);
#pragma unroll
    for (int j = 0; j < 4; ++j) f[j] = hit[j] ? fin : fout;
  }
};

struct Table {
  uint32_t base, cells;   // this wavefront's LDS region
  uint32_t bmask, shift;  // geometry of the hash set
  int kind;               // 0: global search, 1: hash set, 2: merge of sorted rows
  uint64_t po, pd;        // N(prev)
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Chooses (and for the hash set builds) the membership structure of N(prev)
// for one node2vec hop from a vertex of degree d, with the wavefront's lanes.
__device__ __forceinline__ void build_table(Table& tb, const uint32_t* __restrict__ adj,
                                            uint64_t d, int lane, bool allow_merge = true) {
  tb.kind = 0;
  if (tb.pd == 0 || tb.pd > kSearchRatio * d) return;
  if (2 * tb.pd > tb.cells) {
    // Too large for the hash set: merge the sorted rows (the region must
    // hold at least one 256-entry staging round).
    if (allow_merge && tb.cells >= 4 * kWave) tb.kind = 2;
    return;
  }
  // The table takes the whole region: a smaller N(prev) gets a lower load,
  // and a lookup then almost never needs a second bucket (with 64 lanes and
  // four lookups each, any lane needing one costs the whole wavefront).
  const uint32_t bits = log2_ceil(tb.cells / 4);  // cells: a power of two >= 64
  tb.bmask = (1u << bits) - 1;
  tb.shift = 32 - bits;
  const uint4 empty = make_uint4(kEnd, kEnd, kEnd, kEnd);
  for (uint32_t i = lane; i < tb.cells / 4; i += kWave)
    reinterpret_cast<uint4*>(fw_dyn_lds + tb.base)[i] = empty;
  wave_sync_lds();
  for (uint64_t i = lane; i < tb.pd; i += kWave) {
    const uint32_t u = adj[tb.po + i];
    uint32_t b = bucket_of(u, tb.shift);
    for (;;) {
      uint32_t j = 0;
      for (; j < 4; ++j) {
        const uint32_t old = atomicCAS(&fw_dyn_lds[tb.base + 4 * b + j], kEnd, u);
        if (old == kEnd || old == u) break;
      }
      if (j < 4) break;
      b = (b + 1) & tb.bmask;
    }
  }
  wave_sync_lds();
  tb.kind = 1;
}

using lds_ptr = const __attribute__((address_space(3))) uint32_t*;

// One halving step of lds_search4: the lower bound of u[j] is in
// [p[j], p[j] + 2h] before and in [p[j], p[j] + h] after.
__device__ __forceinline__ void lds_step4(lds_ptr p[4], const uint32_t u[4], uint32_t h) {
  uint32_t x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = p[j][h - 1];
#pragma unroll
  for (int j = 0; j < 4; ++j) p[j] = (x[j] < u[j]) ? p[j] + h : p[j];
}

// Four lower-bound searches in the sorted LDS run fw_dyn_lds[b, b + n), one
// trip count for all lanes (n is wave-uniform): hit[j] says whether u[j]
// occurs in the run.  The cell after the run, fw_dyn_lds[b + n], must hold a
// value above every key.  With P the
// largest power of two not above n, one probe at n - P - 1 leaves a range of
// P + 1 candidates, which halving steps narrow to two; the last five steps
// (h = 16 .. 1) are unrolled and entered by a switch, so their probe offsets
// and increments are immediates (4h <= 64 is an inline constant).
__device__ __forceinline__ void lds_search4(uint32_t b, uint32_t n, const uint32_t u[4],
                                            bool hit[4]) {
  if (n == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) hit[j] = false;
    return;
  }
  const lds_ptr run = (lds_ptr)(fw_dyn_lds + b);
  const uint32_t lg = 31u - (uint32_t)__builtin_clz(n);
  const uint32_t P = 1u << lg;
  lds_ptr p[4] = {run, run, run, run};
  if (n > P) {
    const uint32_t x = run[n - P - 1];
#pragma unroll
    for (int j = 0; j < 4; ++j) p[j] = (x < u[j]) ? run + (n - P) : run;
  }
  for (uint32_t h = P >> 1; h >= 32; h >>= 1) lds_step4(p, u, h);
  switch (lg < 5 ? lg : 5) {
    case 5: lds_step4(p, u, 16); [[fallthrough]];
    case 4: lds_step4(p, u, 8); [[fallthrough]];
    case 3: lds_step4(p, u, 4); [[fallthrough]];
    case 2: lds_step4(p, u, 2); [[fallthrough]];
    case 1: lds_step4(p, u, 1); [[fallthrough]];
    default: break;
  }
  // The lower bound is p or p + 1; the run is followed by a sentinel above
  // every key, so p[1] is always there to read.
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t x0 = p[j][0], x1 = p[j][1];
    hit[j] = (x0 == u[j]) | ((x0 < u[j]) & (x1 == u[j]));
  }
}

// One 64-quad chunk of a node2vec hop by merging the sorted rows N(cur) and
// N(prev): quads [c0, min(c0 + 64, ge)) of the slice, lane i taking quad
// c0 + i (256 consecutive entries of N(cur), ascending; the chunk's largest
// key kmax is its last entry).  The entries of N(prev) from `cursor` up to
// kmax are staged into LDS (a first round of 64 entries, then rounds of 256
// while they come back full, with lane-consecutive loads) and the chunk's
// keys are looked up there by binary search.  A run too long for the region
// is taken in region-sized sub-windows whose lookups are or-ed.  Entries
// below kmax cannot match a later key, so the cursor then moves past them
// (the staging rounds count them by ballots).  out[j]
// is the transition weight of entry j of the lane's quad (0 outside the
// slice or the chunk), sum their total.
template <class E>
__device__ __forceinline__ void merge_chunk(const E& ev, const QuadSlice& s, const Table& tb,
                                            uint32_t c0, uint32_t ge, uint64_t& cursor,
                                            int lane, uint64_t out[4], uint64_t& sum) {
  const char* __restrict__ wrun = reinterpret_cast<const char*>(ev.w + s.a);
  const char* __restrict__ arun = reinterpret_cast<const char*>(ev.adj + s.a);
  const uint32_t* __restrict__ prow = ev.adj + tb.po;  // N(prev)
  const uint32_t jend = (s.lead + s.d - 1) & 3u;      // slice's last entry in its quad
  const uint32_t q = c0 + lane;
  const bool valid = q < ge;
  const uint32_t qq = valid ? q : c0;
  uint32_t keep = valid ? 0xFu : 0u;
  if (valid && (qq == 0 || qq + 1 == s.nq)) {
    keep = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) keep |= s.inside(qq, j) ? (1u << j) : 0u;
  }
  uint32_t wq[4] = {1u, 1u, 1u, 1u};
  if (ev.w != nullptr) {
    const uint4 v = *reinterpret_cast<const uint4*>(wrun + qq * 16u);
    wq[0] = v.x; wq[1] = v.y; wq[2] = v.z; wq[3] = v.w;
  }
  const uint4 a = *reinterpret_cast<const uint4*>(arun + qq * 16u);
  const uint32_t key[4] = {a.x, a.y, a.z, a.w};
  // The chunk's last entry: entry jl of the quad in lane L (uniform).
  const uint32_t L = min((uint32_t)kWave, ge - c0) - 1;
  const uint32_t jl = (c0 + L + 1 == s.nq) ? jend : 3u;
  const uint32_t kmax = readlane32(jl == 0 ? key[0] : jl == 1 ? key[1] : jl == 2 ? key[2] : key[3],
                                   (int)L);
  // Factor per key: f_out until a sub-window's lookup finds the key.
  uint32_t fo = ev.f_out, fi = ev.f_in;
  uint32_t f[4] = {fo, fo, fo, fo};
  uint64_t sub = cursor;  // first entry of the current sub-window
  uint64_t below = 0;     // entries below kmax staged so far (every entry is staged once)
  for (;;) {
    // Stage N(prev)[sub, sub + W): the entries <= kmax (a prefix, N(prev)
    // being sorted), or as many full rounds of them as the region holds.
    const uint32_t* __restrict__ pr = prow + sub;
    // Entries left in N(prev) (clamped: a region holds far fewer).
    const uint32_t left = (uint32_t)min(tb.pd - sub, (uint64_t)0xFFFFFFFFu);
    uint32_t W = 0;
    bool more = false;  // the region filled up before the run ended
    if (left != 0) {
      // Most windows are short: a first round of 64 entries, then
      // rounds of 256 while they come back full.
      const uint32_t k0 = (uint32_t)lane;
      const uint32_t v0 = pr[k0 < left ? k0 : 0u];
      const uint32_t x0 = k0 < left ? v0 : kEnd;  // kEnd is above every key
      fw_dyn_lds[tb.base + k0] = x0;
      W = (uint32_t)__builtin_popcountll(ballot(x0 <= kmax));
      below += (uint32_t)__builtin_popcountll(ballot(x0 < kmax));
      bool full = W == (uint32_t)kWave;
      while (full) {
        if (W + 4 * kWave + 1 > tb.cells) {  // one cell stays for the sentinel
          more = true;
          fw_dyn_lds[tb.base + W] = kEnd;  // every lane writes the same value
          break;
        }
        // All four loads first, then the stores and counts.
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t k = W + (uint32_t)j * kWave + (uint32_t)lane;
          v[j] = pr[k < left ? k : 0u];
        }
        uint32_t n_le = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t k = W + (uint32_t)j * kWave + (uint32_t)lane;
          const uint32_t x = k < left ? v[j] : kEnd;
          fw_dyn_lds[tb.base + k] = x;
          n_le += (uint32_t)__builtin_popcountll(ballot(x <= kmax));
          below += (uint32_t)__builtin_popcountll(ballot(x < kmax));
        }
        W += n_le;
        full = n_le == 4u * kWave;
      }
    }
    wave_sync_lds();
    bool h[4];
    lds_search4(tb.base, W, key, h);
#pragma unroll
    for (int j = 0; j < 4; ++j) f[j] = h[j] ? fi : f[j];
    wave_sync_lds();
    if (!more) break;
    sub += W;
  }
  cursor += below;
  const uint32_t fr = ev.f_ret;
#pragma unroll
  for (int j = 0; j < 4; ++j) f[j] = key[j] == ev.prev ? fr : f[j];
  if (keep != 0xFu) {  // the slice's first or last quad, or a lane past the chunk
#pragma unroll
    for (int j = 0; j < 4; ++j) wq[j] = ((keep >> j) & 1u) ? wq[j] : 0u;
  }
  if (ev.narrow) {
    uint32_t p[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      p[j] = (uint32_t)__umul24(wq[j], f[j]);  // (HIP's __umul24 returns an int)
      out[j] = p[j];
    }
    sum = (uint64_t)((p[0] + p[1]) + (p[2] + p[3]));  // four products below 2^24
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = (uint64_t)wq[j] * f[j];
    sum = (out[0] + out[1]) + (out[2] + out[3]);
  }
}

// Pass 1 of a node2vec hop by merging the sorted rows, one chunk after the
// other with a cursor into N(prev) that only moves forward.  Lane g returns
// the total of group g (the layout of GroupSplit) and in gcur the cursor at
// the start of group g, from which the group can be merged again.
template <class E>
__device__ __forceinline__ uint64_t merge_group_totals(const E& ev, const QuadSlice& s,
                                                       const GroupSplit& sp, const Table& tb,
                                                       int lane, uint64_t& gcur) {
  uint64_t cursor = 0;  // entries of N(prev) below every key still to come
  uint64_t mine = 0;
  gcur = 0;
  for (uint32_t g = 0; g < sp.groups; ++g) {
    const uint32_t gb = g * sp.gsz;
    const uint32_t ge = min(gb + sp.gsz, s.nq);
    if ((uint32_t)lane == g) gcur = cursor;
    uint64_t acc = 0;
    for (uint32_t c0 = gb; c0 < ge; c0 += kWave) {
      uint64_t w[4], t;
      merge_chunk(ev, s, tb, c0, ge, cursor, lane, w, t);
      acc += t;
    }
    const uint64_t tot = wave_sum(acc);
    if ((uint32_t)lane == g) mine = tot;
  }
  return mine;
}

// Lower bound of u in the sorted run row[0, n), n >= 1: the first index
// whose entry is >= u (n if none).  One trip count for every lane (n is
// wave-uniform), each probe a load from the run's uniform base.
__device__ __forceinline__ uint32_t row_lower_bound(const uint32_t* __restrict__ row, uint32_t n,
                                                    uint32_t u) {
  uint32_t base = 0, len = n;
  while (len > 1) {  // the lower bound is in [base, base + len]
    const uint32_t half = len >> 1;
    base = row_at(row, base + half) < u ? base + half : base;
    len -= half;
  }
  return base + (row_at(row, base) < u ? 1u : 0u);
}

// Pass 1 of a node2vec hop whose N(prev) is much shorter than N(cur), by the
// identity (Eq. 2, weights w_i over N(cur))
//   T_g = f_out * sum_{i in g} w_i + (f_in - f_out) * sum_{i in g, u_i in N(prev), u_i != prev} w_i
//                                  + (f_ret - f_out) * sum_{i in g, u_i = prev} w_i
// for every group g of GroupSplit: the first sum streams the weights alone
// (entry counts when the graph has none) and never reads N(cur)'s ids; the
// other two look each distinct key of N(prev), and prev itself, up in N(cur)
// by binary search and add the weights they find (all entries of a repeated
// id) to their group in LDS.  Arithmetic is modulo 2^64, exact because every
// T_g is below 2^64.  Lane g returns T_g.  Uses the wavefront's LDS region.
template <class E>
__device__ __forceinline__ uint64_t sparse_prev_group_totals(const E& ev, const QuadSlice& s,
                                                             const GroupSplit& sp,
                                                             const Table& tb, int lane) {
  // Raw totals.
  const char* __restrict__ wrun = reinterpret_cast<const char*>(ev.w + s.a);
  auto quad_raw = [wrun](uint32_t q) { return *reinterpret_cast<const uint4*>(wrun + q * 16u); };
  uint64_t raw = 0;
  if (ev.w != nullptr) {
    for (uint32_t g = 0; g < sp.groups; ++g) {
      const uint32_t gb = g * sp.gsz;
      const uint32_t ge = min(gb + sp.gsz, s.nq);
      uint64_t acc = 0;
      uint32_t q = gb + lane;
#pragma unroll 1
      for (; q + 3 * kWave < ge; q += 4 * kWave) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = quad_raw(q + k * kWave);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += raw_quad_sum(s, q + k * kWave, v[k]);
      }
#pragma unroll 1
      for (; q < ge; q += kWave) acc += raw_quad_sum(s, q, quad_raw(q));
      const uint64_t tot = wave_sum(acc);
      if ((uint32_t)lane == g) raw = tot;
    }
  } else if ((uint32_t)lane < sp.groups) {
    const uint32_t gb = (uint32_t)lane * sp.gsz;
    const uint32_t ge = min(gb + sp.gsz, s.nq);
    uint32_t cnt = 4 * (ge - gb);
    if (gb == 0) cnt -= s.lead;
    if (ge == s.nq) cnt -= 4 * s.nq - s.lead - s.d;
    raw = cnt;
  }
  // Corrections, one 64-bit LDS cell per group.
  unsigned long long* corr = reinterpret_cast<unsigned long long*>(fw_dyn_lds + tb.base);
  corr[lane] = 0ull;
  wave_sync_lds();
  const uint32_t* __restrict__ crow = ev.adj + s.o;  // N(cur)
  const uint32_t* __restrict__ prow = ev.adj + tb.po;  // N(prev)
  const uint64_t d_in = (uint64_t)ev.f_in - (uint64_t)ev.f_out;
  const uint64_t d_ret = (uint64_t)ev.f_ret - (uint64_t)ev.f_out;
  const uint32_t gq = sp.gsz;
  // Round c: lane k looks up entry c + k of N(prev).
  for (uint64_t c = 0; c < tb.pd; c += kWave) {
    const uint64_t i = c + (uint64_t)lane;
    const uint32_t u = i < tb.pd ? prow[i] : 0u;
    // Repeated ids count once; prev's own id is a return, not a neighbour.
    const bool want = i < tb.pd && u != ev.prev && (i == 0 || prow[i - 1] != u);
    if (!ballot(want)) continue;
    uint32_t pos = row_lower_bound(crow, s.d, u);
    if (want) {
      for (; pos < s.d && row_at(crow, pos) == u; ++pos) {
        const uint32_t wt = ev.w != nullptr ? ev.w[s.o + pos] : 1u;
        atomicAdd(&corr[((s.lead + pos) >> 2) / gq], (unsigned long long)(d_in * wt));
      }
    }
  }
  // Entries equal to prev (the return).
  if (lane == 0) {
    for (uint32_t pos = row_lower_bound(crow, s.d, ev.prev);
         pos < s.d && row_at(crow, pos) == ev.prev; ++pos) {
      const uint32_t wt = ev.w != nullptr ? ev.w[s.o + pos] : 1u;
      atomicAdd(&corr[((s.lead + pos) >> 2) / gq], (unsigned long long)(d_ret * wt));
    }
  }
  wave_sync_lds();
  const uint64_t mine = (uint64_t)ev.f_out * raw + (uint64_t)corr[lane];
  wave_sync_lds();
  return (uint32_t)lane < sp.groups ? mine : 0ull;
}

template <int ALGO, bool WEIGHTED, class MEM>
__device__ __forceinline__ Eval<ALGO, WEIGHTED, MEM> base_eval(const DevGraph& g,
                                                              const DevParams& prm, uint64_t o,
                                                              uint32_t prev, uint32_t t) {
  Eval<ALGO, WEIGHTED, MEM> ev;
  ev.adj = g.adj;
  ev.w = g.w;
  ev.lab = g.lab;
  ev.o = o;
  ev.first = (t == 0);
  ev.prev = prev;
  ev.f_ret = prm.f_ret;
  ev.f_in = prm.f_in;
  ev.f_out = prm.f_out;
  ev.want = (ALGO == kMetaPath) ? schema_label(prm, t) : 0u;
  ev.qa = 0;
  ev.narrow = false;
  return ev;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(v >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Request access: a single request passed by value, or a table of requests
// (binary search of the query-count prefix maps a global index to its
// request).
template <bool MULTI>
struct Reqs {
  ReqDesc one;
  ReqTable tab;
  __device__ __forceinline__ uint64_t total() const { return MULTI ? tab.total : one.n; }
  __device__ __forceinline__ uint32_t find(uint64_t q) const {
    if (!MULTI) return 0;
    uint32_t lo = 0, hi = tab.nreq;  // last r with prefix[r] <= q
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (tab.prefix[mid] <= q)
        lo = mid;
      else
        hi = mid;
    }
    return lo;
  }
  __device__ __forceinline__ uint64_t first(uint32_t r) const {
    return MULTI ? tab.prefix[r] : 0;
  }
  __device__ __forceinline__ ReqDesc get(uint32_t r) const { return MULTI ? tab.reqs[r] : one; }
};

// Served form: a retired query adds its realised hops to its request's
// counter (one atomic per query).
__device__ __forceinline__ void count_steps(const ReqDesc& R, uint32_t hops) {
  if (R.steps != nullptr && hops != 0) atomicAdd(R.steps, (unsigned long long)hops);
}

// Eight wavefronts per SIMD (64 VGPRs): the walk is bound by the latency of
// dependent loads (offsets, then the slice, then the LDS membership probes),
// so occupancy pays more than the few per-hop register spills it costs.
template <int ALGO, bool WEIGHTED, bool MULTI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void
k_walk_persistent(
    DevGraph g, Reqs<MULTI> rq, uint32_t* __restrict__ status, uint64_t* __restrict__ head,
    TuneCfg cfg) {
  const int lane = lane_id();
  const int grp = lane / kGroupLanes, gl = lane % kGroupLanes;
  const uint64_t n = rq.total();
  Table tb;
  tb.cells = cfg.hash_cells;
  tb.base = (threadIdx.x / kWave) * cfg.hash_cells;
  tb.kind = 0;

  // This group's query (identical in the 16 lanes of the group): request r,
  // index in the request, vertex state.
  uint64_t s_qid = 0, s_o = 0, s_d = 0;
  uint32_t s_cur = kEnd, s_prev = kEnd, s_t = 0, s_r = 0;
  bool s_live = false;
  bool exhausted = false;

  for (;;) {
    // ---- refill: claim one query for every empty group ----------------
    if (!exhausted) {
      const uint64_t empty_m = ballot(!s_live && gl == 0);
      const uint32_t empty = __builtin_popcountll(empty_m);
      if (empty) {
        uint64_t base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)head, (unsigned long long)empty);
        base = readlane64(base, 0);
        if (base + empty >= n) exhausted = true;
        if (!s_live) {
          const uint32_t rank =
              __builtin_popcountll(empty_m & ((1ull << (grp * kGroupLanes)) - 1));
          const uint64_t q = base + rank;
          if (q < n) {
            const uint32_t r = rq.find(q);
            const ReqDesc R = rq.get(r);
            const uint64_t lq = q - rq.first(r);
            const uint32_t st = R.starts[lq];
            if (st >= g.nv) {
              if (gl == 0) atomicOr(status, 1u);
            } else {
              if (gl == 0) R.out[lq * ((uint64_t)R.length + 1)] = st;
              if (R.length > 0) {
                s_r = r;
                s_qid = lq;
                s_cur = st;
                s_prev = kEnd;
                s_t = 0;
                s_live = true;
              }
            }
          }
          // An invalid or length-0 query leaves its group empty; the next
          // round claims again.
        }
      }
    }
    if (!ballot(s_live)) {
      if (exhausted) break;
      continue;
    }
    if (s_live) {
      s_o = g.off[s_cur];
      s_d = g.off[s_cur + 1] - s_o;
      // A PPR stop ends the query like a dead end: the tiny path pads it.
      if (ALGO == kPPR) {
        const ReqDesc R = rq.get(s_r);
        if (ppr_stops(R.prm, R.seed, R.qid_base + s_qid, s_t)) s_d = 0;
      }
    }

    // ---- tiny hops: one per 16-lane group ------------------------------
    const bool tiny = s_live && s_d <= cfg.tiny_max;
    if (ballot(tiny)) {
      const ReqDesc R = rq.get(tiny ? s_r : 0);
      const DevParams& prm = R.prm;
      const uint32_t length = R.length;
      const uint64_t row_len = (uint64_t)length + 1;
      auto ev = base_eval<ALGO, WEIGHTED, MemberGlobal>(g, prm, tiny ? s_o : 0,
                                                        tiny ? s_prev : kEnd, tiny ? s_t : 0);
      ev.mem.adj = g.adj;
      ev.mem.po = 0;
      ev.mem.pd = 0;
      if (ALGO == kNode2Vec && tiny && s_t > 0) {
        ev.mem.po = g.off[s_prev];
        ev.mem.pd = g.off[s_prev + 1] - ev.mem.po;
      }
      const bool valid = tiny && (uint64_t)gl < s_d;
      uint64_t x = valid ? ev(gl) : 0ull;
      x += dpp64<0x111, 0xF>(x);  // inclusive scan inside each 16-lane row
      x += dpp64<0x112, 0xF>(x);
      x += dpp64<0x114, 0xF>(x);
      x += dpp64<0x118, 0xF>(x);
      const uint64_t total = shfl64(x, lane | 15);
      const uint64_t u = philox_draw(R.seed, R.qid_base + s_qid, s_t);
      const uint64_t r = scale_draw(u, total);
      const uint64_t m = ballot(valid && x > r);
      const uint32_t gm = (uint32_t)(m >> (grp * kGroupLanes)) & 0xFFFFu;
      if (tiny) {
        uint32_t* row = R.out + s_qid * row_len;
        if (total == 0) {
          for (uint32_t p = s_t + 1 + gl; p <= length; p += kGroupLanes) row[p] = kEnd;
          s_live = false;
          if (MULTI && gl == 0) count_steps(R, s_t);
        } else {
          const uint32_t next = g.adj[s_o + (gm ? __builtin_ctz(gm) : 0)];
          if (gl == 0) row[s_t + 1] = next;
          s_prev = s_cur;
          s_cur = next;
          s_t += 1;
          if (s_t == length) {
            s_live = false;
            if (MULTI && gl == 0) count_steps(R, length);
          }
        }
      }
    }

    // ---- other hops: one at a time on the whole wavefront --------------
    uint64_t big = ballot(s_live && !tiny && gl == 0);
    while (big) {
      const int src = first_lane(big);
      big &= big - 1;
      const uint64_t qid = readlane64(s_qid, src), o = readlane64(s_o, src),
                     d = readlane64(s_d, src);
      const uint32_t t = readlane32(s_t, src), prev = readlane32(s_prev, src);
      const ReqDesc R = rq.get(readlane32(s_r, src));
      const DevParams& prm = R.prm;
      const uint32_t length = R.length;
      tb.kind = 0;
      tb.po = tb.pd = 0;
      if (ALGO == kNode2Vec && t > 0) {
        // Wave-uniform: kept in scalar registers.
        tb.po = uniform64(g.off[prev]);
        tb.pd = uniform64(g.off[prev + 1]) - tb.po;
        // N(prev) much shorter than N(cur): look its keys up in N(cur)
        // instead of testing every entry of N(cur) against it.
        if (cfg.sparse_ratio != 0 && d >= kSparseMinDegree && tb.cells >= 2 * kWave &&
            (uint64_t)cfg.sparse_ratio * tb.pd <= d)
          tb.kind = 3;
        else
          build_table(tb, g.adj, d, lane);
      }
      const uint64_t u = philox_draw(R.seed, R.qid_base + qid, t);
      auto ev = base_eval<ALGO, WEIGHTED, MemberAny>(g, prm, o, prev, t);
      ev.narrow = cfg.narrow != 0;
      ev.mem.mode = tb.kind == 1 ? 1 : 0;
      ev.mem.base = tb.base;
      ev.mem.bmask = tb.bmask;
      ev.mem.shift = tb.shift;
      ev.mem.adj = g.adj;
      ev.mem.po = tb.po;
      ev.mem.pd = tb.pd;
      int64_t idx;
      if (ALGO == kNode2Vec && (tb.kind == 2 || tb.kind == 3)) {
        // Pass 1 by merging the sorted rows (kind 2), or from raw weights
        // and N(prev)'s keys looked up in N(cur) (kind 3).  The locate
        // evaluates the drawn group's entries one by one: a one-chunk group
        // of the merge is merged again from its cursor; otherwise against a
        // hash set of N(prev) (kind 3, when it fits) or by binary searches.
        const QuadSlice qs(o, d);
        const GroupSplit sp(qs.nq);
        const bool sparse = tb.kind == 3;
        uint64_t gcur = 0;
        const uint64_t mine = sparse ? sparse_prev_group_totals(ev, qs, sp, tb, lane)
                                     : merge_group_totals(ev, qs, sp, tb, lane, gcur);
        const uint64_t incl = wave_incl_scan(mine);
        const uint64_t total = readlane64(incl, kWave - 1);
        idx = -1;
        if (total != 0) {
          uint64_t r = scale_draw(u, total);
          const uint64_t m = ballot(incl > r);
          const int gs = m ? first_lane(m) : (int)sp.groups - 1;
          r -= readlane64(incl - mine, gs);
          const uint32_t lo = (uint32_t)gs * sp.gsz;
          const uint32_t len = min(sp.gsz, qs.nq - lo);
          if (!sparse && len <= (uint32_t)kWave) {
            // A one-chunk group (rows up to 16,384 entries).
            uint64_t cur = readlane64(gcur, gs);
            uint64_t w[4], t;
            merge_chunk(ev, qs, tb, lo, lo + len, cur, lane, w, t);
            idx = pick_in_quads(w, qs, lo, len, r, true, 0);
          } else {
            if (sparse) {
              build_table(tb, g.adj, d, lane, false);
              ev.mem.mode = tb.kind == 1 ? 1 : 0;
              ev.mem.bmask = tb.bmask;
              ev.mem.shift = tb.shift;
            }
            idx = (int64_t)wave_locate(ev, qs, lo, len, r);
          }
        }
      } else {
        idx = wave_pick(ev, o, d, u);
      }
      uint32_t* row = R.out + qid * ((uint64_t)length + 1);
      const bool mine = grp == src / kGroupLanes;
      if (idx < 0) {
        for (uint32_t p = t + 1 + lane; p <= length; p += kWave) row[p] = kEnd;
        if (mine) s_live = false;
        if (MULTI && lane == src) count_steps(R, t);
      } else {
        const uint32_t next = g.adj[o + (uint64_t)idx];
        if (lane == 0) row[t + 1] = next;
        if (mine) {
          s_prev = s_cur;
          s_cur = next;
          s_t += 1;
          if (s_t == length) s_live = false;
        }
        if (MULTI && lane == src && t + 1 == length) count_steps(R, length);
      }
      wave_sync_lds();
    }
  }
}

__global__ void k_reset_counter(uint64_t* p) { *p = 0; }

template <int ALGO, bool W, bool MULTI>
static hipError_t go(const DevGraph& g, const Reqs<MULTI>& rq, uint32_t* status, uint64_t* head,
                     const TuneCfg& cfg, unsigned blocks, hipStream_t stream) {
  const size_t lds = (size_t)cfg.hash_cells * sizeof(uint32_t) * (kBlock / kWave);
  hipLaunchKernelGGL((k_walk_persistent<ALGO, W, MULTI>), dim3(blocks), dim3(kBlock), lds,
                     stream, g, rq, status, head, cfg);
  return hipGetLastError();
}

template <bool MULTI>
static hipError_t launch_any(int algo, const DevGraph& g, const Reqs<MULTI>& rq, uint32_t* status,
                             uint64_t* head, int num_cus, const TuneCfg& c, uint64_t n,
                             hipStream_t stream) {
  if (c.tiny_max > 16 || c.wgs_per_cu == 0 || c.hash_cells < 64 ||
      (c.hash_cells & (c.hash_cells - 1)) || head == nullptr)
    return hipErrorInvalidValue;
  uint64_t blocks = (uint64_t)num_cus * c.wgs_per_cu;
  const uint64_t per_block = (kBlock / kWave) * kGroups;
  const uint64_t need = (n + per_block - 1) / per_block;
  if (blocks > need) blocks = need;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, stream, head);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool wt = g.w != nullptr;
  const unsigned b = (unsigned)blocks;
  switch (algo) {
    case kDeepWalk:
      return wt ? go<kDeepWalk, true>(g, rq, status, head, c, b, stream)
                : go<kDeepWalk, false>(g, rq, status, head, c, b, stream);
    case kNode2Vec:
      return wt ? go<kNode2Vec, true>(g, rq, status, head, c, b, stream)
                : go<kNode2Vec, false>(g, rq, status, head, c, b, stream);
    case kMetaPath:
      return wt ? go<kMetaPath, true>(g, rq, status, head, c, b, stream)
                : go<kMetaPath, false>(g, rq, status, head, c, b, stream);
    case kPPR:
      return wt ? go<kPPR, true>(g, rq, status, head, c, b, stream)
                : go<kPPR, false>(g, rq, status, head, c, b, stream);
    default:
      return hipErrorInvalidValue;
  }
}

// Enqueues (reset head; persistent kernel) on `stream`.
hipError_t launch_persistent(const LaunchArgs& a, hipStream_t stream) {
  Reqs<false> rq;
  rq.one.starts = a.starts;
  rq.one.out = a.out;
  rq.one.steps = nullptr;
  rq.one.n = a.n;
  rq.one.seed = a.seed;
  rq.one.qid_base = a.qid_base;
  rq.one.length = a.length;
  rq.one.pad = 0;
  rq.one.prm = a.prm;
  rq.tab = ReqTable{nullptr, nullptr, 0, 0};
  return launch_any<false>(a.algo, a.g, rq, a.status, a.head, a.num_cus, a.cfg, a.n, stream);
}

hipError_t launch_persistent_multi(int algo, const DevGraph& g, const ReqTable& t,
                                   uint32_t* status, uint64_t* head, int num_cus,
                                   const TuneCfg& cfg, hipStream_t stream) {
  Reqs<true> rq;
  std::memset(&rq.one, 0, sizeof(rq.one));
  rq.tab = t;
  return launch_any<true>(algo, g, rq, status, head, num_cus, cfg, t.total, stream);
}

}  // namespace fw
