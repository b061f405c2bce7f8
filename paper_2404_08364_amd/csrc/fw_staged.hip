// Workgroup-staged persistent walker: the paper's two-stage block design
// (sections 5.1 and 5.2) mapped onto wave64 workgroups (FW_MODE_STAGED).
//
// A fixed grid of workgroups stays resident.  Each workgroup keeps a local
// task pool of `slots` live queries in LDS (query id, current and previous
// vertex, hop index, cached CSR range) and refills empty slots from the
// global task pool with one 64-bit atomicAdd on a head counter per refill.
// Every iteration advances every live query by one hop, in two stages:
//   stage A  tiny hops (degree <= tiny_max <= 16) run four to a wavefront on
//            16-lane groups; mid-degree hops run one per wavefront;
//   stage B  hub hops (degree >= hub_min) run one at a time on the whole
//            workgroup: each wavefront streams a contiguous part of the
//            neighbour slice and leaves 64 group totals in LDS, one
//            wavefront scans the totals, draws, and locates the pick inside
//            the chosen group.
// Node2vec membership tests against N(prev) use an open-addressing hash set
// of N(prev) built in LDS for the hop (per wavefront in stage A, per
// workgroup in stage B) when it fits, and binary search of the sorted row in
// global memory otherwise.  No global memory beyond the inputs, the output
// paths and one head counter is used.
#include "fw_kernels.h"
#include "fw_wave_sampler.h"

namespace fw {
namespace staged {

extern __shared__ __attribute__((aligned(16))) uint32_t fw_dyn_lds[];  // hash sets (u32 cells)

constexpr int kMaxSlots = 128;
constexpr int kMaxWaves = 16;
constexpr uint32_t kFib = 0x9E3779B1u;

struct PoolLds {
  uint64_t qid[kMaxSlots];
  uint64_t o[kMaxSlots];
  uint64_t d[kMaxSlots];
  uint32_t cur[kMaxSlots];
  uint32_t prev[kMaxSlots];
  uint32_t t[kMaxSlots];
  uint32_t live[kMaxSlots];
  uint16_t tiny[kMaxSlots], mid[kMaxSlots], hub[kMaxSlots];
  uint32_t n_tiny, n_mid, n_hub, next_tiny, next_mid, exhausted;
  uint64_t gt[kMaxWaves * kWave];  // hub pass-1 group totals
};

// Hash set of the ids of N(prev) in LDS: nb buckets of 4 cells (16 bytes) at
// fw_dyn_lds[base, base + 4 * nb); kEnd marks an empty cell.  A key lives in
// the first bucket, in probe order from its hash, that had a free cell when it
// was inserted, so a lookup stops at a hit or at a bucket with a free cell.
// The load factor is at most 1/2, so one 16-byte read answers almost every
// lookup.
struct MemberLds {
  uint32_t base, bmask, shift;
  __device__ __forceinline__ bool contains(uint32_t u) const {
    uint32_t b = (u * kFib) >> shift;
    for (;;) {
      const uint4 v = *reinterpret_cast<const uint4*>(&fw_dyn_lds[base + 4 * b]);
      const bool hit = (v.x == u) | (v.y == u) | (v.z == u) | (v.w == u);
      const bool open = (v.x == kEnd) | (v.y == kEnd) | (v.z == kEnd) | (v.w == kEnd);
      if (hit | open) return hit;
      b = (b + 1) & bmask;
    }
  }
  // f[j] = fin if u[j] is in the set, else fout.
  __device__ __forceinline__ void factors4(const uint32_t u[4], uint32_t fin, uint32_t fout,
                                           uint32_t f[4]) const {
#pragma unroll
    for (int j = 0; j < 4; ++j) f[j] = contains(u[j]) ? fin : fout;
  }
};

struct HashTable {
  uint32_t base, bmask, shift;
  const uint32_t* adj;
  uint64_t po, pd;
};

__device__ __forceinline__ uint32_t log2_ceil(uint64_t x) {
  uint32_t b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// Sizes the table for n keys: 4-cell buckets, load factor <= 1/2, at least
// 16 buckets.  Returns the number of cells.
__device__ __forceinline__ uint32_t hash_geometry(uint64_t n, HashTable& h) {
  uint32_t bits = log2_ceil((2 * n + 3) / 4);
  if (bits < 4) bits = 4;
  h.bmask = (1u << bits) - 1;
  h.shift = 32 - bits;
  return 4u << bits;
}

// Builds the set with threads [tix, tix + nthr) of the caller; the caller
// synchronises between clear and insert and after insert.
__device__ __forceinline__ void hash_clear(const HashTable& h, int tix, int nthr) {
  const uint32_t cells = 4 * (h.bmask + 1);
  for (uint32_t i = tix; i < cells; i += nthr) fw_dyn_lds[h.base + i] = kEnd;
}

__device__ __forceinline__ void hash_insert(const HashTable& h, int tix, int nthr) {
  for (uint64_t i = tix; i < h.pd; i += nthr) {
    const uint32_t u = h.adj[h.po + i];
    uint32_t b = (u * kFib) >> h.shift;
    for (;;) {
      uint32_t j = 0;
      for (; j < 4; ++j) {
        const uint32_t old = atomicCAS(&fw_dyn_lds[h.base + 4 * b + j], kEnd, u);
        if (old == kEnd || old == u) break;
      }
      if (j < 4) break;
      b = (b + 1) & h.bmask;
    }
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
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
  return ev;
}

// Size of N(prev) for a node2vec hop (0 when membership is not needed).
template <int ALGO>
__device__ __forceinline__ void prev_row(const DevGraph& g, uint32_t prev, uint32_t t,
                                         uint64_t* po, uint64_t* pd) {
  *po = 0;
  *pd = 0;
  if (ALGO == kNode2Vec && t > 0) {
    *po = g.off[prev];
    *pd = g.off[prev + 1] - *po;
  }
}

// Calls f(ev) with the evaluator type that fits the hop: the first node2vec
// hop weighs like DeepWalk; later node2vec hops test membership in the LDS
// hash set when `h` is built (h.pd > 0 and use_lds), else by binary search.
template <int ALGO, bool WEIGHTED, class F>
__device__ __forceinline__ void with_eval(const DevGraph& g, const DevParams& prm, uint64_t o,
                                          uint32_t prev, uint32_t t, const HashTable& h,
                                          bool use_lds, F&& f) {
  if (ALGO == kNode2Vec) {
    if (t == 0) {
      f(base_eval<kDeepWalk, WEIGHTED, MemberGlobal>(g, prm, o, prev, t));
    } else if (use_lds) {
      auto ev = base_eval<kNode2Vec, WEIGHTED, MemberLds>(g, prm, o, prev, t);
      ev.mem.base = h.base;
      ev.mem.bmask = h.bmask;
      ev.mem.shift = h.shift;
      f(ev);
    } else {
      auto ev = base_eval<kNode2Vec, WEIGHTED, MemberGlobal>(g, prm, o, prev, t);
      ev.mem.adj = g.adj;
      ev.mem.po = h.po;
      ev.mem.pd = h.pd;
      f(ev);
    }
  } else {
    f(base_eval<ALGO, WEIGHTED, MemberGlobal>(g, prm, o, prev, t));
  }
}

// Records hop t -> next of slot s (lane `l` of `nl` cooperating lanes), or
// pads the row with kEnd after a dead end.  Slot state changes by l == 0.
__device__ __forceinline__ void advance(PoolLds& P, int s, bool dead, uint32_t next,
                                        uint32_t length, uint32_t* __restrict__ out, int l,
                                        int nl) {
  const uint64_t q = P.qid[s];
  const uint32_t t = P.t[s];
  uint32_t* row = out + q * ((uint64_t)length + 1);
  if (dead) {
    for (uint32_t p = t + 1 + l; p <= length; p += nl) row[p] = kEnd;
    if (l == 0) P.live[s] = 0;
  } else if (l == 0) {
    row[t + 1] = next;
    P.prev[s] = P.cur[s];
    P.cur[s] = next;
    P.t[s] = t + 1;
    if (t + 1 == length) P.live[s] = 0;
  }
}

// Wave part of a 64-bit value from lane `src` (any lane of the wavefront).
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(v >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Pass-1 partition of a hub slice of nq quads: wavefront w owns 64-quad
// chunks [c0, c1).
struct HubPart {
  uint32_t lo, len;
  __device__ __forceinline__ HubPart(uint32_t nq, int w, int nw) {
    const uint32_t chunks = (nq + kWave - 1) / kWave;
    const uint32_t c0 = chunks * w / nw, c1 = chunks * (w + 1) / nw;
    lo = c0 * kWave;
    const uint32_t hi = min(c1 * kWave, nq);
    len = hi > lo ? hi - lo : 0;
  }
};

// One hub hop on the whole workgroup (every thread calls it).  Pass 1: each
// wavefront streams its part of the slice and leaves 64 group totals in LDS;
// then wavefront 0 scans the NW * 64 totals, draws, and locates the pick in
// the chosen group.
template <int NW, class E>
__device__ __forceinline__ void hub_hop(const E& ev, PoolLds& P, int s, uint64_t o, uint64_t d,
                                        uint64_t seed, uint64_t qid, uint32_t t,
                                        const uint32_t* __restrict__ adj, uint32_t length,
                                        uint32_t* __restrict__ out, int wave, int lane) {
  const QuadSlice qs(o, d);
  {
    const HubPart part(qs.nq, wave, NW);
    uint64_t mine = 0;
    if (part.len)
      mine = wave_group_totals(bind_quads(ev, qs), qs, part.lo, part.len, GroupSplit(part.len));
    P.gt[wave * kWave + lane] = mine;
  }
  __syncthreads();
  if (wave != 0) return;
  // Lane j owns the NW consecutive group totals [j*NW, j*NW + NW).
  uint64_t sj = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) sj += P.gt[lane * NW + i];
  const uint64_t incl = wave_incl_scan(sj);
  const uint64_t total = readlane64(incl, kWave - 1);
  const bool dead = (total == 0);
  uint32_t next = kEnd;
  if (!dead) {
    uint64_t r = scale_draw(philox_draw(seed, qid, t), total);
    const uint64_t m = ballot(incl > r);
    const int j = m ? first_lane(m) : kWave - 1;
    r -= readlane64(incl - sj, j);
    int e = j * NW + NW - 1;
    for (int i = 0; i < NW; ++i) {
      const uint64_t v = P.gt[j * NW + i];
      if (r < v) {
        e = j * NW + i;
        break;
      }
      r -= v;
    }
    const HubPart part(qs.nq, e / kWave, NW);
    const GroupSplit sp(part.len);
    const uint32_t gi = (uint32_t)(e % kWave);
    const uint32_t gb = part.lo + gi * sp.gsz;
    const uint32_t glen = min(sp.gsz, part.len - gi * sp.gsz);
    const uint64_t idx = wave_locate(ev, qs, gb, glen, r);
    next = adj[o + idx];
  }
  advance(P, s, dead, next, length, out, lane, kWave);
}

template <int ALGO, bool WEIGHTED, int NW>
__global__ __launch_bounds__(NW* kWave) void k_walk_persistent(
    DevGraph g, DevParams prm, const uint32_t* __restrict__ starts, uint64_t n, uint32_t length,
    uint64_t seed, uint64_t qid_base, uint32_t* __restrict__ out, uint32_t* __restrict__ status,
    uint64_t* __restrict__ head, TuneCfg cfg, uint32_t hash_cells) {
  __shared__ PoolLds P;
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  constexpr int NT = NW * kWave;
  const int S = (int)cfg.slots;
  const uint32_t wave_cells = hash_cells / NW;  // per-wavefront table in stage A

  for (int i = tid; i < S; i += NT) P.live[i] = 0;
  if (tid == 0) P.exhausted = 0;
  __syncthreads();

  for (;;) {
    // ---- refill empty slots from the global pool (wavefront 0) ----------
    if (wave == 0 && !P.exhausted) {
      uint32_t empty = 0;
      for (int s0 = 0; s0 < S; s0 += kWave) {
        const int s = s0 + lane;
        empty += __builtin_popcountll(ballot(s < S && !P.live[s]));
      }
      if (empty) {
        uint64_t base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)head, (unsigned long long)empty);
        base = readlane64(base, 0);
        uint32_t rank0 = 0;
        for (int s0 = 0; s0 < S; s0 += kWave) {
          const int s = s0 + lane;
          const bool emp = s < S && !P.live[s];
          const uint64_t m = ballot(emp);
          if (emp) {
            const uint64_t q = base + rank0 + __builtin_popcountll(m & ((1ull << lane) - 1));
            if (q < n) {
              const uint32_t st = starts[q];
              if (st >= g.nv) {
                atomicOr(status, 1u);
              } else {
                out[q * ((uint64_t)length + 1)] = st;
                if (length > 0) {
                  P.qid[s] = q;
                  P.cur[s] = st;
                  P.prev[s] = kEnd;
                  P.t[s] = 0;
                  P.live[s] = 1;
                }
              }
            }
          }
          rank0 += __builtin_popcountll(m);
        }
        if (lane == 0 && base + empty >= n) P.exhausted = 1;
      }
    }
    if (tid == 0) {
      P.n_tiny = P.n_mid = P.n_hub = 0;
      P.next_tiny = P.next_mid = 0;
    }
    __syncthreads();

    // ---- classify live slots by degree ---------------------------------
    for (int s = tid; s < S; s += NT) {
      if (!P.live[s]) continue;
      const uint32_t c = P.cur[s];
      const uint64_t o = g.off[c];
      uint64_t d = g.off[c + 1] - o;
      // A PPR stop ends the query like a dead end (the tiny stage pads it).
      if (ALGO == kPPR && ppr_stops(prm, seed, qid_base + P.qid[s], P.t[s])) d = 0;
      P.o[s] = o;
      P.d[s] = d;
      if (d <= cfg.tiny_max)
        P.tiny[atomicAdd(&P.n_tiny, 1u)] = (uint16_t)s;
      else if (d < cfg.hub_min)
        P.mid[atomicAdd(&P.n_mid, 1u)] = (uint16_t)s;
      else
        P.hub[atomicAdd(&P.n_hub, 1u)] = (uint16_t)s;
    }
    __syncthreads();
    const uint32_t nt = P.n_tiny, nm = P.n_mid, nh = P.n_hub;
    if (nt + nm + nh == 0 && P.exhausted) break;

    // ---- stage A: tiny hops, four per wavefront (16-lane groups) -------
    for (;;) {
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(&P.next_tiny, 4u);
      k = readlane32(k, 0);
      if (k >= nt) break;
      const int grp = lane >> 4, l16 = lane & 15;
      const bool has = k + grp < nt;
      const int s = has ? P.tiny[k + grp] : 0;
      // Lanes of a group without a task use a neutral state (no loads).
      const uint64_t o = has ? P.o[s] : 0, d = has ? P.d[s] : 0;
      const uint32_t t = has ? P.t[s] : 0, prev = has ? P.prev[s] : kEnd;
      const uint64_t qid = has ? P.qid[s] : 0;
      auto ev = base_eval<ALGO, WEIGHTED, MemberGlobal>(g, prm, o, prev, t);
      ev.mem.adj = g.adj;
      prev_row<ALGO>(g, prev, t, &ev.mem.po, &ev.mem.pd);
      const bool valid = (uint64_t)l16 < d;
      uint64_t x = valid ? ev(l16) : 0ull;
      x += dpp64<0x111, 0xF>(x);  // inclusive scan inside each 16-lane row
      x += dpp64<0x112, 0xF>(x);
      x += dpp64<0x114, 0xF>(x);
      x += dpp64<0x118, 0xF>(x);
      const uint64_t total = shfl64(x, lane | 15);
      const uint64_t u = philox_draw(seed, qid_base + qid, t);
      const uint64_t r = scale_draw(u, total);
      const uint64_t m = ballot(valid && total > 0 && x > r);
      const uint32_t gm = (uint32_t)(m >> (grp * 16)) & 0xFFFFu;
      const uint32_t idx = gm ? (uint32_t)__builtin_ctz(gm) : 0u;
      const bool dead = (total == 0);
      const uint32_t next = (has && !dead) ? g.adj[o + idx] : kEnd;
      if (has) advance(P, s, dead, next, length, out, l16, 16);
    }

    // ---- stage A: mid-degree hops, one per wavefront -------------------
    for (;;) {
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(&P.next_mid, 1u);
      k = readlane32(k, 0);
      if (k >= nm) break;
      const int s = P.mid[k];
      const uint64_t o = P.o[s], d = P.d[s];
      const uint32_t t = P.t[s], prev = P.prev[s];
      HashTable h;
      h.adj = g.adj;
      h.base = wave * wave_cells;
      prev_row<ALGO>(g, prev, t, &h.po, &h.pd);
      bool use_lds = false;
      if (ALGO == kNode2Vec && t > 0 && 2 * h.pd <= wave_cells && h.pd <= 4 * d) {
        hash_geometry(h.pd, h);
        hash_clear(h, lane, kWave);
        wave_sync_lds();
        hash_insert(h, lane, kWave);
        wave_sync_lds();
        use_lds = true;
      }
      const uint64_t u = philox_draw(seed, qid_base + P.qid[s], t);
      int64_t idx = -1;
      with_eval<ALGO, WEIGHTED>(g, prm, o, prev, t, h, use_lds,
                                [&](const auto& ev) { idx = wave_pick(ev, o, d, u); });
      const uint32_t next = idx >= 0 ? g.adj[o + (uint64_t)idx] : kEnd;
      advance(P, s, idx < 0, next, length, out, lane, kWave);
      wave_sync_lds();
    }
    __syncthreads();

    // ---- stage B: hub hops, one at a time on the whole workgroup -------
    for (uint32_t k = 0; k < nh; ++k) {
      const int s = P.hub[k];
      const uint64_t o = P.o[s], d = P.d[s];
      const uint32_t t = P.t[s], prev = P.prev[s];
      HashTable h;
      h.adj = g.adj;
      h.base = 0;
      prev_row<ALGO>(g, prev, t, &h.po, &h.pd);
      bool use_lds = false;
      if (ALGO == kNode2Vec && t > 0 && 2 * h.pd <= hash_cells) {
        hash_geometry(h.pd, h);
        hash_clear(h, tid, NT);
        __syncthreads();
        hash_insert(h, tid, NT);
        __syncthreads();
        use_lds = true;
      }
      const uint64_t qid = P.qid[s];
      with_eval<ALGO, WEIGHTED>(g, prm, o, prev, t, h, use_lds, [&](const auto& ev) {
        hub_hop<NW>(ev, P, s, o, d, seed, qid_base + qid, t, g.adj, length, out, wave, lane);
      });
      __syncthreads();
    }
  }
}

__global__ void k_reset_counter_staged(uint64_t* p) { *p = 0; }

template <int ALGO, bool W, int NW>
static hipError_t go(const LaunchArgs& a, uint64_t* head, unsigned blocks, uint32_t cells,
                     hipStream_t stream) {
  const size_t lds = (size_t)cells * sizeof(uint32_t);
  hipLaunchKernelGGL((k_walk_persistent<ALGO, W, NW>), dim3(blocks), dim3(NW * kWave), lds,
                     stream, a.g, a.prm, a.starts, a.n, a.length, a.seed, a.qid_base, a.out,
                     a.status, head, a.cfg, cells);
  return hipGetLastError();
}

template <int ALGO, bool W>
static hipError_t go_nw(const LaunchArgs& a, uint64_t* head, unsigned blocks, uint32_t cells,
                        hipStream_t stream) {
  switch (a.cfg.wg_size) {
    case 256: return go<ALGO, W, 4>(a, head, blocks, cells, stream);
    case 512: return go<ALGO, W, 8>(a, head, blocks, cells, stream);
    case 1024: return go<ALGO, W, 16>(a, head, blocks, cells, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace staged

// Enqueues (reset head; staged kernel) on `stream`.
hipError_t launch_staged(const LaunchArgs& a, hipStream_t stream) {
  using namespace staged;
  const TuneCfg& c = a.cfg;
  if (c.slots == 0 || c.slots > (uint32_t)kMaxSlots || c.tiny_max > 16 ||
      c.hub_min <= c.tiny_max || c.wgs_per_cu == 0 || c.hash_cells < 64 * (c.wg_size / 64) ||
      (c.hash_cells & (c.hash_cells - 1)) || a.head == nullptr)
    return hipErrorInvalidValue;
  uint64_t blocks = (uint64_t)a.num_cus * c.wgs_per_cu;
  const uint64_t need = (a.n + c.slots - 1) / c.slots;
  if (blocks > need) blocks = need;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_reset_counter_staged, dim3(1), dim3(1), 0, stream, a.head);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool wt = a.g.w != nullptr;
  switch (a.algo) {
    case kDeepWalk:
      return wt ? go_nw<kDeepWalk, true>(a, a.head, (unsigned)blocks, c.hash_cells, stream)
                : go_nw<kDeepWalk, false>(a, a.head, (unsigned)blocks, c.hash_cells, stream);
    case kNode2Vec:
      return wt ? go_nw<kNode2Vec, true>(a, a.head, (unsigned)blocks, c.hash_cells, stream)
                : go_nw<kNode2Vec, false>(a, a.head, (unsigned)blocks, c.hash_cells, stream);
    case kMetaPath:
      return wt ? go_nw<kMetaPath, true>(a, a.head, (unsigned)blocks, c.hash_cells, stream)
                : go_nw<kMetaPath, false>(a, a.head, (unsigned)blocks, c.hash_cells, stream);
    case kPPR:
      return wt ? go_nw<kPPR, true>(a, a.head, (unsigned)blocks, c.hash_cells, stream)
                : go_nw<kPPR, false>(a, a.head, (unsigned)blocks, c.hash_cells, stream);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fw
