// Persistent, dynamically scheduled walker (sections 5.1 and 5.2).
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

extern __shared__ uint32_t fw_dyn_lds[];  // hash-set region (u32 entries)

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

// Open-addressing (linear probing) hash set of the ids of N(prev), in
// fw_dyn_lds[base, base + mask + 1); kEnd marks an empty cell.
struct MemberHybrid {
  const uint32_t* __restrict__ adj;
  uint64_t po, pd;
  uint32_t base, mask, shift;
  bool lds;
  __device__ __forceinline__ bool contains(uint32_t u) const {
    if (!lds) return row_contains(adj, po, pd, u);
    uint32_t h = (u * kFib) >> shift;
    for (;;) {
      const uint32_t x = fw_dyn_lds[base + h];
      if (x == u) return true;
      if (x == kEnd) return false;
      h = (h + 1) & mask;
    }
  }
};

__device__ __forceinline__ uint32_t log2_ceil(uint64_t x) {
  uint32_t b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// Sizes the table for n keys (load factor <= 1/2, at least 64 cells).
__device__ __forceinline__ void hash_geometry(uint64_t n, MemberHybrid& m) {
  uint32_t bits = log2_ceil(2 * n);
  if (bits < 6) bits = 6;
  m.mask = (1u << bits) - 1;
  m.shift = 32 - bits;
}

// Builds the set with threads [tix, tix + nthr) of the caller; the caller
// synchronises between clear and insert and after insert.
__device__ __forceinline__ void hash_clear(const MemberHybrid& m, int tix, int nthr) {
  for (uint32_t i = tix; i <= m.mask; i += nthr) fw_dyn_lds[m.base + i] = kEnd;
}

__device__ __forceinline__ void hash_insert(const MemberHybrid& m, int tix, int nthr) {
  for (uint64_t i = tix; i < m.pd; i += nthr) {
    const uint32_t u = m.adj[m.po + i];
    uint32_t h = (u * kFib) >> m.shift;
    for (;;) {
      const uint32_t old = atomicCAS(&fw_dyn_lds[m.base + h], kEnd, u);
      if (old == kEnd || old == u) break;
      h = (h + 1) & m.mask;
    }
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int ALGO, bool WEIGHTED>
__device__ __forceinline__ Eval<ALGO, WEIGHTED, MemberHybrid> make_eval(const DevGraph& g,
                                                                        const DevParams& prm,
                                                                        uint64_t o, uint32_t prev,
                                                                        uint32_t t) {
  Eval<ALGO, WEIGHTED, MemberHybrid> ev;
  ev.adj = g.adj;
  ev.w = g.w;
  ev.lab = g.lab;
  ev.o = o;
  ev.first = (t == 0);
  ev.prev = prev;
  ev.f_ret = prm.f_ret;
  ev.f_in = prm.f_in;
  ev.f_out = prm.f_out;
  ev.want = (ALGO == kMetaPath) ? prm.schema[t % prm.schema_len] : 0u;
  ev.mem.adj = g.adj;
  ev.mem.po = 0;
  ev.mem.pd = 0;
  ev.mem.base = 0;
  ev.mem.mask = 0;
  ev.mem.shift = 0;
  ev.mem.lds = false;
  if (ALGO == kNode2Vec && t > 0) {
    ev.mem.po = g.off[prev];
    ev.mem.pd = g.off[prev + 1] - ev.mem.po;
  }
  return ev;
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
  uint64_t lo, len;
  __device__ __forceinline__ HubPart(uint64_t nq, int w, int nw) {
    const uint64_t chunks = (nq + kWave - 1) / kWave;
    const uint64_t c0 = chunks * w / nw, c1 = chunks * (w + 1) / nw;
    lo = c0 * kWave;
    const uint64_t hi = min(c1 * kWave, nq);
    len = hi > lo ? hi - lo : 0;
  }
};

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
      const uint64_t o = g.off[c], d = g.off[c + 1] - o;
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
      auto ev = make_eval<ALGO, WEIGHTED>(g, prm, o, prev, t);
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
      auto ev = make_eval<ALGO, WEIGHTED>(g, prm, o, prev, t);
      if (ALGO == kNode2Vec && t > 0 && 2 * ev.mem.pd <= wave_cells &&
          ev.mem.pd <= 4 * d) {
        ev.mem.base = wave * wave_cells;
        hash_geometry(ev.mem.pd, ev.mem);
        hash_clear(ev.mem, lane, kWave);
        wave_sync_lds();
        hash_insert(ev.mem, lane, kWave);
        wave_sync_lds();
        ev.mem.lds = true;
      }
      const uint64_t u = philox_draw(seed, qid_base + P.qid[s], t);
      const int64_t idx = wave_pick(ev, o, d, u);
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
      auto ev = make_eval<ALGO, WEIGHTED>(g, prm, o, prev, t);
      if (ALGO == kNode2Vec && t > 0 && 2 * ev.mem.pd <= hash_cells) {
        ev.mem.base = 0;
        hash_geometry(ev.mem.pd, ev.mem);
        hash_clear(ev.mem, tid, NT);
        __syncthreads();
        hash_insert(ev.mem, tid, NT);
        __syncthreads();
        ev.mem.lds = true;
      }
      const QuadSlice qs(o, d);
      {
        const HubPart part(qs.nq, wave, NW);
        uint64_t mine = 0;
        if (part.len) mine = wave_group_totals(ev, qs, part.lo, part.len, GroupSplit(part.len));
        P.gt[wave * kWave + lane] = mine;
      }
      __syncthreads();
      if (wave == 0) {
        // Lane j owns the NW consecutive group totals [j*NW, j*NW + NW).
        uint64_t sj = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) sj += P.gt[lane * NW + i];
        const uint64_t incl = wave_incl_scan(sj);
        const uint64_t total = readlane64(incl, kWave - 1);
        bool dead = (total == 0);
        uint32_t next = kEnd;
        if (!dead) {
          uint64_t r = scale_draw(philox_draw(seed, qid_base + P.qid[s], t), total);
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
          const uint64_t gi = (uint64_t)(e % kWave);
          const uint64_t gb = part.lo + gi * sp.gsz;
          const uint64_t glen = min(sp.gsz, part.len - gi * sp.gsz);
          const uint64_t idx = wave_locate(ev, qs, gb, glen, r);
          next = g.adj[o + idx];
        }
        advance(P, s, dead, next, length, out, lane, kWave);
      }
      __syncthreads();
    }
  }
}

__global__ void k_reset_counter(uint64_t* p) { *p = 0; }

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

// Enqueues (reset head; persistent kernel) on `stream`.
hipError_t launch_persistent(const LaunchArgs& a, hipStream_t stream) {
  const TuneCfg& c = a.cfg;
  if (c.slots == 0 || c.slots > (uint32_t)kMaxSlots || c.tiny_max > 16 ||
      c.hub_min <= c.tiny_max || c.wgs_per_cu == 0 || c.hash_cells < 64 * (c.wg_size / 64) ||
      (c.hash_cells & (c.hash_cells - 1)) || a.head == nullptr)
    return hipErrorInvalidValue;
  uint64_t blocks = (uint64_t)a.num_cus * c.wgs_per_cu;
  const uint64_t need = (a.n + c.slots - 1) / c.slots;
  if (blocks > need) blocks = need;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, stream, a.head);
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
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fw
