// Reservoir-sampling walkers (section 4): the paper's two parallel reservoir
// samplers as alternatives to the inverse-CDF pick, one wavefront per query
// (static assignment, as the plain walker).
//
// Each entry i of the hop's neighbour sequence gets its own uniform word:
// word i mod 4 of Philox4x64-10 at counter (qid, t, i / 4, 1), key (seed, 0).
// Lane L handles quads of four consecutive entries.  Visiting entry i of
// weight w_i with W the running total including it, the selection becomes i
// when floor(u_i * W / 2^64) < w_i (the integer form of "random(0,1) <
// w_i / W"); the last selection is the pick.
//
//   DPRS (Algorithm 3): 256-entry chunks in sequence order (lane L holds
//   quad 64c + L); per chunk one wave scan gives each entry its running total
//   and one ballot keeps the last selection.  The result is that of the
//   sequential reservoir over S.
//   ZPRS (Algorithm 4): lane L owns quads L, L + 64, ... ; pass 1 sums each
//   lane's weights, an exclusive wave scan gives each lane its starting
//   total, pass 2 re-reads the lane's quads and selects along the zig-zag
//   order S' (lane 0's entries, then lane 1's, ...); the last lane holding a
//   selection wins.
// Node2vec membership is the binary search of N(prev) in global memory, as
// the paper's samplers do it.
#include "fw_kernels.h"
#include "fw_reservoir.h"

namespace fw {

template <int ALGO, bool WEIGHTED, bool ZIGZAG>
__global__ __launch_bounds__(256) void k_walk_reservoir(DevGraph g, DevParams prm,
                                                        const uint32_t* __restrict__ starts,
                                                        uint64_t n, uint32_t length,
                                                        uint64_t seed, uint64_t qid_base,
                                                        uint32_t* __restrict__ out,
                                                        uint32_t* __restrict__ status) {
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  for (uint64_t q = wave; q < n; q += nwaves) {
    const uint32_t s = uniform32(starts[q]);
    uint32_t* row = out + q * ((uint64_t)length + 1);
    if (s >= g.nv) {
      if (lane == 0) atomicOr(status, 1u);
      continue;
    }
    if (lane == 0) row[0] = s;
    const uint64_t qid = qid_base + q;
    uint32_t cur = s, prev = kEnd, t = 0;
    for (; t < length; ++t) {
      if (ALGO == kPPR && ppr_stops(prm, seed, qid, t)) break;
      const uint64_t o = g.off[cur];
      const uint64_t d = g.off[cur + 1] - o;
      Eval<ALGO, WEIGHTED> ev;
      ev.adj = g.adj;
      ev.w = g.w;
      ev.lab = g.lab;
      ev.o = o;
      ev.first = (t == 0);
      ev.prev = prev;
      ev.f_ret = prm.f_ret;
      ev.f_in = prm.f_in;
      ev.f_out = prm.f_out;
      ev.mem.adj = g.adj;
      ev.mem.po = ev.mem.pd = 0;
      if (ALGO == kNode2Vec && t > 0) {
        ev.mem.po = g.off[prev];
        ev.mem.pd = g.off[prev + 1] - ev.mem.po;
      }
      ev.want = (ALGO == kMetaPath) ? schema_label(prm, t) : 0u;
      const int64_t idx = ZIGZAG ? zprs_pick(ev, d, seed, qid, t) : dprs_pick(ev, d, seed, qid, t);
      if (idx < 0) break;
      const uint32_t nxt = uniform32(g.adj[o + (uint64_t)idx]);
      if (lane == 0) row[t + 1] = nxt;
      prev = cur;
      cur = nxt;
    }
    for (uint32_t p = t + 1 + lane; p <= length; p += kWave) row[p] = kEnd;
  }
}

hipError_t launch_reservoir(const LaunchArgs& a, int sampler, hipStream_t stream) {
  const int block = 256;
  uint64_t blocks = (a.n + (block / kWave) - 1) / (block / kWave);
  const uint64_t cap = (uint64_t)a.num_cus * 32;
  if (blocks > cap) blocks = cap;
  if (blocks == 0) blocks = 1;
  const bool wt = a.g.w != nullptr;
  const bool zz = sampler == 2;
#define FW_GO(A, W, Z)                                                                          \
  hipLaunchKernelGGL((k_walk_reservoir<A, W, Z>), dim3((unsigned)blocks), dim3(block), 0,       \
                     stream, a.g, a.prm, a.starts, a.n, a.length, a.seed, a.qid_base, a.out,     \
                     a.status)
#define FW_GO2(A)                                 \
  if (wt) {                                       \
    if (zz) FW_GO(A, true, true); else FW_GO(A, true, false);   \
  } else {                                        \
    if (zz) FW_GO(A, false, true); else FW_GO(A, false, false); \
  }
  switch (a.algo) {
    case kDeepWalk: FW_GO2(kDeepWalk); break;
    case kNode2Vec: FW_GO2(kNode2Vec); break;
    case kMetaPath: FW_GO2(kMetaPath); break;
    case kPPR: FW_GO2(kPPR); break;
    default:
      return hipErrorInvalidValue;
  }
#undef FW_GO2
#undef FW_GO
  return hipGetLastError();
}

}  // namespace fw
