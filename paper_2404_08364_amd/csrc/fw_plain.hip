// Plain batch walker: one wavefront per query, queries assigned to
// wavefronts statically (query q goes to wavefront q mod W).  A PPR query
// tosses its stop coin before each hop.  This is the
// query-centric baseline that section 5.2 argues against on GPUs; the
// persistent form (fw_persistent.hip) adds dynamic scheduling.
#include "fw_kernels.h"
#include "fw_wave_sampler.h"

namespace fw {

// Buffers a path row in the lanes of a wavefront (lane k holds entry
// base + k) and stores 64 entries at a time.
struct RowWriter {
  uint32_t* row;
  uint64_t base;
  uint32_t buf;
  int fill;

  __device__ __forceinline__ void push(uint32_t v) {
    if (lane_id() == fill) buf = v;
    if (++fill == kWave) {
      row[base + lane_id()] = buf;
      base += kWave;
      fill = 0;
    }
  }
  // Writes the buffered entries and pads the row up to `last` with kEnd.
  __device__ __forceinline__ void finish(uint64_t last) {
    const int lane = lane_id();
    for (uint64_t p = base; p <= last; p += kWave) {
      const uint64_t pos = p + lane;
      if (pos <= last) row[pos] = (p == base && lane < fill) ? buf : kEnd;
    }
  }
};

template <int ALGO, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_walk_plain(DevGraph g, DevParams prm,
                                                    const uint32_t* __restrict__ starts,
                                                    uint64_t n, uint32_t length, uint64_t seed,
                                                    uint64_t qid_base,
                                                    uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ status) {
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
  for (uint64_t q = wave; q < n; q += nwaves) {
    const uint32_t s = uniform32(starts[q]);
    if (s >= g.nv) {
      if (lane_id() == 0) atomicOr(status, 1u);
      continue;
    }
    RowWriter rw{out + q * ((uint64_t)length + 1), 0, 0, 0};
    rw.push(s);
    uint32_t cur = s, prev = kEnd;
    uint32_t t = 0;
    for (; t < length; ++t) {
      if (ALGO == kPPR && ppr_stops(prm, seed, qid_base + q, t)) break;
      const uint64_t o = g.off[cur];
      const uint64_t d = g.off[cur + 1] - o;
      Eval<ALGO, WEIGHTED> ev;
      ev.adj = g.adj;
      ev.w = g.w;
      ev.lab = g.lab;
      ev.o = o;
      ev.first = (t == 0);
      if (ALGO == kNode2Vec) {
        ev.prev = prev;
        ev.f_ret = prm.f_ret;
        ev.f_in = prm.f_in;
        ev.f_out = prm.f_out;
        ev.mem.adj = g.adj;
        if (t > 0) {
          ev.mem.po = g.off[prev];
          ev.mem.pd = g.off[prev + 1] - ev.mem.po;
        } else {
          ev.mem.po = ev.mem.pd = 0;
        }
      }
      if (ALGO == kMetaPath) ev.want = schema_label(prm, t);
      const uint64_t u = philox_draw(seed, qid_base + q, t);
      int64_t idx;
      if ((ALGO == kDeepWalk || ALGO == kPPR) && !WEIGHTED) {
        // All weights 1: the prefix sum at i is i + 1, so the pick is r.
        idx = d ? (int64_t)scale_draw(u, d) : -1;
      } else {
        idx = wave_pick(ev, o, d, u);
      }
      if (idx < 0) break;
      const uint32_t nxt = uniform32(g.adj[o + (uint64_t)idx]);
      rw.push(nxt);
      prev = cur;
      cur = nxt;
    }
    rw.finish(length);
  }
}

hipError_t launch_plain(const LaunchArgs& a, hipStream_t stream) {
  const int block = 256;
  const uint64_t waves_needed = a.n;
  uint64_t blocks = (waves_needed + (block / kWave) - 1) / (block / kWave);
  const uint64_t cap = (uint64_t)a.num_cus * 32;  // 8 wavefronts per SIMD
  if (blocks > cap) blocks = cap;
  if (blocks == 0) blocks = 1;
  const bool wt = a.g.w != nullptr;
#define FW_GO(A, W)                                                                         \
  hipLaunchKernelGGL((k_walk_plain<A, W>), dim3((unsigned)blocks), dim3(block), 0, stream,  \
                     a.g, a.prm, a.starts, a.n, a.length, a.seed, a.qid_base, a.out,         \
                     a.status)
  switch (a.algo) {
    case kDeepWalk:
      if (wt) FW_GO(kDeepWalk, true); else FW_GO(kDeepWalk, false);
      break;
    case kNode2Vec:
      if (wt) FW_GO(kNode2Vec, true); else FW_GO(kNode2Vec, false);
      break;
    case kMetaPath:
      if (wt) FW_GO(kMetaPath, true); else FW_GO(kMetaPath, false);
      break;
    case kPPR:
      if (wt) FW_GO(kPPR, true); else FW_GO(kPPR, false);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef FW_GO
  return hipGetLastError();
}

}  // namespace fw
