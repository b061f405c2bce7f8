// Sampler microbenchmark (the comparison of sampling methods in section
// 6.3): n_tasks independent tasks, task j picking one index of the `size`
// weights w[j*size, (j+1)*size) with chance w_i / T, one wavefront per task
// (grid-stride).  The bufferless samplers (ITS, DPRS, ZPRS) are the walkers'
// own; the buffered ones keep O(size) state per task in a device scratch
// slice owned by the wavefront: ITS_BUFFERED stores the prefix sums and
// binary-searches them (the C-SAW layout), ALIAS builds Vose's table with
// the index-order sweep on one lane and samples it in O(1), REJECTION draws
// candidates until one is accepted against the maximum weight, 64 trials per
// round, the first accepted trial in trial order winning.
#include <algorithm>
#include <cstring>
#include <string>

#include "flowwalk.h"
#include "fw_reservoir.h"
#include "fw_runtime.h"
#include "fw_wave_sampler.h"

namespace fw {

namespace {

constexpr uint32_t kRjsMaxTrials = 1u << 24;

// Weights of one task, by absolute position (quads masked at the array end).
struct TaskEval {
  const uint32_t* __restrict__ w;
  uint64_t o;    // first weight of the task
  uint64_t end;  // n_tasks * size
  uint64_t qa;   // quad run base (set by bind_quads)
  __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return w[o + i]; }
  static constexpr bool kCheapTotal = false;
  static constexpr bool kRawWeights = false;
  __device__ __forceinline__ uint64_t quad_total4(uint32_t q) const {
    uint64_t o[4];
    quad(q, o);
    return (o[0] + o[1]) + (o[2] + o[3]);
  }
  __device__ __forceinline__ void quad(uint32_t q, uint64_t out[4]) const {
    const uint64_t p = qa + 4ull * q;
    if (p + 4 <= end) {
      const uint4 v = *reinterpret_cast<const uint4*>(w + p);
      out[0] = v.x;
      out[1] = v.y;
      out[2] = v.z;
      out[3] = v.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) out[j] = p + j < end ? w[p + j] : 0ull;
    }
  }
};

__device__ __forceinline__ uint64_t mulhi(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// Sum and maximum of the task's weights (every lane gets both).
__device__ __forceinline__ void task_totals(const TaskEval& ev, uint32_t size, uint64_t& total,
                                            uint32_t& wmax) {
  uint64_t s = 0;
  uint32_t m = 0;
  for (uint32_t i = lane_id(); i < size; i += kWave) {
    const uint32_t x = (uint32_t)ev(i);
    s += x;
    m = max(m, x);
  }
  total = wave_sum(s);
  wmax = wave_max32(m);
}

__device__ int64_t its_buffered(const TaskEval& ev, uint32_t size, uint64_t seed, uint64_t task,
                                uint64_t* __restrict__ prefix) {
  const int lane = lane_id();
  uint64_t carry = 0;
  for (uint32_t c = 0; c < size; c += kWave) {
    const uint32_t i = c + lane;
    const uint64_t x = i < size ? ev(i) : 0ull;
    const uint64_t incl = wave_incl_scan(x) + carry;
    if (i < size) prefix[i] = incl;
    carry = readlane64(incl, kWave - 1);
  }
  const uint64_t total = carry;
  if (total == 0) return -1;
  uint64_t blk[4];
  philox4x64_10(task, 0, 0, 0, seed, blk);
  const uint64_t r = mulhi(blk[0], total);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  // First index whose inclusive prefix exceeds r (lower bound on prefix > r).
  uint32_t lo = 0, len = size;
  while (len > 0) {
    const uint32_t half = len / 2;
    if (prefix[lo + half] <= r) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo < size ? (int64_t)lo : -1;
}

__device__ int64_t alias_pick(const TaskEval& ev, uint32_t size, uint64_t seed, uint64_t task,
                              uint64_t* __restrict__ prob, uint32_t* __restrict__ alias) {
  const int lane = lane_id();
  uint64_t total;
  uint32_t wmax;
  task_totals(ev, size, total, wmax);
  if (total == 0) return -1;
  const uint64_t T = total, n = size;
  for (uint32_t c = lane; c < size; c += kWave) {
    prob[c] = T;
    alias[c] = c;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if (lane == 0) {
    // The sweep: heavy j fills the light items in index order; when its
    // remaining mass is at most T it becomes a column filled from the next
    // heavy item.
    uint32_t i = 0, j = 0;
    while (i < size && (uint64_t)ev(i) * n >= T) ++i;
    while (j < size && (uint64_t)ev(j) * n < T) ++j;
    uint64_t rem = j < size ? (uint64_t)ev(j) * n : 0;
    while (j < size) {
      if (rem > T) {
        if (i >= size) break;
        const uint64_t q = (uint64_t)ev(i) * n;
        prob[i] = q;
        alias[i] = j;
        rem -= T - q;
        do ++i; while (i < size && (uint64_t)ev(i) * n >= T);
      } else {
        uint32_t nj = j + 1;
        while (nj < size && (uint64_t)ev(nj) * n < T) ++nj;
        prob[j] = rem;
        alias[j] = nj < size ? nj : j;
        if (nj < size) rem = (uint64_t)ev(nj) * n - (T - rem);
        j = nj;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  uint64_t blk[4];
  philox4x64_10(task, 0, 0, 2, seed, blk);
  const uint64_t c = mulhi(blk[0], n);
  return mulhi(blk[1], T) < prob[c] ? (int64_t)c : (int64_t)alias[c];
}

__device__ int64_t rejection_pick(const TaskEval& ev, uint32_t size, uint64_t seed,
                                  uint64_t task) {
  uint64_t total;
  uint32_t wmax;
  task_totals(ev, size, total, wmax);
  if (total == 0) return -1;
  for (uint32_t k0 = 0; k0 < kRjsMaxTrials; k0 += kWave) {
    const uint32_t k = k0 + lane_id();
    uint64_t blk[4];
    philox4x64_10(task, k, 0, 3, seed, blk);
    const uint64_t c = mulhi(blk[0], size);
    const bool ok = mulhi(blk[1], wmax) < ev(c);
    const uint64_t m = ballot(ok);
    if (m) return (int64_t)readlane64(c, __builtin_ctzll(m));
  }
  return -1;
}

template <int S>
__global__ __launch_bounds__(256) void k_tasks(const uint32_t* __restrict__ w, uint64_t n_tasks,
                                               uint32_t size, uint64_t seed,
                                               uint32_t* __restrict__ picks,
                                               uint64_t* __restrict__ s64,
                                               uint32_t* __restrict__ s32) {
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
  for (uint64_t j = wave; j < n_tasks; j += nwaves) {
    TaskEval ev{w, j * size, n_tasks * size, 0};
    int64_t pick;
    if (S == FW_TASK_ITS) {
      uint64_t blk[4];
      philox4x64_10(j, 0, 0, 0, seed, blk);
      pick = wave_pick(ev, ev.o, size, blk[0]);
    } else if (S == FW_TASK_DPRS) {
      pick = dprs_pick(ev, size, seed, j, 0);
    } else if (S == FW_TASK_ZPRS) {
      pick = zprs_pick(ev, size, seed, j, 0);
    } else if (S == FW_TASK_ITS_BUFFERED) {
      pick = its_buffered(ev, size, seed, j, s64 + wave * size);
    } else if (S == FW_TASK_ALIAS) {
      pick = alias_pick(ev, size, seed, j, s64 + wave * size, s32 + wave * size);
    } else {
      pick = rejection_pick(ev, size, seed, j);
    }
    if (lane_id() == 0) picks[j] = pick < 0 ? kEnd : (uint32_t)pick;
  }
}

}  // namespace

}  // namespace fw

extern "C" {

int fw_sample_tasks(int sampler, const uint32_t* weights, uint64_t n_tasks, uint32_t size,
                    uint64_t seed, uint32_t* picks, void* stream) {
  if (sampler < FW_TASK_ITS || sampler > FW_TASK_REJECTION)
    return fw::set_error(FW_EINVAL, "unknown task sampler");
  if (n_tasks == 0) return FW_OK;
  if (size == 0 || size >= fw::kMaxDegree)
    return fw::set_error(FW_EINVAL, "size must be in 1 .. 2^28 - 1");
  if (!weights || !picks) return fw::set_error(FW_EINVAL, "weights or picks is NULL");
  if (n_tasks > (UINT64_MAX >> 2) / size) return fw::set_error(FW_EINVAL, "n_tasks * size too large");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fw::set_error(FW_EHIP, hipGetErrorString(e));
  uint64_t waves = std::min<uint64_t>(n_tasks, (uint64_t)prop.multiProcessorCount * 32);
  const bool buffered = sampler == FW_TASK_ITS_BUFFERED || sampler == FW_TASK_ALIAS;
  uint64_t* s64 = nullptr;
  uint32_t* s32 = nullptr;
  if (buffered) {
    // O(size) per task in flight: bound the slices by 8 GiB of scratch.
    const uint64_t per = (uint64_t)size * (sampler == FW_TASK_ALIAS ? 12 : 8);
    waves = std::max<uint64_t>(1, std::min<uint64_t>(waves, (8ull << 30) / per));
  }
  // The grid has 4 wavefronts per block; wavefront w owns scratch slice w.
  waves = (waves + 3) / 4 * 4;
  if (buffered) {
    e = hipMalloc((void**)&s64, waves * size * sizeof(uint64_t));
    if (e == hipSuccess && sampler == FW_TASK_ALIAS)
      e = hipMalloc((void**)&s32, waves * size * sizeof(uint32_t));
    if (e != hipSuccess) {
      (void)hipFree(s64);
      return fw::set_error(FW_ENOMEM, "task scratch");
    }
  }
  const unsigned blocks = (unsigned)(waves / 4);
#define FW_GO(S)                                                                             \
  hipLaunchKernelGGL((fw::k_tasks<S>), dim3(blocks), dim3(256), 0, st, weights, n_tasks, size, \
                     seed, picks, s64, s32)
  switch (sampler) {
    case FW_TASK_ITS: FW_GO(FW_TASK_ITS); break;
    case FW_TASK_DPRS: FW_GO(FW_TASK_DPRS); break;
    case FW_TASK_ZPRS: FW_GO(FW_TASK_ZPRS); break;
    case FW_TASK_ITS_BUFFERED: FW_GO(FW_TASK_ITS_BUFFERED); break;
    case FW_TASK_ALIAS: FW_GO(FW_TASK_ALIAS); break;
    default: FW_GO(FW_TASK_REJECTION); break;
  }
#undef FW_GO
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(s64);
  (void)hipFree(s32);
  if (e != hipSuccess) return fw::set_error(FW_EHIP, hipGetErrorString(e));
  return FW_OK;
}

}  // extern "C"
