// Walks whose results live in host memory, run in batches that fit a device
// budget (section 5.2, Eq. 5): the queries are split into batches whose
// start vertices and result rows fit half of the budget, and consecutive
// batches alternate between two streams and two buffers (ping-pong), so the
// device-to-host copy of one batch overlaps the walk of the next.  Query i
// keeps id i (each batch walks with qid_base = its first query), so the rows
// equal fw_walk's on the whole query set.
#include <algorithm>
#include <cstring>
#include <vector>

#include "flowwalk.h"
#include "fw_runtime.h"

namespace {

int fail(int code, const char* msg) { return fw::set_error(code, msg); }

int hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fw::set_error(e == hipErrorOutOfMemory ? FW_ENOMEM : FW_EHIP, m.c_str());
}

struct Side {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint32_t* d_starts = nullptr;
  uint32_t* d_rows = nullptr;
  uint32_t* h_starts = nullptr;  // pinned staging
  uint32_t* h_rows = nullptr;    // pinned staging
  uint64_t first = 0, count = 0;  // the batch it holds
  bool pending = false;
};

void release(Side& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  (void)hipFree(s.d_starts);
  (void)hipFree(s.d_rows);
  (void)hipHostFree(s.h_starts);
  (void)hipHostFree(s.h_rows);
  s = Side{};
}

}  // namespace

extern "C" {

int fw_walk_host(const fw_graph* g, fw_algo algo, const fw_params* params,
                 const uint32_t* starts_host, uint64_t n, uint32_t length, uint64_t seed,
                 uint32_t* out_host, fw_batch_opts* opts) {
  fw::DevParams dp;
  // Host pointers stand in for the device ones in the argument check.
  int rc = fw::check_walk_args(g, (int)algo, params, n, length, starts_host, out_host, &dp);
  if (rc) return rc;
  fw_batch_opts o{};
  if (opts) o = *opts;
  const uint64_t cols = (uint64_t)length + 1;
  for (uint64_t i = 0; i < n; ++i)
    if (starts_host[i] >= g->nv) return fail(FW_EINVAL, "a start vertex is >= n_vertices");
  if (n == 0) {
    if (opts) opts->batch_queries = 0, opts->batches = 0;
    return FW_OK;
  }
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "selecting the graph's device");
  uint64_t budget = o.device_budget_bytes;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return hip_fail(e, "querying free device memory");
    const uint64_t reserve = 1ull << 30;
    budget = free_b > reserve ? free_b - reserve : free_b / 2;
  }
  // Eq. 5: each of the two buffers holds a batch's start vertices and rows.
  const uint64_t per_query = (cols + 1) * sizeof(uint32_t);
  uint64_t batch = budget / (2 * per_query);
  if (o.max_batch_queries && batch > o.max_batch_queries) batch = o.max_batch_queries;
  if (batch == 0) return fail(FW_EINVAL, "device_budget_bytes holds no query");
  batch = std::min(batch, n);
  const uint64_t nb = (n + batch - 1) / batch;

  Side side[2];
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    Side& s = side[k];
    e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_starts, batch * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_rows, batch * cols * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_starts, batch * sizeof(uint32_t), 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_rows, batch * cols * sizeof(uint32_t), 0);
  }
  if (e != hipSuccess) {
    rc = hip_fail(e, "allocating the batch buffers");
    release(side[0]);
    release(side[1]);
    return rc;
  }

  // Copies a finished batch from its pinned staging into out_host.
  auto drain = [&](Side& s) -> int {
    if (!s.pending) return FW_OK;
    hipError_t err = hipEventSynchronize(s.done);
    if (err != hipSuccess) return hip_fail(err, "waiting for a batch");
    std::memcpy(out_host + s.first * cols, s.h_rows, s.count * cols * sizeof(uint32_t));
    s.pending = false;
    return FW_OK;
  };

  fw_walk_opts wo{};
  wo.mode = o.mode;
  wo.async = 1;
  for (uint64_t b = 0; b < nb && rc == FW_OK; ++b) {
    Side& s = side[b % 2];
    rc = drain(s);  // the buffers of batch b - 2 are free once it is copied out
    if (rc) break;
    s.first = b * batch;
    s.count = std::min(batch, n - s.first);
    std::memcpy(s.h_starts, starts_host + s.first, s.count * sizeof(uint32_t));
    e = hipMemcpyAsync(s.d_starts, s.h_starts, s.count * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s.stream);
    if (e != hipSuccess) {
      rc = hip_fail(e, "copying start vertices");
      break;
    }
    wo.stream = s.stream;
    wo.qid_base = s.first;
    rc = fw_walk_ex(g, algo, params, s.d_starts, s.count, length, seed, s.d_rows, &wo);
    if (rc) break;
    e = hipMemcpyAsync(s.h_rows, s.d_rows, s.count * cols * sizeof(uint32_t),
                       hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e != hipSuccess) {
      rc = hip_fail(e, "copying result rows");
      break;
    }
    s.pending = true;
  }
  // Drain in batch order (the older batch sits on the other side).
  if (rc == FW_OK) {
    Side& a = side[nb % 2];
    Side& c = side[(nb + 1) % 2];
    rc = drain(a);
    if (rc == FW_OK) rc = drain(c);
  }
  if (rc == FW_OK) rc = fw_sync(g, side[0].stream);
  release(side[0]);
  release(side[1]);
  if (rc == FW_OK && opts) {
    opts->batch_queries = batch;
    opts->batches = (uint32_t)nb;
  }
  return rc;
}

}  // extern "C"
