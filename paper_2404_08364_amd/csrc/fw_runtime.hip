// Host runtime behind the C ABI of flowwalk.h: CSR validation and upload,
// argument checking, kernel dispatch and error reporting.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "flowwalk.h"
#include "fw_device.h"
#include "fw_kernels.h"
#include "fw_runtime.h"

namespace {

thread_local std::string t_err;

int fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

unsigned host_threads() {
  unsigned n = std::thread::hardware_concurrency();
  return std::max(1u, std::min(16u, n ? n : 1u));
}

// Splits [0, n) over host threads; f(lo, hi) returns false on a problem.
template <class F>
bool parallel_all(uint64_t n, F&& f) {
  const unsigned nt = n < (1u << 16) ? 1u : host_threads();
  std::atomic<bool> ok{true};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    const uint64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    th.emplace_back([&, lo, hi] {
      if (!f(lo, hi)) ok = false;
    });
  }
  for (auto& x : th) x.join();
  return ok;
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

namespace fw {

int set_error(int code, const char* msg) { return fail(code, msg); }

int check_walk_args(const fw_graph* g, int algo, const fw_params* params, uint64_t n,
                    uint32_t length, const void* starts, const void* out, DevParams* dp) {
  if (!g) return fail(FW_EINVAL, "graph is NULL");
  if (algo != FW_DEEPWALK && algo != FW_NODE2VEC && algo != FW_METAPATH && algo != FW_PPR)
    return fail(FW_EINVAL, "unknown algorithm");
  std::memset(dp, 0, sizeof(*dp));
  uint64_t max_f = 1;
  if (algo == FW_NODE2VEC) {
    if (!params) return fail(FW_EINVAL, "node2vec needs parameters");
    if (!params->f_ret && !params->f_in && !params->f_out)
      return fail(FW_EINVAL, "node2vec factors are all zero");
    dp->f_ret = params->f_ret;
    dp->f_in = params->f_in;
    dp->f_out = params->f_out;
    max_f = std::max({params->f_ret, params->f_in, params->f_out});
  } else if (algo == FW_METAPATH) {
    if (!params) return fail(FW_EINVAL, "MetaPath needs a schema");
    if (!g->d_lab) return fail(FW_EINVAL, "MetaPath on a graph without labels");
    if (params->schema_len < 1 || params->schema_len > 16)
      return fail(FW_EINVAL, "schema_len must be in 1..16");
    dp->schema_len = params->schema_len;
    std::memcpy(dp->schema, params->schema, sizeof(dp->schema));
  } else if (algo == FW_PPR) {
    if (!params) return fail(FW_EINVAL, "PPR needs a stop chance");
    if (params->stop_den == 0 || params->stop_num > params->stop_den)
      return fail(FW_EINVAL, "PPR stop chance must satisfy 0 <= stop_num <= stop_den, stop_den > 0");
    dp->stop_num = params->stop_num;
    dp->stop_den = params->stop_den;
  }
  const unsigned __int128 bound = (unsigned __int128)g->max_w * max_f * g->max_deg;
  if (bound >> 64) return fail(FW_EOVERFLOW, "max_weight * max_factor * max_degree >= 2^64");
  if (n) {
    if (!starts || !out) return fail(FW_EINVAL, "starts or out_paths is NULL");
    const unsigned __int128 cells = (unsigned __int128)n * ((uint64_t)length + 1);
    if (cells >> 62) return fail(FW_EINVAL, "n * (length + 1) too large");
  }
  return FW_OK;
}

DevGraph dev_graph(const fw_graph* g) {
  DevGraph d;
  d.off = g->d_off;
  d.adj = g->d_adj;
  d.w = g->d_w;
  d.lab = g->d_lab;
  d.nv = g->nv;
  return d;
}

int read_status(const fw_graph* g, hipStream_t stream) {
  uint32_t st = 0;
  hipError_t e = hipMemcpyAsync(&st, g->d_status, sizeof(st), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "reading the walk status");
  if (st) {
    e = hipMemsetAsync(g->d_status, 0, sizeof(uint32_t), stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "clearing the walk status");
    return fail(FW_EINVAL, "a start vertex is >= n_vertices");
  }
  return FW_OK;
}

// Counts the entries of p[0, m) that are not FW_END: one grid-stride pass,
// wave sums, one 64-bit atomic per wavefront.
__global__ void k_count_not_end(const uint32_t* __restrict__ p, uint64_t m,
                                unsigned long long* total) {
  uint64_t c = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    c += p[i] != FW_END;
  const uint64_t s = wave_sum(c);
  if (lane_id() == 0 && s) atomicAdd(total, (unsigned long long)s);
}

}  // namespace fw

extern "C" {

const char* fw_last_error(void) { return t_err.c_str(); }

int fw_node2vec_factors(uint32_t p_num, uint32_t p_den, uint32_t q_num, uint32_t q_den,
                        fw_params* out) {
  if (!out) return fail(FW_EINVAL, "out is NULL");
  if (!p_num || !p_den || !q_num || !q_den) return fail(FW_EINVAL, "p and q must be positive");
  uint64_t fr = (uint64_t)p_den * q_num, fi = (uint64_t)p_num * q_num,
           fo = (uint64_t)p_num * q_den;
  const uint64_t c = gcd64(gcd64(fr, fi), fo);
  fr /= c;
  fi /= c;
  fo /= c;
  if (fr > 0xFFFFFFFFull || fi > 0xFFFFFFFFull || fo > 0xFFFFFFFFull)
    return fail(FW_EINVAL, "node2vec factors do not fit in 32 bits");
  out->f_ret = (uint32_t)fr;
  out->f_in = (uint32_t)fi;
  out->f_out = (uint32_t)fo;
  return FW_OK;
}

int fw_graph_upload(const fw_csr* csr, const uint32_t* weights, const uint8_t* labels,
                    fw_graph** out) {
  if (!out) return fail(FW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!csr || !csr->offsets || (csr->n_edges && !csr->adj))
    return fail(FW_EINVAL, "CSR pointers are NULL");
  const uint64_t nv = csr->n_vertices, ne = csr->n_edges;
  if (nv >= 0xFFFFFFFFull) return fail(FW_EINVAL, "n_vertices must be below 2^32 - 1");
  const uint64_t* off = csr->offsets;
  const uint32_t* adj = csr->adj;
  if (off[0] != 0 || off[nv] != ne) return fail(FW_EINVAL, "offsets[0] != 0 or offsets[V] != E");
  std::atomic<uint64_t> max_deg{0}, max_w{weights ? 0u : 1u};
  const bool ok = parallel_all(nv, [&](uint64_t lo, uint64_t hi) {
    uint64_t md = 0, mw = 0;
    for (uint64_t v = lo; v < hi; ++v) {
      const uint64_t b = off[v], e = off[v + 1];
      if (e < b || e > ne) return false;
      md = std::max(md, e - b);
      for (uint64_t i = b; i < e; ++i) {
        if (adj[i] >= nv) return false;
        if (i > b && adj[i] < adj[i - 1]) return false;
        if (weights) mw = std::max<uint64_t>(mw, weights[i]);
      }
    }
    uint64_t cur = max_deg.load();
    while (md > cur && !max_deg.compare_exchange_weak(cur, md)) {
    }
    cur = max_w.load();
    while (weights && mw > cur && !max_w.compare_exchange_weak(cur, mw)) {
    }
    return true;
  });
  if (!ok) return fail(FW_EINVAL, "malformed CSR (offsets, id range or row order)");
  // The samplers index a neighbour slice with 32-bit quad offsets.
  if (max_deg.load() >= fw::kMaxDegree)
    return fail(FW_EINVAL, "a vertex has 2^28 or more neighbours");

  fw_graph* g = new (std::nothrow) fw_graph();
  if (!g) return fail(FW_ENOMEM, "host allocation");
  g->nv = nv;
  g->ne = ne;
  g->max_deg = max_deg.load();
  g->max_w = max_w.load();
  hipError_t e = hipGetDevice(&g->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, g->device);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "querying the device");
  }
  g->fingerprint = fw::graph_fingerprint(g, off, adj, weights, labels);
  g->num_cus = prop.multiProcessorCount;
  g->lds_per_block = prop.sharedMemPerBlock;
  auto alloc = [&](void** p, size_t bytes) -> hipError_t {
    g->bytes += bytes;
    return hipMalloc(p, bytes ? bytes : 4);
  };
  // Per-edge arrays get kPad zeroed entries past the end: the kernels read
  // whole 16-byte quads, which may reach up to 3 entries beyond entry E - 1.
  constexpr uint64_t kPad = 16;
  e = alloc((void**)&g->d_off, (nv + 1) * sizeof(uint64_t));
  if (e == hipSuccess) e = alloc((void**)&g->d_adj, (ne + kPad) * sizeof(uint32_t));
  if (e == hipSuccess && weights) e = alloc((void**)&g->d_w, (ne + kPad) * sizeof(uint32_t));
  if (e == hipSuccess && labels) e = alloc((void**)&g->d_lab, ne + kPad);
  if (e == hipSuccess) e = hipMemset(g->d_adj + ne, 0, kPad * sizeof(uint32_t));
  if (e == hipSuccess && weights) e = hipMemset(g->d_w + ne, 0, kPad * sizeof(uint32_t));
  if (e == hipSuccess && labels) e = hipMemset(g->d_lab + ne, 0, kPad);
  if (e == hipSuccess) e = alloc((void**)&g->d_status, 256);
  if (e == hipSuccess)
    e = alloc((void**)&g->d_head, fw::kHeadSlots * fw::kHeadStride * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemcpy(g->d_off, off, (nv + 1) * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && ne) e = hipMemcpy(g->d_adj, adj, ne * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && weights && ne)
    e = hipMemcpy(g->d_w, weights, ne * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && labels && ne) e = hipMemcpy(g->d_lab, labels, ne, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(g->d_status, 0, 256);
  if (e == hipSuccess)
    e = hipMemset(g->d_head, 0, fw::kHeadSlots * fw::kHeadStride * sizeof(uint64_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    const int rc = (e == hipErrorOutOfMemory) ? fail(FW_ENOMEM, "device allocation")
                                              : hip_fail(e, "uploading the graph");
    fw_graph_free(g);
    return rc;
  }
  *out = g;
  return FW_OK;
}

int fw_graph_free(fw_graph* g) {
  if (!g) return FW_OK;
  (void)hipFree(g->d_off);
  (void)hipFree(g->d_adj);
  (void)hipFree(g->d_w);
  (void)hipFree(g->d_lab);
  (void)hipFree(g->d_status);
  (void)hipFree(g->d_head);
  fw::release_graph_state(g);
  delete g;
  return FW_OK;
}

int fw_graph_info_get(const fw_graph* g, fw_graph_info* out) {
  if (!g || !out) return fail(FW_EINVAL, "NULL argument");
  out->n_vertices = g->nv;
  out->n_edges = g->ne;
  out->max_degree = g->max_deg;
  out->max_weight = g->max_w;
  out->device_bytes = g->bytes;
  out->weighted = g->d_w != nullptr;
  out->labelled = g->d_lab != nullptr;
  out->device = g->device;
  return FW_OK;
}

int fw_walk_ex(const fw_graph* g, fw_algo algo, const fw_params* params,
               const uint32_t* starts, uint64_t n, uint32_t length, uint64_t seed,
               uint32_t* out_paths, const fw_walk_opts* opts) {
  fw::DevParams dp;
  int rc = fw::check_walk_args(g, (int)algo, params, n, length, starts, out_paths, &dp);
  if (rc) return rc;
  if (n == 0) return FW_OK;
  fw_walk_opts o{};
  if (opts) o = *opts;
  hipStream_t stream = (hipStream_t)o.stream;
  fw::LaunchArgs a;
  a.algo = (int)algo;
  a.g = fw::dev_graph(g);
  a.prm = dp;
  a.starts = starts;
  a.n = n;
  a.length = length;
  a.seed = seed;
  a.qid_base = o.qid_base;
  a.out = out_paths;
  a.status = g->d_status;
  a.head = g->d_head + fw::kHeadStride * (g->launches.fetch_add(1) % fw::kHeadSlots);
  a.num_cus = g->num_cus;
  hipError_t e;
  if (o.sampler != FW_SAMPLER_ITS) {
    if (o.sampler != FW_SAMPLER_DPRS && o.sampler != FW_SAMPLER_ZPRS)
      return fail(FW_EINVAL, "unknown sampler");
    if (o.mode != FW_MODE_PLAIN)
      return fail(FW_EINVAL, "the reservoir samplers run in FW_MODE_PLAIN");
    e = fw::launch_reservoir(a, o.sampler, stream);
  } else if (o.mode == FW_MODE_PLAIN) {
    e = fw::launch_plain(a, stream);
  } else if (o.mode == FW_MODE_PERSISTENT || o.mode == FW_MODE_AUTO ||
             o.mode == FW_MODE_STAGED) {
    bool staged = false;
    rc = fw::resolve_tune(g, (int)algo, o.mode, o.tune, &a.cfg, &staged);
    if (rc) return rc;
    a.cfg.narrow = fw::narrow_products(g->max_w, dp);
    e = fw::launch_persistent_checked(g, a, stream, o.use_graph != 0, staged);
  } else {
    return fail(FW_EINVAL, "unknown mode");
  }
  if (e != hipSuccess) return hip_fail(e, "launching the walk");
  if (o.async) return FW_OK;
  return fw::read_status(g, stream);
}

int fw_walk(const fw_graph* g, fw_algo algo, const fw_params* params, const uint32_t* starts,
            uint64_t n, uint32_t length, uint64_t seed, uint32_t* out_paths) {
  return fw_walk_ex(g, algo, params, starts, n, length, seed, out_paths, nullptr);
}

int fw_autotune(fw_graph* g, fw_algo algo, const fw_params* params, const uint32_t* starts,
                uint64_t n, uint32_t length, uint64_t seed, void* stream, fw_tune* best) {
  fw::DevParams dp;
  int rc = fw::check_walk_args(g, (int)algo, params, n, length, starts, starts, &dp);
  if (rc) return rc;
  if (n == 0) return fw::set_error(FW_EINVAL, "empty sample");
  fw::TuneCfg c;
  bool staged = false;
  rc = fw::autotune(g, (int)algo, dp, starts, n, length, seed, (hipStream_t)stream, &c, &staged);
  if (rc) return rc;
  if (best) {
    std::memset(best, 0, sizeof(*best));
    best->wg_size = c.wg_size;
    best->slots = c.slots;
    best->tiny_max = c.tiny_max;
    best->hub_min = c.hub_min;
    best->wgs_per_cu = c.wgs_per_cu;
    best->hash_cells = c.hash_cells;
    best->mode = staged ? FW_MODE_STAGED : FW_MODE_PERSISTENT;
    best->sparse_ratio = c.sparse_ratio ? c.sparse_ratio : 0xFFFFFFFFu;
  }
  return FW_OK;
}

int fw_count_steps(const uint32_t* out_paths, uint64_t n, uint32_t length, void* stream,
                   uint64_t* steps) {
  if (!steps) return fail(FW_EINVAL, "steps is NULL");
  *steps = 0;
  if (n == 0 || length == 0) return FW_OK;
  if (!out_paths) return fail(FW_EINVAL, "out_paths is NULL");
  const uint64_t cols = (uint64_t)length + 1;
  if (n > UINT64_MAX / cols) return fail(FW_EINVAL, "n * (length + 1) overflows");
  const uint64_t m = n * cols;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long* d_total = nullptr;
  hipError_t e = hipMalloc(&d_total, sizeof(unsigned long long));
  if (e != hipSuccess) return hip_fail(e, "allocating the step counter");
  unsigned long long total = 0;
  e = hipMemsetAsync(d_total, 0, sizeof(unsigned long long), st);
  if (e == hipSuccess) {
    const uint64_t blocks = std::min<uint64_t>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(fw::k_count_not_end, dim3((unsigned)blocks), dim3(256), 0, st, out_paths,
                       m, d_total);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(&total, d_total, sizeof(total), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(d_total);
  if (e != hipSuccess) return hip_fail(e, "counting steps");
  // Column 0 holds the start vertex of every row (never FW_END).
  *steps = total >= n ? total - n : 0;
  return FW_OK;
}

int fw_sync(const fw_graph* g, void* stream) {
  if (!g) return fail(FW_EINVAL, "graph is NULL");
  return fw::read_status(g, (hipStream_t)stream);
}

}  // extern "C"
