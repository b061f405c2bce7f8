/* flowwalk.h - C ABI of the MI355X (gfx950) dynamic-graph random-walk library.
 *
 * The library runs random-walk queries over a CSR graph resident in HBM.
 * Every hop computes the transition weight of each neighbour of the current
 * vertex on the fly (the initialisation phase of Algorithm 1, section 2.1)
 * and then picks one neighbour with probability proportional to it (the
 * selection phase), without any per-vertex or per-query buffer in device
 * memory (the memory property of section 5.3).  The pick is an exact integer
 * inverse-CDF draw: with w'_i the transition weights of the d neighbours in
 * CSR order and T = sum(w'_i) (64-bit),
 *     u = word 0 of Philox4x64-10(counter = (qid, t, 0, 0), key = (seed, 0))
 *     r = floor(u * T / 2^64)
 *     next = neighbour i* = min { i : w'_0 + ... + w'_i > r },
 * so every walk is a pure function of (graph, algorithm, parameters, seed,
 * query id, start vertex) and is reproducible bit for bit.
 *
 * Transition weights (section 2.1; w = edge weight, 1 when the graph has
 * none):
 *   FW_DEEPWALK  w'_i = w_i.
 *   FW_NODE2VEC  Eq. 2 times w_i, with integer factors for 1/a, 1, 1/b:
 *                f_ret if u_i is the previous vertex, else f_in if u_i is a
 *                neighbour of the previous vertex (binary search in its
 *                sorted row), else f_out.  The first hop (t = 0) has no
 *                previous vertex and uses w_i alone.
 *   FW_METAPATH  Eq. 1 times w_i: w_i if label_i == schema[t mod schema_len],
 *                else 0.
 * A hop whose total T is 0 (no neighbours, or every neighbour masked) ends
 * the walk; the remaining entries of its row are FW_END.
 *
 * Conventions.  Every function returns an int status (FW_OK or a negative
 * FW_E* code) and never throws.  fw_last_error() gives a message for the
 * last failure on the calling thread.  Pointers documented as "device" must
 * point to memory of the current HIP device (hipMalloc, or a torch CUDA
 * tensor's data_ptr()); "host" pointers to ordinary host memory.
 */
#ifndef FLOWWALK_H
#define FLOWWALK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FW_OK 0
#define FW_EINVAL (-1)     /* bad argument, malformed CSR, start vertex >= V */
#define FW_ENOMEM (-2)     /* device or host allocation failed */
#define FW_EOVERFLOW (-3)  /* max_w * max_factor * max_degree >= 2^64 */
#define FW_EHIP (-4)       /* a HIP runtime call failed */
#define FW_ECANCELED (-5)  /* request cancelled (server shut down) */

#define FW_END 0xFFFFFFFFu /* path entry after an early end */

typedef enum { FW_DEEPWALK = 0, FW_NODE2VEC = 1, FW_METAPATH = 2 } fw_algo;

/* Host CSR view (section 2.1: G = (V, E), N(v), d(v)).
 *   offsets  host, uint64[n_vertices + 1], offsets[0] = 0, non-decreasing,
 *            offsets[n_vertices] = n_edges
 *   adj      host, uint32[n_edges]; row v = adj[offsets[v] .. offsets[v+1])
 *            sorted ascending (a repeated id is a parallel edge and is its
 *            own candidate); every id < n_vertices
 * n_vertices must be below 2^32 - 1 (FW_END is reserved). */
typedef struct fw_csr {
  uint64_t n_vertices, n_edges;
  const uint64_t* offsets;
  const uint32_t* adj;
} fw_csr;

/* Algorithm parameters.  f_ret, f_in, f_out: node2vec integer factors (see
 * fw_node2vec_factors); not all zero.  schema[0 .. schema_len): MetaPath
 * label schema, 1 <= schema_len <= 16, cycled. */
typedef struct fw_params {
  uint32_t f_ret, f_in, f_out;
  uint32_t schema_len;
  uint8_t schema[16];
} fw_params;

typedef struct fw_graph fw_graph; /* opaque device-resident graph */

typedef struct fw_graph_info {
  uint64_t n_vertices, n_edges;
  uint64_t max_degree;   /* max over v of d(v) */
  uint64_t max_weight;   /* max edge weight (1 for an unweighted graph) */
  uint64_t device_bytes; /* HBM held by the graph and its walk state */
  int weighted, labelled, device;
} fw_graph_info;

/* Validates a host CSR (O(V + E), multi-threaded) and copies it, with the
 * optional per-edge weights (host uint32[n_edges], NULL = all 1) and labels
 * (host uint8[n_edges], NULL = none), into HBM of the current device.  The
 * library owns the device copy; the caller keeps its host arrays.
 * Errors: FW_EINVAL (NULL pointers, malformed CSR), FW_ENOMEM, FW_EHIP. */
int fw_graph_upload(const fw_csr* csr, const uint32_t* weights, const uint8_t* labels,
                    fw_graph** out);

/* Frees the device copy and the handle (NULL is accepted). */
int fw_graph_free(fw_graph* g);

/* Fills *out with the graph's sizes. */
int fw_graph_info_get(const fw_graph* g, fw_graph_info* out);

/* Eq. 2's factors 1/a, 1, 1/b for a = p_num/p_den and b = q_num/q_den
 * (a is p, the return parameter; b is q, the in-out parameter), scaled to
 * the smallest integers: (p_den*q_num, p_num*q_num, p_num*q_den) / gcd.
 * Fills f_ret, f_in, f_out of *out and leaves its schema alone.
 * Errors: FW_EINVAL (a zero argument, a factor >= 2^32). */
int fw_node2vec_factors(uint32_t p_num, uint32_t p_den, uint32_t q_num, uint32_t q_den,
                        fw_params* out);

/* Runs n walk queries of `length` hops.
 *   starts     device, uint32[n]: query i (id i) starts at starts[i]
 *   out_paths  device, uint32[n * (length + 1)], row-major: row i receives
 *              the start and then one vertex per hop, FW_END after an early
 *              end.  length = 0 gives rows [start].  n = 0 is a no-op.
 *   params     ignored for FW_DEEPWALK (may be NULL)
 * Runs on the null stream and returns when the walks are done.
 * Errors: FW_EINVAL (bad algorithm or parameters, MetaPath on a graph
 * without labels, NULL pointers, a start vertex >= V: then out_paths is
 * unspecified), FW_EOVERFLOW, FW_EHIP. */
int fw_walk(const fw_graph* g, fw_algo algo, const fw_params* params, const uint32_t* starts,
            uint64_t n, uint32_t length, uint64_t seed, uint32_t* out_paths);

/* Kernel choice for fw_walk_ex.
 *   FW_MODE_PLAIN       one wavefront per query, queries assigned statically
 *                       (no load balancing: the baseline).
 *   FW_MODE_PERSISTENT  persistent workgroups with a local slot pool refilled
 *                       from a global atomic head (dynamic scheduling,
 *                       section 5.2), degree-class samplers (sub-wave, wave,
 *                       whole workgroup; section 5.1).
 *   FW_MODE_AUTO        the persistent form with the tuned configuration. */
typedef enum { FW_MODE_AUTO = 0, FW_MODE_PLAIN = 1, FW_MODE_PERSISTENT = 2 } fw_mode;

/* Launch configuration of the persistent form (0 in any field = default). */
typedef struct fw_tune {
  uint32_t wg_size;      /* threads per workgroup: 256, 512 or 1024 */
  uint32_t slots;        /* local task-pool slots per workgroup, <= 256 */
  uint32_t tiny_max;     /* degree <= tiny_max: sub-wave sampler */
  uint32_t hub_min;      /* degree >= hub_min: whole-workgroup sampler */
  uint32_t wgs_per_cu;   /* persistent workgroups per compute unit */
  uint32_t fetch;        /* reserved, 0 */
  uint32_t hash_cells;   /* LDS cells per workgroup for the node2vec
                            membership hash set (power of two) */
} fw_tune;

typedef struct fw_walk_opts {
  int mode;               /* fw_mode */
  void* stream;           /* hipStream_t to run on (NULL = null stream) */
  int async;              /* 1: return after enqueueing; errors detected in
                             the kernel are then reported by fw_sync */
  uint64_t qid_base;      /* query i has id qid_base + i (default 0) */
  const fw_tune* tune;    /* NULL = tuned/default configuration */
  int use_graph;          /* 1: replay a captured hipGraph of the launch
                             (persistent form; ignored otherwise) */
} fw_walk_opts;

/* fw_walk with options (opts may be NULL: synchronous FW_MODE_AUTO on the
 * null stream).  Same results bit for bit in every mode. */
int fw_walk_ex(const fw_graph* g, fw_algo algo, const fw_params* params,
               const uint32_t* starts, uint64_t n, uint32_t length, uint64_t seed,
               uint32_t* out_paths, const fw_walk_opts* opts);

/* Waits for `stream` (a hipStream_t, NULL = null stream) and returns the
 * status that kernels of graph g detected since the last check (FW_EINVAL
 * for a start vertex >= V), clearing it. */
int fw_sync(const fw_graph* g, void* stream);

/* Message for the last failure on this thread ("" if none). */
const char* fw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
