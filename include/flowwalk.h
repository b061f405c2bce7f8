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
 *   FW_PPR       the personalized-PageRank walk of the experiments (section
 *                6.1): w'_i = w_i, and before every hop the query stops
 *                with chance stop_num / stop_den, tossed on word 1 of the
 *                same Philox block: it stops when
 *                floor(word1 * stop_den / 2^64) < stop_num.  `length` caps
 *                its hops.
 * A hop whose total T is 0 (no neighbours, or every neighbour masked) ends
 * the walk, as does a PPR stop; the remaining entries of its row are FW_END.
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

typedef enum { FW_DEEPWALK = 0, FW_NODE2VEC = 1, FW_METAPATH = 2, FW_PPR = 3 } fw_algo;

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
 * label schema, 1 <= schema_len <= 16, cycled.  stop_num / stop_den: PPR's
 * stop chance per hop, 0 <= stop_num <= stop_den, stop_den > 0 (the
 * experiments use 1/5). */
typedef struct fw_params {
  uint32_t f_ret, f_in, f_out;
  uint32_t schema_len;
  uint8_t schema[16];
  uint32_t stop_num, stop_den;
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
 * Every degree must be below 2^28.
 * Errors: FW_EINVAL (NULL pointers, malformed CSR, a degree of 2^28 or
 * more), FW_ENOMEM, FW_EHIP. */
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
 *   params     ignored for FW_DEEPWALK (may be NULL); required otherwise
 * Runs on the null stream and returns when the walks are done.
 * Errors: FW_EINVAL (bad algorithm or parameters, MetaPath on a graph
 * without labels, a PPR stop chance outside [0, 1], NULL pointers, a start
 * vertex >= V: then out_paths is
 * unspecified), FW_EOVERFLOW, FW_EHIP. */
int fw_walk(const fw_graph* g, fw_algo algo, const fw_params* params, const uint32_t* starts,
            uint64_t n, uint32_t length, uint64_t seed, uint32_t* out_paths);

/* Kernel choice for fw_walk_ex.
 *   FW_MODE_PLAIN       one wavefront per query, queries assigned statically
 *                       (no load balancing: the baseline).
 *   FW_MODE_PERSISTENT  persistent wavefronts that claim queries from a
 *                       global atomic head (dynamic scheduling, section 5.2);
 *                       each keeps four queries, batches tiny-degree hops
 *                       four to a wavefront and runs the others on the whole
 *                       wavefront (sampler organisation of section 5.1).
 *   FW_MODE_AUTO        FW_MODE_PERSISTENT with the tuned configuration.
 *   FW_MODE_STAGED      the paper's two-stage block design on wave64:
 *                       persistent workgroups with an LDS task pool, wave
 *                       samplers, then a whole-workgroup sampler for hubs. */
typedef enum {
  FW_MODE_AUTO = 0,
  FW_MODE_PLAIN = 1,
  FW_MODE_PERSISTENT = 2,
  FW_MODE_STAGED = 3
} fw_mode;

/* Launch configuration of the persistent and staged forms (0 in any field =
 * the tuned or default value).
 *   persistent: tiny_max, wgs_per_cu (256-thread workgroups per CU),
 *               hash_cells (LDS cells per wavefront, power of two >= 64);
 *   staged:     wg_size, slots, tiny_max, hub_min, wgs_per_cu,
 *               hash_cells (LDS cells per workgroup). */
typedef struct fw_tune {
  uint32_t wg_size;      /* staged: threads per workgroup, 256/512/1024 */
  uint32_t slots;        /* staged: local task-pool slots, <= 128 */
  uint32_t tiny_max;     /* degree <= tiny_max (<= 16): sub-wave sampler */
  uint32_t hub_min;      /* staged: degree >= hub_min: workgroup sampler */
  uint32_t wgs_per_cu;   /* resident workgroups per compute unit */
  uint32_t fetch;        /* reserved, 0 */
  uint32_t hash_cells;   /* LDS cells for the node2vec membership structure */
  uint32_t mode;         /* fw_autotune's output: the form FW_MODE_AUTO runs,
                            FW_MODE_PERSISTENT or FW_MODE_STAGED (ignored as
                            input) */
  uint32_t sparse_ratio; /* persistent node2vec: a hop whose degree is at
                            least 2048 and at least sparse_ratio times
                            d(prev) computes its total from the raw weights
                            and looks N(prev)'s ids up in N(cur), instead of
                            testing every entry of N(cur) against N(prev)
                            (0 = tuned/default 128, 0xFFFFFFFF = never) */
} fw_tune;

/* How each hop picks its neighbour (fw_walk_opts.sampler).
 *   FW_SAMPLER_ITS   the exact inverse-CDF pick above (every mode).
 *   FW_SAMPLER_DPRS  direct parallel reservoir sampling (Algorithm 3);
 *   FW_SAMPLER_ZPRS  zig-zag parallel reservoir sampling (Algorithm 4).
 * The reservoir samplers draw one word per entry i of the neighbour
 * sequence, word i mod 4 of Philox4x64-10(counter = (qid, t, i / 4, 1),
 * key = (seed, 0)), and visiting entry i with running total W (including
 * it) select it when floor(u_i * W / 2^64) < w'_i; the last selection is
 * the pick.  DPRS visits the entries in CSR order.  ZPRS visits them in the
 * zig-zag order of 64 lanes over quads: lane j owns quads j, j + 64, ...
 * (quad q = entries 4q .. 4q + 3), lane 0's entries first.  Both pick
 * neighbour i with chance w'_i / T (Propositions 1 and 2), but not the same
 * neighbour as ITS or as each other.  They run in FW_MODE_PLAIN only; node2vec
 * membership is a binary search of N(prev) per entry, as in the paper. */
typedef enum { FW_SAMPLER_ITS = 0, FW_SAMPLER_DPRS = 1, FW_SAMPLER_ZPRS = 2 } fw_sampler;

typedef struct fw_walk_opts {
  int mode;               /* fw_mode */
  void* stream;           /* hipStream_t to run on (NULL = null stream) */
  int async;              /* 1: return after enqueueing; errors detected in
                             the kernel are then reported by fw_sync */
  uint64_t qid_base;      /* query i has id qid_base + i (default 0) */
  const fw_tune* tune;    /* NULL = tuned/default configuration */
  int use_graph;          /* 1: replay a captured hipGraph of the launch
                             (persistent form; ignored otherwise) */
  int sampler;            /* fw_sampler (0 = FW_SAMPLER_ITS) */
} fw_walk_opts;

/* fw_walk with options (opts may be NULL: synchronous FW_MODE_AUTO on the
 * null stream).  Same results bit for bit in every mode. */
int fw_walk_ex(const fw_graph* g, fw_algo algo, const fw_params* params,
               const uint32_t* starts, uint64_t n, uint32_t length, uint64_t seed,
               uint32_t* out_paths, const fw_walk_opts* opts);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the walk of
 * fw_walk in FW_MODE_PERSISTENT with the graph's tuned configuration,
 * enqueued on `stream` (a hipStream_t, NULL = null stream) without waiting
 * and without allocating anything.  The task-pool head counter its
 * wavefronts claim queries from lives in a 256-byte static device array of
 * the library, one per GPU, held until the process ends (the other entry
 * points use counters allocated with the graph).  That counter is shared by
 * every fw_walk_noalloc call on the GPU: calls whose launches overlap on the
 * device (on different streams, or from several threads) race and may skip
 * or repeat queries; calls on one stream run one after the other and are
 * safe.  Each launch resets the counter with a one-thread kernel (no memset).
 * Arguments and rows as fw_walk's (query i has id i).  The graph must live
 * on the current device.  Host-side argument errors are returned; a start
 * vertex >= V found by the kernel is reported by fw_sync on the same stream.
 * Errors: as fw_walk, FW_EINVAL for a graph of another device, FW_EHIP. */
int fw_walk_noalloc(const fw_graph* g, fw_algo algo, const fw_params* params,
                    const uint32_t* starts, uint64_t n, uint32_t length, uint64_t seed,
                    uint32_t* out_paths, void* stream);

/* Autotuner (the hyper-parameter study of Appendix C.2, run on the target
 * GPU): times candidate configurations on the n queries of `starts`
 * (device, a sample of the real query set):
 *   persistent form: resident workgroups per CU, node2vec membership-table
 *     size, then the tiny-degree threshold (coordinate search);
 *   staged form (the paper's block design): threads per workgroup
 *     (256/512/1024), hub threshold d_t (1024/4096/16384) and local pool
 *     size |P_L| (32/64).
 * The fastest of each form is kept for the graph and `algo`, keyed by the
 * graph's fingerprint (sizes, degree and weight maxima, and sampled offsets,
 * ids, weights and labels) and device, so a re-upload of the same graph
 * finds it; FW_MODE_AUTO runs the faster form, FW_MODE_PERSISTENT and
 * FW_MODE_STAGED their own tuned configuration (walks and servers created
 * afterwards that pass no explicit fw_tune).  The winner is copied to *best
 * (may be NULL; best->mode names its form).  Runs on `stream` and blocks;
 * allocates a temporary n * (length + 1) output.
 * Errors: as fw_walk, FW_ENOMEM. */
int fw_autotune(fw_graph* g, fw_algo algo, const fw_params* params, const uint32_t* starts,
                uint64_t n, uint32_t length, uint64_t seed, void* stream, fw_tune* best);

/* Results larger than device memory (section 5.2, Eq. 5).  fw_walk_host
 * runs n queries whose rows go to host memory, in batches of
 *     B = floor(device_budget_bytes / (2 * (length + 2) * 4))
 * queries (each of two ping-pong buffers holds a batch's start vertices and
 * its rows of length + 1 entries; Eq. 5 with M - M_G = the budget), capped at
 * max_batch_queries when that is non-zero.  Consecutive batches alternate
 * between two streams, so one batch's device-to-host copy overlaps the next
 * batch's walk.  Query i has id i: the rows equal fw_walk's. */
typedef struct fw_batch_opts {
  uint64_t device_budget_bytes;  /* 0 = the free device memory less 1 GiB */
  uint64_t max_batch_queries;    /* 0 = no cap */
  int mode;                      /* fw_mode of each batch (0 = FW_MODE_AUTO) */
  uint64_t batch_queries;        /* out: B */
  uint32_t batches;              /* out: number of batches */
} fw_batch_opts;

/*   starts_host  host, uint32[n]
 *   out_host     host, uint32[n * (length + 1)], row-major as fw_walk's
 *   opts         may be NULL (defaults); receives B and the batch count
 * Allocates two device buffers of B queries, two pinned host staging
 * buffers and two streams for the call, and blocks until every row is in
 * out_host.  Errors: as fw_walk (start vertices are checked on the host
 * first), FW_EINVAL when the budget holds no query, FW_ENOMEM, FW_EHIP. */
int fw_walk_host(const fw_graph* g, fw_algo algo, const fw_params* params,
                 const uint32_t* starts_host, uint64_t n, uint32_t length, uint64_t seed,
                 uint32_t* out_host, fw_batch_opts* opts);

/* Realised hops of a walk result (Alg. 1: a step is one appended vertex):
 * the entries of columns 1..length of the n x (length + 1) row-major device
 * matrix out_paths that are not FW_END, written to *steps (host).  Runs on
 * `stream` (a hipStream_t, NULL = null stream) after the work already queued
 * there and blocks until the count is known; allocates 8 bytes of device
 * memory for the call.  out_paths must hold a completed walk result (column
 * 0 = the start vertices).  Errors: FW_EINVAL (steps NULL, out_paths NULL
 * with n * length > 0, size overflow), FW_EHIP. */
int fw_count_steps(const uint32_t* out_paths, uint64_t n, uint32_t length, void* stream,
                   uint64_t* steps);

/* Sampler microbenchmark (the comparison of sampling methods, section 6.3,
 * and of rejection sampling, Appendix C).  n_tasks independent tasks; task j
 * picks one index i of the weights w = weights[j * size .. (j + 1) * size)
 * with chance w_i / T, T = sum(w), and writes it to picks[j] (FW_END when
 * T = 0, or when REJECTION rejected FW_RJS_MAX_TRIALS candidates).
 *   FW_TASK_ITS           the walkers' bufferless two-pass pick: word 0 u of
 *                         Philox4x64-10(counter (j, 0, 0, 0), key (seed, 0)),
 *                         r = floor(u T / 2^64), first prefix above r;
 *   FW_TASK_DPRS / ZPRS   the reservoir samplers of fw_sampler, entry i's word
 *                         from counter (j, 0, i / 4, 1);
 *   FW_TASK_ITS_BUFFERED  the same pick as FW_TASK_ITS from an O(size) array
 *                         of prefix sums (a device scratch slice per task in
 *                         flight) and a binary search;
 *   FW_TASK_ALIAS         Vose's alias table (capacities in units of w_i *
 *                         size, so exact) built by an index-order sweep:
 *                         the current heavy item fills the light items in
 *                         order, and once its remaining mass is at most T it
 *                         becomes a column filled from the next heavy item;
 *                         then words u0, u1 of counter (j, 0, 0, 2) pick
 *                         column c = floor(u0 size / 2^64), kept when
 *                         floor(u1 T / 2^64) < prob[c], else its alias;
 *   FW_TASK_REJECTION     trial k: words u0, u1 of counter (j, k, 0, 3),
 *                         candidate c = floor(u0 size / 2^64), accepted when
 *                         floor(u1 wmax / 2^64) < w_c; the first accepted
 *                         trial wins.
 *   weights  device, uint32[n_tasks * size]; picks  device, uint32[n_tasks]
 * Runs on `stream` and blocks until done; the buffered samplers allocate at
 * most 8 GiB of scratch for the call.  Errors: FW_EINVAL (unknown sampler,
 * size 0 or >= 2^28, NULL pointers, size overflow), FW_ENOMEM, FW_EHIP. */
typedef enum {
  FW_TASK_ITS = 0,
  FW_TASK_DPRS = 1,
  FW_TASK_ZPRS = 2,
  FW_TASK_ITS_BUFFERED = 3,
  FW_TASK_ALIAS = 4,
  FW_TASK_REJECTION = 5
} fw_task_sampler;
#define FW_RJS_MAX_TRIALS (1u << 24)

int fw_sample_tasks(int sampler, const uint32_t* weights, uint64_t n_tasks, uint32_t size,
                    uint64_t seed, uint32_t* picks, void* stream);

/* Waits for `stream` (a hipStream_t, NULL = null stream) and returns the
 * status that kernels of graph g detected since the last check (FW_EINVAL
 * for a start vertex >= V), clearing it. */
int fw_sync(const fw_graph* g, void* stream);

/* ------------------------------------------------------------------------
 * Served form: continuous batching of walk requests (graph and in-flight
 * walks resident in HBM).  Requests are admitted in arrival order while
 * their device memory, a 256-byte hop counter plus n * 4 bytes of start
 * vertices (rounded up to 256) plus n * (length + 1) * 4 bytes of rows,
 * fits in mem_budget_bytes (the per-request form of Eq. 5's rule that
 * result memory bounds the batch, section 5.2).  Admitted requests run as
 * multi-request persistent launches on up to max_inflight streams at once,
 * so work that arrives while other work is on the GPU joins it there.  A
 * request's walks equal fw_walk's on the same starts and seed (query i of
 * the request has id i), alone or in any mix.
 * ---------------------------------------------------------------------- */
typedef struct fw_server fw_server;

typedef struct fw_server_opts {
  uint64_t mem_budget_bytes;   /* device bytes for request buffers (default 1 GiB) */
  uint32_t max_inflight;       /* concurrent batches / streams (default 3, <= 16) */
  uint32_t max_batch_requests; /* requests per batch (default 256, <= 4096) */
  uint32_t small_max_queries;  /* non-zero: requests of at most this many
                                  queries run in their batch's first phase and
                                  complete without waiting for its larger
                                  requests (default 0: one phase; on the
                                  R-MAT-24 mix a split at 2048 raised p50 and
                                  p99 at 1000 requests/s) */
  uint32_t express_max_queries; /* non-zero: one of the max_inflight streams is
                                  an express lane for requests of at most this
                                  many queries (taken from anywhere in the
                                  queue), with 2 workgroups per CU kept for it;
                                  the other streams share the rest (default 0) */
} fw_server_opts;

typedef struct fw_req_stats {
  uint64_t submit_ns, admit_ns, done_ns; /* steady-clock timestamps */
  uint64_t n;
  uint32_t length;
  int status;
  uint64_t steps; /* realised hops of the request's walks (Alg. 1: one per
                     appended vertex), counted on the device */
} fw_req_stats;

/* Creates a server for graph g (which must outlive it): allocates the device
 * arena and its pinned mirror, the streams, and starts the scheduler thread.
 * opts may be NULL (defaults).  Errors: FW_EINVAL, FW_ENOMEM, FW_EHIP. */
int fw_server_create(const fw_graph* g, const fw_server_opts* opts, fw_server** out);

/* Queues a request (thread-safe).  starts_host: host uint32[n], copied; every
 * start must be < n_vertices (checked here).  *ticket identifies it.
 * Errors: FW_EINVAL (as fw_walk, n = 0), FW_EOVERFLOW, FW_ENOMEM (larger
 * than the whole budget), FW_ECANCELED (server shutting down). */
int fw_server_submit(fw_server* s, fw_algo algo, const fw_params* params,
                     const uint32_t* starts_host, uint64_t n, uint32_t length, uint64_t seed,
                     uint64_t* ticket);

/* 1 if the request has finished (successfully or not), 0 if not yet,
 * FW_EINVAL for an unknown ticket. */
int fw_server_poll(fw_server* s, uint64_t ticket);

/* Blocks until the request finishes, copies its n * (length + 1) path
 * entries to out_host (host, may be NULL), fills *stats (may be NULL), and
 * releases the request and its memory.  Returns the request's status
 * (FW_ECANCELED if the server shut down first).  Requests may be waited for
 * in any order: a finished request gives its device memory back at once and
 * keeps its rows in the server's pinned host staging (twice
 * mem_budget_bytes) until it is collected; when the next request in arrival
 * order finds no staging left, uncollected rows move to ordinary host
 * memory (held until the wait).  A ticket is waited for once: another wait
 * for it, also one from another thread while the first blocks, returns
 * FW_EINVAL. */
int fw_server_wait(fw_server* s, uint64_t ticket, uint32_t* out_host, fw_req_stats* stats);

/* Stops admitting, cancels queued requests (FW_ECANCELED), waits for
 * launched batches and for threads blocked in fw_server_wait, frees all. */
int fw_server_destroy(fw_server* s);

/* Message for the last failure on this thread ("" if none). */
const char* fw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
