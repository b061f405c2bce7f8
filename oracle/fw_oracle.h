/* CPU oracle for graph random walks (DeepWalk, node2vec, MetaPath, PPR).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * definition that the HIP library is checked against, bit for bit.  Only the
 * test suite, the smoke check and the bench's CPU-baseline leg may load it;
 * the product library never does, and the two share no code.
 *
 * What one walk computes (Algorithm 1, "Random Walk Computation Paradigm",
 * section 2.1): from the start vertex, each step computes the transition
 * weight of every neighbour of the current vertex (initialisation phase) and
 * then picks one neighbour with probability proportional to it (selection
 * phase).  The weights are those of section 2.1: the edge weight (weighted
 * DeepWalk), Eq. 2 times the edge weight (node2vec), Eq. 1 times the edge
 * weight (MetaPath).  The pick is inverse transform sampling (section 2.2)
 * over exact integer prefix sums, driven by one Philox4x64-10 draw per step
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC 2011).  Both the reservoir samplers of section 4 (Propositions 1 and 2)
 * and this pick select neighbour i with probability w'_i / sum(w').
 *
 * PPR (the personalized-PageRank walk of the experiments, section 6.1) moves
 * like weighted DeepWalk but ends before each hop with a fixed stop chance;
 * the coin is word 1 of the hop's Philox block, the draw stays word 0.
 */
#ifndef FW_ORACLE_H
#define FW_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (same numeric values as the library's, defined separately). */
#define FWO_OK 0
#define FWO_EINVAL (-1)
#define FWO_ENOMEM (-2)
#define FWO_EOVERFLOW (-3)

#define FWO_DEEPWALK 0
#define FWO_NODE2VEC 1
#define FWO_METAPATH 2
#define FWO_PPR 3

#define FWO_END 0xFFFFFFFFu /* path padding after an early end */

/* Host CSR view.  offsets[V+1], adj[E] with each row sorted ascending;
 * weights[E] (NULL = every weight 1); labels[E] (NULL = no labels). */
typedef struct {
  uint64_t n_vertices, n_edges;
  const uint64_t* offsets;
  const uint32_t* adj;
  const uint32_t* weights;
  const uint8_t* labels;
} fwo_graph;

/* Integer node2vec factors (return, in-out: stay near prev, move away), the
 * MetaPath label schema, cycled: hop t uses schema[t mod schema_len], and
 * PPR's stop chance stop_num / stop_den (0 <= stop_num <= stop_den, 0 < stop_den). */
typedef struct {
  uint32_t f_ret, f_in, f_out;
  uint32_t schema_len;
  uint8_t schema[16];
  uint32_t stop_num, stop_den;
} fwo_params;

/* Philox4x64 with 10 rounds; out[0..3] for counter ctr[0..3], key key[0..1]. */
void fwo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* The step draw: word 0 of Philox4x64-10(counter = (qid, t, 0, 0),
 * key = (seed, 0)). */
uint64_t fwo_draw(uint64_t seed, uint64_t qid, uint64_t t);

/* PPR's coin on a uniform 64-bit word u1: 1 (stop) when
 * floor(u1 * stop_den / 2^64) < stop_num, i.e. with chance stop_num / stop_den
 * up to 2^-64. */
int fwo_stop_coin(uint64_t u1, uint32_t stop_num, uint32_t stop_den);

/* Does PPR query qid stop before hop t?  The coin on word 1 of
 * Philox4x64-10(counter = (qid, t, 0, 0), key = (seed, 0)). */
int fwo_stop(uint64_t seed, uint64_t qid, uint64_t t, uint32_t stop_num, uint32_t stop_den);

/* floor(u * total / 2^64): maps a uniform 64-bit word to [0, total). */
uint64_t fwo_scale(uint64_t u, uint64_t total);

/* Inverse CDF: smallest i with w[0] + ... + w[i] > r, or -1 when r is not
 * below the total. */
int64_t fwo_pick(const uint64_t* w, uint64_t d, uint64_t r);

/* p, q as rationals -> reduced integer factors proportional to (1/p, 1, 1/q).
 * Returns FWO_EINVAL for a zero numerator/denominator or factors >= 2^32. */
int fwo_node2vec_factors(uint32_t p_num, uint32_t p_den, uint32_t q_num, uint32_t q_den,
                         fwo_params* out);

/* Checks the CSR: offsets[0] = 0, monotone, offsets[V] = E, every id < V,
 * rows ascending (a repeated id is a parallel edge, its own candidate),
 * V < 2^32 - 1. */
int fwo_validate(const fwo_graph* g);

/* Transition weights of every neighbour of `cur` at hop t (prev is ignored at
 * t = 0).  w_out receives d(cur) values.  Returns FWO_OK or FWO_EINVAL. */
int fwo_transition_weights(const fwo_graph* g, int algo, const fwo_params* p, uint32_t prev,
                           uint32_t cur, uint32_t t, uint64_t* w_out);

/* Reservoir samplers (section 4).  DPRS (Algorithm 3) visits the neighbour
 * sequence S in order; ZPRS (Algorithm 4) visits it in the zig-zag order S'
 * of k lanes: the d entries form quads of four consecutive entries (entry i
 * is in quad i / 4), lane j owns quads j, j + k, j + 2k, ... and visits
 * their entries in order, and S' is lane 0's entries, then lane 1's, ...
 * Each visited entry i of weight w_i replaces the selection when
 * floor(u_i * W / 2^64) < w_i, with W the total of the entries visited so
 * far including i (the integer form of "random(0,1) < w_i / W"); the result
 * is the last selection.  Either way neighbour i is picked with chance
 * w_i / T (Propositions 1 and 2), but which neighbour is picked differs. */
#define FWO_SAMPLER_ITS 0
#define FWO_SAMPLER_DPRS 1
#define FWO_SAMPLER_ZPRS 2
#define FWO_ZPRS_LANES 64

/* The uniform word of entry i at hop t: word (i mod 4) of
 * Philox4x64-10(counter = (qid, t, floor(i / 4), 1), key = (seed, 0)). */
uint64_t fwo_entry_draw(uint64_t seed, uint64_t qid, uint64_t t, uint64_t i);

/* ZPRS's visiting order of d entries with k lanes into order[0 .. d). */
void fwo_zigzag_order(uint64_t d, uint32_t k, uint64_t* order);

/* Sequential weighted reservoir sampling (Algorithm 2) over the entries
 * order[0 .. d) with weights w[] and words u[] (indexed by entry); returns
 * the last selected entry, or -1 when every weight is 0. */
int64_t fwo_reservoir(const uint64_t* w, const uint64_t* u, const uint64_t* order, uint64_t d);

/* Sampler microbenchmark tasks (section 6.3's comparison of sampling
 * methods): task j picks one index of the `size` weights w[0 .. size) with
 * chance w_i / T, T = sum(w), or returns -1 when T = 0.  Draws are keyed by
 * (seed, task j):
 *   ITS            word 0 of Philox(counter (j, 0, 0, 0)): r = floor(u T / 2^64),
 *                  first inclusive prefix above r (the buffered variant picks
 *                  the same index from a stored prefix array);
 *   DPRS / ZPRS    entry i's word = word i mod 4 of Philox(j, 0, i / 4, 1);
 *   ALIAS          Vose's alias table built by the sweep below, then column
 *                  c = floor(u0 size / 2^64) and, with words u0, u1 of
 *                  Philox(j, 0, 0, 2), c itself when floor(u1 T / 2^64) < prob[c],
 *                  else alias[c];
 *   REJECTION      trial k uses words u0, u1 of Philox(j, k, 0, 3): candidate
 *                  c = floor(u0 size / 2^64), accepted when
 *                  floor(u1 wmax / 2^64) < w_c; after FWO_RJS_MAX_TRIALS
 *                  rejections the task returns -1. */
#define FWO_TASK_ITS 0
#define FWO_TASK_DPRS 1
#define FWO_TASK_ZPRS 2
#define FWO_TASK_ITS_BUFFERED 3
#define FWO_TASK_ALIAS 4
#define FWO_TASK_REJECTION 5
#define FWO_RJS_MAX_TRIALS (1u << 24)

/* Alias table of w[0 .. n) with column capacity T = sum(w) in units of
 * w_i * n (so every probability is an exact integer): a sweep over the light
 * items (w_i n < T) and the heavy items (w_i n >= T), both in index order.
 * The current heavy item fills the light items one after the other; once its
 * remaining mass is at most T it becomes a column of its own, filled from the
 * next heavy item.  prob[c] = the part of column c kept by c (<= T), alias[c]
 * = the item that owns the rest.  Returns T (0: the table is not built). */
uint64_t fwo_alias_table(const uint32_t* w, uint32_t n, uint64_t* prob, uint32_t* alias);

/* One task of the given sampler over w[0 .. size); -1 when nothing is picked. */
int64_t fwo_sample_task(int sampler, const uint32_t* w, uint32_t size, uint64_t seed,
                        uint64_t task);

/* Walks n queries.  Query i has id qid_base + i and starts at starts[i];
 * row i of out_paths (length + 1 entries) receives its path. */
int fwo_walk(const fwo_graph* g, int algo, const fwo_params* p, const uint32_t* starts,
             uint64_t n, uint32_t length, uint64_t seed, uint64_t qid_base,
             uint32_t* out_paths);

/* fwo_walk with the pick of each hop made by `sampler` (FWO_SAMPLER_*). */
int fwo_walk_sampler(const fwo_graph* g, int algo, const fwo_params* p, int sampler,
                     const uint32_t* starts, uint64_t n, uint32_t length, uint64_t seed,
                     uint64_t qid_base, uint32_t* out_paths);

/* Walks the m queries qids[j] (start starts[qids[j]]), row j of out_paths. */
int fwo_walk_ids(const fwo_graph* g, int algo, const fwo_params* p, const uint32_t* starts,
                 const uint64_t* qids, uint64_t m, uint32_t length, uint64_t seed,
                 uint32_t* out_paths);

#ifdef __cplusplus
}
#endif
#endif
