/* CPU oracle for dynamic-graph random walks.  TEST INFRASTRUCTURE ONLY: see
 * fw_oracle.h.  Plain C, single-threaded, written for checking by eye. */
#include "fw_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon et al., SC 2011, section 4): each round multiplies */
/* words 0 and 2 by the two round constants, swaps and xors the high halves */
/* with words 1, 3 and the round key; the key is bumped by the Weyl          */
/* constants (golden ratio, sqrt(3) - 1) between rounds.                     */
/* ---------------------------------------------------------------------- */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void fwo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul128(PHILOX_M0, x0, &hi0, &lo0);
    mul128(PHILOX_M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

uint64_t fwo_draw(uint64_t seed, uint64_t qid, uint64_t t) {
  uint64_t ctr[4] = {qid, t, 0, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  fwo_philox4x64_10(ctr, key, out);
  return out[0];
}

int fwo_stop_coin(uint64_t u1, uint32_t stop_num, uint32_t stop_den) {
  unsigned __int128 p = (unsigned __int128)u1 * stop_den;
  return (uint64_t)(p >> 64) < stop_num;
}

int fwo_stop(uint64_t seed, uint64_t qid, uint64_t t, uint32_t stop_num, uint32_t stop_den) {
  uint64_t ctr[4] = {qid, t, 0, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  fwo_philox4x64_10(ctr, key, out);
  return fwo_stop_coin(out[1], stop_num, stop_den);
}

uint64_t fwo_entry_draw(uint64_t seed, uint64_t qid, uint64_t t, uint64_t i) {
  uint64_t ctr[4] = {qid, t, i / 4, 1};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  fwo_philox4x64_10(ctr, key, out);
  return out[i % 4];
}

void fwo_zigzag_order(uint64_t d, uint32_t k, uint64_t* order) {
  uint64_t quads = (d + 3) / 4, m = 0;
  for (uint32_t j = 0; j < k; ++j)
    for (uint64_t q = j; q < quads; q += k)
      for (uint64_t i = 4 * q; i < 4 * q + 4 && i < d; ++i) order[m++] = i;
}

int64_t fwo_reservoir(const uint64_t* w, const uint64_t* u, const uint64_t* order, uint64_t d) {
  int64_t selected = -1;
  uint64_t total = 0;
  for (uint64_t m = 0; m < d; ++m) {
    uint64_t i = order[m];
    if (w[i] == 0) continue;
    total += w[i];
    unsigned __int128 p = (unsigned __int128)u[i] * total;
    if ((uint64_t)(p >> 64) < w[i]) selected = (int64_t)i;
  }
  return selected;
}

uint64_t fwo_scale(uint64_t u, uint64_t total) {
  unsigned __int128 p = (unsigned __int128)u * total;
  return (uint64_t)(p >> 64);
}

/* Inverse transform sampling (section 2.2): the first index whose inclusive
 * prefix sum exceeds r. */
int64_t fwo_pick(const uint64_t* w, uint64_t d, uint64_t r) {
  uint64_t prefix = 0;
  for (uint64_t i = 0; i < d; ++i) {
    prefix += w[i];
    if (prefix > r) return (int64_t)i;
  }
  return -1;
}

static uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

/* Eq. 2 with a = p (return) and b = q (in-out): the relative chances are
 * 1/p, 1, 1/q = p_den/p_num, 1, q_den/q_num.  Scale by p_num * q_num and
 * divide out the common factor. */
int fwo_node2vec_factors(uint32_t p_num, uint32_t p_den, uint32_t q_num, uint32_t q_den,
                         fwo_params* out) {
  if (!out || !p_num || !p_den || !q_num || !q_den) return FWO_EINVAL;
  uint64_t ret = (uint64_t)p_den * q_num;
  uint64_t in = (uint64_t)p_num * q_num;
  uint64_t outf = (uint64_t)p_num * q_den;
  uint64_t g = gcd64(gcd64(ret, in), outf);
  ret /= g;
  in /= g;
  outf /= g;
  if (ret > 0xFFFFFFFFull || in > 0xFFFFFFFFull || outf > 0xFFFFFFFFull) return FWO_EINVAL;
  out->f_ret = (uint32_t)ret;
  out->f_in = (uint32_t)in;
  out->f_out = (uint32_t)outf;
  return FWO_OK;
}

int fwo_validate(const fwo_graph* g) {
  if (!g || !g->offsets || (g->n_edges && !g->adj)) return FWO_EINVAL;
  if (g->n_vertices >= 0xFFFFFFFFull) return FWO_EINVAL;
  if (g->offsets[0] != 0 || g->offsets[g->n_vertices] != g->n_edges) return FWO_EINVAL;
  for (uint64_t v = 0; v < g->n_vertices; ++v) {
    uint64_t b = g->offsets[v], e = g->offsets[v + 1];
    if (e < b || e > g->n_edges) return FWO_EINVAL;
    for (uint64_t i = b; i < e; ++i) {
      if (g->adj[i] >= g->n_vertices) return FWO_EINVAL;
      if (i > b && g->adj[i] < g->adj[i - 1]) return FWO_EINVAL;
    }
  }
  return FWO_OK;
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* Is u a neighbour of v?  Rows are sorted, so libc bsearch answers it. */
static int is_neighbour(const fwo_graph* g, uint32_t v, uint32_t u) {
  uint64_t b = g->offsets[v], e = g->offsets[v + 1];
  if (e == b) return 0;
  return bsearch(&u, g->adj + b, (size_t)(e - b), sizeof(uint32_t), cmp_u32) != NULL;
}

static int check_params(const fwo_graph* g, int algo, const fwo_params* p) {
  if (algo == FWO_DEEPWALK) return FWO_OK;
  if (!p) return FWO_EINVAL;
  if (algo == FWO_PPR) {
    if (p->stop_den == 0 || p->stop_num > p->stop_den) return FWO_EINVAL;
    return FWO_OK;
  }
  if (algo == FWO_NODE2VEC) {
    if (p->f_ret == 0 && p->f_in == 0 && p->f_out == 0) return FWO_EINVAL;
    return FWO_OK;
  }
  if (algo == FWO_METAPATH) {
    if (!g->labels || p->schema_len < 1 || p->schema_len > 16) return FWO_EINVAL;
    return FWO_OK;
  }
  return FWO_EINVAL;
}

/* Section 2.1: weighted DeepWalk f(e(v,u)) = w(v,u); node2vec multiplies the
 * weight by Eq. 2, where dist(v',u) = 0 means u is v', dist 1 means u is a
 * neighbour of v', and every other neighbour of v is at distance 2; MetaPath
 * multiplies the weight by Eq. 1, the indicator that the edge label equals
 * the schema label of this hop.  At the first hop node2vec has no v' and uses
 * the weight alone.  PPR's transition weights are DeepWalk's. */
int fwo_transition_weights(const fwo_graph* g, int algo, const fwo_params* p, uint32_t prev,
                           uint32_t cur, uint32_t t, uint64_t* w_out) {
  if (!g || cur >= g->n_vertices) return FWO_EINVAL;
  int rc = check_params(g, algo, p);
  if (rc) return rc;
  if (algo == FWO_NODE2VEC && t > 0 && prev >= g->n_vertices) return FWO_EINVAL;
  uint64_t b = g->offsets[cur], d = g->offsets[cur + 1] - b;
  for (uint64_t i = 0; i < d; ++i) {
    uint64_t w = g->weights ? g->weights[b + i] : 1;
    uint32_t u = g->adj[b + i];
    uint64_t f = 1;
    if (algo == FWO_NODE2VEC && t > 0) {
      if (u == prev)
        f = p->f_ret;
      else if (is_neighbour(g, prev, u))
        f = p->f_in;
      else
        f = p->f_out;
    } else if (algo == FWO_METAPATH) {
      f = (g->labels[b + i] == p->schema[t % p->schema_len]) ? 1 : 0;
    }
    w_out[i] = w * f;
  }
  return FWO_OK;
}

/* The total of one step must fit in 64 bits: max_w * max_f * max_deg < 2^64. */
static int check_overflow(const fwo_graph* g, int algo, const fwo_params* p) {
  uint64_t max_w = 1, max_deg = 0, max_f = 1;
  if (g->weights) {
    max_w = 0;
    for (uint64_t e = 0; e < g->n_edges; ++e)
      if (g->weights[e] > max_w) max_w = g->weights[e];
  }
  for (uint64_t v = 0; v < g->n_vertices; ++v) {
    uint64_t d = g->offsets[v + 1] - g->offsets[v];
    if (d > max_deg) max_deg = d;
  }
  if (algo == FWO_NODE2VEC) {
    max_f = p->f_ret;
    if (p->f_in > max_f) max_f = p->f_in;
    if (p->f_out > max_f) max_f = p->f_out;
    if (max_f == 0) max_f = 1;
  }
  unsigned __int128 bound = (unsigned __int128)max_w * max_f * max_deg;
  return (bound >> 64) ? FWO_EOVERFLOW : FWO_OK;
}

static uint64_t max_degree(const fwo_graph* g) {
  uint64_t m = 0;
  for (uint64_t v = 0; v < g->n_vertices; ++v) {
    uint64_t d = g->offsets[v + 1] - g->offsets[v];
    if (d > m) m = d;
  }
  return m;
}

uint64_t fwo_alias_table(const uint32_t* w, uint32_t n, uint64_t* prob, uint32_t* alias) {
  uint64_t T = 0;
  for (uint32_t i = 0; i < n; ++i) T += w[i];
  if (T == 0) return 0;
  for (uint32_t c = 0; c < n; ++c) {
    prob[c] = T;
    alias[c] = c;
  }
  /* q_i = w_i * n: light when q_i < T, heavy otherwise. */
  uint32_t i = 0, j = 0;
  while (i < n && (uint64_t)w[i] * n >= T) ++i;
  while (j < n && (uint64_t)w[j] * n < T) ++j;
  if (j >= n) return T; /* cannot happen: some item is at least the mean */
  uint64_t rem = (uint64_t)w[j] * n; /* mass left in heavy j */
  while (j < n) {
    if (rem > T) {
      if (i >= n) break;
      uint64_t q = (uint64_t)w[i] * n;
      prob[i] = q;
      alias[i] = j;
      rem -= T - q;
      do ++i; while (i < n && (uint64_t)w[i] * n >= T);
    } else {
      uint32_t nj = j + 1;
      while (nj < n && (uint64_t)w[nj] * n < T) ++nj;
      prob[j] = rem;
      alias[j] = nj < n ? nj : j;
      if (nj < n) rem = (uint64_t)w[nj] * n - (T - rem);
      j = nj;
    }
  }
  return T;
}

static uint64_t mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

int64_t fwo_sample_task(int sampler, const uint32_t* w, uint32_t size, uint64_t seed,
                        uint64_t task) {
  uint64_t T = 0, wmax = 0;
  for (uint32_t i = 0; i < size; ++i) {
    T += w[i];
    if (w[i] > wmax) wmax = w[i];
  }
  if (T == 0) return -1;
  uint64_t key[2] = {seed, 0}, out[4];
  if (sampler == FWO_TASK_ITS || sampler == FWO_TASK_ITS_BUFFERED) {
    uint64_t ctr[4] = {task, 0, 0, 0};
    fwo_philox4x64_10(ctr, key, out);
    uint64_t r = mulhi64(out[0], T), prefix = 0;
    for (uint32_t i = 0; i < size; ++i) {
      prefix += w[i];
      if (prefix > r) return i;
    }
    return -1;
  }
  if (sampler == FWO_TASK_DPRS || sampler == FWO_TASK_ZPRS) {
    uint64_t *wb = malloc(size * sizeof(uint64_t)), *ub = malloc(size * sizeof(uint64_t)),
             *ob = malloc(size * sizeof(uint64_t));
    int64_t pick = -1;
    if (wb && ub && ob) {
      for (uint32_t i = 0; i < size; ++i) {
        wb[i] = w[i];
        ub[i] = fwo_entry_draw(seed, task, 0, i);
        ob[i] = i;
      }
      if (sampler == FWO_TASK_ZPRS) fwo_zigzag_order(size, FWO_ZPRS_LANES, ob);
      pick = fwo_reservoir(wb, ub, ob, size);
    }
    free(wb);
    free(ub);
    free(ob);
    return pick;
  }
  if (sampler == FWO_TASK_ALIAS) {
    uint64_t* prob = malloc(size * sizeof(uint64_t));
    uint32_t* alias = malloc(size * sizeof(uint32_t));
    int64_t pick = -1;
    if (prob && alias) {
      fwo_alias_table(w, size, prob, alias);
      uint64_t ctr[4] = {task, 0, 0, 2};
      fwo_philox4x64_10(ctr, key, out);
      uint64_t c = mulhi64(out[0], size);
      pick = mulhi64(out[1], T) < prob[c] ? (int64_t)c : (int64_t)alias[c];
    }
    free(prob);
    free(alias);
    return pick;
  }
  if (sampler == FWO_TASK_REJECTION) {
    for (uint64_t k = 0; k < FWO_RJS_MAX_TRIALS; ++k) {
      uint64_t ctr[4] = {task, k, 0, 3};
      fwo_philox4x64_10(ctr, key, out);
      uint64_t c = mulhi64(out[0], size);
      if (mulhi64(out[1], wmax) < w[c]) return (int64_t)c;
    }
    return -1;
  }
  return -1;
}

/* Scratch of one walker: weights, entry words and a visiting order, each
 * max_degree long. */
typedef struct {
  uint64_t *w, *u, *order;
} scratch;

/* The pick of one hop among d entries of weights w (total > 0). */
static int64_t pick_entry(int sampler, const scratch* b, uint64_t d, uint64_t total,
                          uint64_t seed, uint64_t qid, uint32_t t) {
  if (sampler == FWO_SAMPLER_ITS) return fwo_pick(b->w, d, fwo_scale(fwo_draw(seed, qid, t), total));
  for (uint64_t i = 0; i < d; ++i) b->u[i] = fwo_entry_draw(seed, qid, t, i);
  if (sampler == FWO_SAMPLER_DPRS)
    for (uint64_t i = 0; i < d; ++i) b->order[i] = i;
  else
    fwo_zigzag_order(d, FWO_ZPRS_LANES, b->order);
  return fwo_reservoir(b->w, b->u, b->order, d);
}

/* One query: Algorithm 1's loop with inverse transform sampling (or a
 * reservoir sampler).  A PPR query first tosses its stop coin at every hop;
 * `length` caps its hops. */
static int walk_one(const fwo_graph* g, int algo, const fwo_params* p, int sampler,
                    uint32_t start, uint64_t qid, uint32_t length, uint64_t seed,
                    const scratch* scr, uint32_t* row) {
  uint64_t* wbuf = scr->w;
  if (start >= g->n_vertices) return FWO_EINVAL;
  row[0] = start;
  for (uint32_t t = 0; t < length; ++t) {
    if (algo == FWO_PPR && fwo_stop(seed, qid, t, p->stop_num, p->stop_den)) {
      for (uint32_t s = t + 1; s <= length; ++s) row[s] = FWO_END;
      return FWO_OK;
    }
    uint32_t cur = row[t];
    uint32_t prev = t > 0 ? row[t - 1] : FWO_END;
    uint64_t b = g->offsets[cur], d = g->offsets[cur + 1] - b;
    int rc = fwo_transition_weights(g, algo, p, prev, cur, t, wbuf);
    if (rc) return rc;
    uint64_t total = 0;
    for (uint64_t i = 0; i < d; ++i) total += wbuf[i];
    if (total == 0) {
      for (uint32_t s = t + 1; s <= length; ++s) row[s] = FWO_END;
      return FWO_OK;
    }
    int64_t i = pick_entry(sampler, scr, d, total, seed, qid, t);
    row[t + 1] = g->adj[b + (uint64_t)i];
  }
  return FWO_OK;
}

static void scratch_free(scratch* b) {
  free(b->w);
  free(b->u);
  free(b->order);
}

static int walk_setup(const fwo_graph* g, int algo, const fwo_params* p, int sampler,
                      scratch* b) {
  b->w = b->u = b->order = NULL;
  if (!g || !g->offsets) return FWO_EINVAL;
  if (sampler < FWO_SAMPLER_ITS || sampler > FWO_SAMPLER_ZPRS) return FWO_EINVAL;
  int rc = check_params(g, algo, p);
  if (rc) return rc;
  rc = check_overflow(g, algo, p);
  if (rc) return rc;
  uint64_t md = max_degree(g);
  size_t bytes = (md ? md : 1) * sizeof(uint64_t);
  b->w = (uint64_t*)malloc(bytes);
  if (sampler != FWO_SAMPLER_ITS) {
    b->u = (uint64_t*)malloc(bytes);
    b->order = (uint64_t*)malloc(bytes);
  }
  if (!b->w || (sampler != FWO_SAMPLER_ITS && (!b->u || !b->order))) {
    scratch_free(b);
    return FWO_ENOMEM;
  }
  return FWO_OK;
}

int fwo_walk_sampler(const fwo_graph* g, int algo, const fwo_params* p, int sampler,
                     const uint32_t* starts, uint64_t n, uint32_t length, uint64_t seed,
                     uint64_t qid_base, uint32_t* out_paths) {
  if (n == 0) return FWO_OK;
  if (!starts || !out_paths) return FWO_EINVAL;
  scratch b;
  int rc = walk_setup(g, algo, p, sampler, &b);
  if (rc) return rc;
  for (uint64_t i = 0; i < n && rc == FWO_OK; ++i)
    rc = walk_one(g, algo, p, sampler, starts[i], qid_base + i, length, seed, &b,
                  out_paths + i * ((uint64_t)length + 1));
  scratch_free(&b);
  return rc;
}

int fwo_walk(const fwo_graph* g, int algo, const fwo_params* p, const uint32_t* starts,
             uint64_t n, uint32_t length, uint64_t seed, uint64_t qid_base,
             uint32_t* out_paths) {
  return fwo_walk_sampler(g, algo, p, FWO_SAMPLER_ITS, starts, n, length, seed, qid_base,
                          out_paths);
}

int fwo_walk_ids(const fwo_graph* g, int algo, const fwo_params* p, const uint32_t* starts,
                 const uint64_t* qids, uint64_t m, uint32_t length, uint64_t seed,
                 uint32_t* out_paths) {
  if (m == 0) return FWO_OK;
  if (!starts || !qids || !out_paths) return FWO_EINVAL;
  scratch b;
  int rc = walk_setup(g, algo, p, FWO_SAMPLER_ITS, &b);
  if (rc) return rc;
  for (uint64_t j = 0; j < m && rc == FWO_OK; ++j)
    rc = walk_one(g, algo, p, FWO_SAMPLER_ITS, starts[qids[j]], qids[j], length, seed, &b,
                  out_paths + j * ((uint64_t)length + 1));
  scratch_free(&b);
  return rc;
}
