// Seeded synthetic graph and query generators.
//
// Input generation only: this module holds none of the random-walk method's
// arithmetic (no transition weights, no draw, no pick).  Both the CPU oracle
// and the HIP library consume what it produces.  Every value is a pure
// function of (seed, index), computed with a SplitMix64-based hash, so the
// outputs do not depend on the thread count.
//
// Graph families:
//   * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): recursive quadrant
//     choice with probabilities (a, b, c, d), no per-level noise.
//   * Chung-Lu, edge-sampling form: each of M draws picks both endpoints
//     independently with probability proportional to (i + i0)^(-1/(gamma-1)),
//     sampled by the inverse of the continuous cumulative weight.
// Both are symmetrised, self-loops and duplicate edges are removed, rows are
// sorted ascending, and vertex ids are relabelled by a seeded bijection so
// that hub ids are spread over [0, V).
//
// Edge attributes are drawn per undirected edge {u, v} (so w(u,v) = w(v,u)):
// uniform integers, Zipf(s) clipped to a maximum (Devroye's rejection method,
// "Non-Uniform Random Variate Generation", 1986, ch. X.6), uniform labels.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

inline uint64_t mix64(uint64_t z) {
  // SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t h2(uint64_t seed, uint64_t a) { return mix64(mix64(seed) ^ a); }
inline uint64_t h3(uint64_t seed, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(seed) ^ a) ^ (b * 0xD6E8FEB86659FD93ull));
}
inline double unit(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }  // [0,1)

template <class F>
void parallel_for(uint64_t n, int nthreads, F&& f) {
  if (nthreads <= 1 || n < 4096) {
    f(0, (uint64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) {
    uint64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
    th.emplace_back([&f, t, lo, hi] { f(t, lo, hi); });
  }
  for (auto& x : th) x.join();
}

// Dynamic row scheduling (rows differ wildly in cost on power-law graphs).
template <class F>
void parallel_rows(uint64_t n, int nthreads, F&& f) {
  std::atomic<uint64_t> next{0};
  const uint64_t grain = 1024;
  auto body = [&] {
    for (;;) {
      uint64_t lo = next.fetch_add(grain);
      if (lo >= n) break;
      uint64_t hi = std::min(n, lo + grain);
      for (uint64_t r = lo; r < hi; ++r) f(r);
    }
  };
  if (nthreads <= 1) { body(); return; }
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) th.emplace_back(body);
  for (auto& x : th) x.join();
}

// Seeded bijection on [0, n): 4-round Feistel network on 2h bits
// (2^(2h) >= n), cycle-walked back into range.
struct Relabel {
  uint64_t n, half_mask, keys[4];
  int h;
  bool identity;
  Relabel(uint64_t n_, uint64_t seed, bool on) : n(n_), identity(!on) {
    int bits = 1;
    while ((1ull << bits) < n) ++bits;
    h = (bits + 1) / 2;
    half_mask = (1ull << h) - 1;
    for (int i = 0; i < 4; ++i) keys[i] = h2(seed ^ 0x5EED5EEDull, (uint64_t)i);
  }
  uint64_t once(uint64_t x) const {
    uint64_t l = x >> h, r = x & half_mask;
    for (int i = 0; i < 4; ++i) {
      uint64_t nl = r;
      r = l ^ (mix64(r ^ keys[i]) & half_mask);
      l = nl;
    }
    return (l << h) | r;
  }
  uint64_t operator()(uint64_t x) const {
    if (identity) return x;
    do { x = once(x); } while (x >= n);
    return x;
  }
};

struct EdgeSource {
  virtual ~EdgeSource() = default;
  virtual uint64_t count() const = 0;
  // Returns false if the draw is a self-loop (dropped).
  virtual bool edge(uint64_t i, uint64_t* u, uint64_t* v) const = 0;
};

struct RmatSource : EdgeSource {
  int scale;
  uint64_t m, seed;
  double a, ab, abc;
  Relabel rl;
  RmatSource(int s, uint64_t m_, double a_, double b_, double c_, uint64_t seed_, bool permute)
      : scale(s), m(m_), seed(seed_), a(a_), ab(a_ + b_), abc(a_ + b_ + c_),
        rl(1ull << s, seed_, permute) {}
  uint64_t count() const override { return m; }
  bool edge(uint64_t i, uint64_t* u, uint64_t* v) const override {
    uint64_t r = 0, c = 0;
    for (int l = 0; l < scale; ++l) {
      double x = unit(h3(seed, i, (uint64_t)l));
      r <<= 1;
      c <<= 1;
      if (x < a) {
      } else if (x < ab) {
        c |= 1;
      } else if (x < abc) {
        r |= 1;
      } else {
        r |= 1;
        c |= 1;
      }
    }
    if (r == c) return false;
    *u = rl(r);
    *v = rl(c);
    return true;
  }
};

struct ChungLuSource : EdgeSource {
  uint64_t n, m, seed;
  double i0, alpha, base, span;
  Relabel rl;
  ChungLuSource(uint64_t n_, uint64_t m_, double gamma, double i0_, uint64_t seed_, bool permute)
      : n(n_), m(m_), seed(seed_), i0(i0_), rl(n_, seed_, permute) {
    alpha = 1.0 / (gamma - 1.0);
    if (std::fabs(alpha - 1.0) < 1e-12) {
      base = 0.0;
      span = std::log((n + i0) / i0);
    } else {
      base = std::pow(i0, 1.0 - alpha);
      span = std::pow((double)n + i0, 1.0 - alpha) - base;
    }
  }
  uint64_t pick(double x) const {
    double y;
    if (std::fabs(alpha - 1.0) < 1e-12)
      y = i0 * std::exp(x * span) - i0;
    else
      y = std::pow(x * span + base, 1.0 / (1.0 - alpha)) - i0;
    if (!(y >= 0.0)) y = 0.0;
    uint64_t k = (uint64_t)y;
    return k >= n ? n - 1 : k;
  }
  uint64_t count() const override { return m; }
  bool edge(uint64_t i, uint64_t* u, uint64_t* v) const override {
    uint64_t a = pick(unit(h3(seed, i, 0))), b = pick(unit(h3(seed, i, 1)));
    if (a == b) return false;
    *u = rl(a);
    *v = rl(b);
    return true;
  }
};

// Large graphs take minutes: their builds report each finished phase on stderr.
void progress(uint64_t m, const char* phase) {
  if (m >= (1ull << 28)) {
    std::fprintf(stderr, "[synth] %llu draws: %s\n", (unsigned long long)m, phase);
    std::fflush(stderr);
  }
}

int build_csr(const EdgeSource& src, uint64_t nv, int nthreads, uint64_t** offsets_out,
              uint32_t** adj_out, uint64_t* ne_out) {
  if (nthreads < 1) nthreads = 1;
  const uint64_t m = src.count();
  // Pass 1: degree counts (both directions).
  uint32_t* deg = (uint32_t*)std::calloc(nv + 1, sizeof(uint32_t));
  uint64_t* off = (uint64_t*)std::malloc((nv + 1) * sizeof(uint64_t));
  if (!deg || !off) { std::free(deg); std::free(off); return -1; }
  parallel_for(m, nthreads, [&](int, uint64_t lo, uint64_t hi) {
    uint64_t u, v;
    for (uint64_t i = lo; i < hi; ++i)
      if (src.edge(i, &u, &v)) {
        __atomic_fetch_add(&deg[u], 1u, __ATOMIC_RELAXED);
        __atomic_fetch_add(&deg[v], 1u, __ATOMIC_RELAXED);
      }
  });
  progress(m, "degrees counted");
  off[0] = 0;
  for (uint64_t i = 0; i < nv; ++i) off[i + 1] = off[i] + deg[i];
  const uint64_t raw = off[nv];
  uint32_t* tmp = (uint32_t*)std::malloc((raw ? raw : 1) * sizeof(uint32_t));
  uint64_t* cur = (uint64_t*)std::malloc((nv + 1) * sizeof(uint64_t));
  if (!tmp || !cur) { std::free(deg); std::free(off); std::free(tmp); std::free(cur); return -1; }
  std::memcpy(cur, off, (nv + 1) * sizeof(uint64_t));
  // Pass 2: regenerate and scatter.
  parallel_for(m, nthreads, [&](int, uint64_t lo, uint64_t hi) {
    uint64_t u, v;
    for (uint64_t i = lo; i < hi; ++i)
      if (src.edge(i, &u, &v)) {
        tmp[__atomic_fetch_add(&cur[u], 1ull, __ATOMIC_RELAXED)] = (uint32_t)v;
        tmp[__atomic_fetch_add(&cur[v], 1ull, __ATOMIC_RELAXED)] = (uint32_t)u;
      }
  });
  std::free(cur);
  progress(m, "edges scattered");
  // Sort and deduplicate each row.
  parallel_rows(nv, nthreads, [&](uint64_t r) {
    uint32_t* b = tmp + off[r];
    uint32_t* e = tmp + off[r + 1];
    std::sort(b, e);
    deg[r] = (uint32_t)(std::unique(b, e) - b);
  });
  progress(m, "rows sorted and deduplicated");
  uint64_t* noff = (uint64_t*)std::malloc((nv + 1) * sizeof(uint64_t));
  if (!noff) { std::free(deg); std::free(off); std::free(tmp); return -1; }
  noff[0] = 0;
  for (uint64_t i = 0; i < nv; ++i) noff[i + 1] = noff[i] + deg[i];
  const uint64_t ne = noff[nv];
  uint32_t* adj = (uint32_t*)std::malloc((ne ? ne : 1) * sizeof(uint32_t));
  if (!adj) { std::free(deg); std::free(off); std::free(tmp); std::free(noff); return -1; }
  parallel_rows(nv, nthreads, [&](uint64_t r) {
    std::memcpy(adj + noff[r], tmp + off[r], (size_t)deg[r] * sizeof(uint32_t));
  });
  std::free(tmp);
  std::free(off);
  std::free(deg);
  *offsets_out = noff;
  *adj_out = adj;
  *ne_out = ne;
  return 0;
}

inline uint64_t pair_key(uint64_t u, uint64_t v) {
  return u < v ? (u << 32) | v : (v << 32) | u;
}

template <class F>
void per_edge(const uint64_t* off, const uint32_t* adj, uint64_t nv, int nthreads, F&& f) {
  parallel_rows(nv, nthreads, [&](uint64_t r) {
    for (uint64_t e = off[r]; e < off[r + 1]; ++e) f(e, pair_key(r, adj[e]));
  });
}

// Devroye's rejection sampler for Zipf(s), s > 1, support k >= 1.
uint64_t zipf_draw(double s, uint64_t seed, uint64_t key, uint64_t cap) {
  const double am1 = s - 1.0, b = std::pow(2.0, am1);
  for (uint64_t attempt = 0;; ++attempt) {
    double u = 1.0 - unit(h3(seed, key, 2 * attempt));
    double v = unit(h3(seed, key, 2 * attempt + 1));
    double x = std::floor(std::pow(u, -1.0 / am1));
    if (!(x >= 1.0)) continue;
    if (x > 9.0e15) return cap;  // far beyond any cap used here
    double t = std::pow(1.0 + 1.0 / x, am1);
    if (v * x * (t - 1.0) / (b - 1.0) <= t / b) {
      uint64_t k = (uint64_t)x;
      return k > cap ? cap : k;
    }
  }
}

}  // namespace

extern "C" {

// Status: 0 ok, -1 out of memory, -2 bad argument.
int synth_rmat(int scale, uint64_t edge_factor, double a, double b, double c, uint64_t seed,
               int permute, int nthreads, uint64_t** offsets, uint32_t** adj,
               uint64_t* n_edges) {
  if (scale < 1 || scale > 31 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -2;
  RmatSource s(scale, edge_factor << scale, a, b, c, seed, permute != 0);
  return build_csr(s, 1ull << scale, nthreads, offsets, adj, n_edges);
}

int synth_chung_lu(uint64_t n, uint64_t draws, double gamma, double i0, uint64_t seed,
                   int permute, int nthreads, uint64_t** offsets, uint32_t** adj,
                   uint64_t* n_edges) {
  if (n < 2 || n >= 0xFFFFFFFFull || gamma <= 1.0 || i0 <= 0.0) return -2;
  ChungLuSource s(n, draws, gamma, i0, seed, permute != 0);
  return build_csr(s, n, nthreads, offsets, adj, n_edges);
}

void synth_free(void* p) { std::free(p); }

// Uniform integers in [lo, hi] per undirected edge.
int synth_weights_uniform(const uint64_t* off, const uint32_t* adj, uint64_t nv, uint32_t lo,
                          uint32_t hi, uint64_t seed, int nthreads, uint32_t* out) {
  if (hi < lo) return -2;
  const uint64_t span = (uint64_t)hi - lo + 1;
  per_edge(off, adj, nv, nthreads, [&](uint64_t e, uint64_t key) {
    out[e] = lo + (uint32_t)(((unsigned __int128)h2(seed, key) * span) >> 64);
  });
  return 0;
}

// Zipf(s) per undirected edge, clipped to [1, cap].
int synth_weights_zipf(const uint64_t* off, const uint32_t* adj, uint64_t nv, double s,
                       uint32_t cap, uint64_t seed, int nthreads, uint32_t* out) {
  if (!(s > 1.0) || cap < 1) return -2;
  per_edge(off, adj, nv, nthreads, [&](uint64_t e, uint64_t key) {
    out[e] = (uint32_t)zipf_draw(s, seed, key, cap);
  });
  return 0;
}

// Uniform labels in [0, k) per undirected edge.
int synth_labels_uniform(const uint64_t* off, const uint32_t* adj, uint64_t nv, uint32_t k,
                         uint64_t seed, int nthreads, uint8_t* out) {
  if (k < 1 || k > 256) return -2;
  per_edge(off, adj, nv, nthreads, [&](uint64_t e, uint64_t key) {
    out[e] = (uint8_t)(((unsigned __int128)h2(seed, key) * k) >> 64);
  });
  return 0;
}

// n vertex ids uniform in [0, nv), with replacement.
int synth_uniform_ids(uint64_t n, uint64_t nv, uint64_t seed, int nthreads, uint32_t* out) {
  if (nv == 0 || nv > 0xFFFFFFFFull) return -2;
  parallel_for(n, nthreads, [&](int, uint64_t lo, uint64_t hi) {
    for (uint64_t i = lo; i < hi; ++i)
      out[i] = (uint32_t)(((unsigned __int128)h2(seed, i) * nv) >> 64);
  });
  return 0;
}

}  // extern "C"
