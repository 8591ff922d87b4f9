// Seeded synthetic graphs for the ChebyPower workloads.
//
// This module only builds inputs: undirected Chung-Lu power-law graphs in
// symmetric CSR form (int64 row offsets, int32 column indices).  It contains
// none of the propagation arithmetic and is shared, unchanged, by the CPU
// reference checks and by the GPU library's tests and benchmark.
//
// Model (the recipe is the builder's; the paper's SNAP graphs are not
// available, so Chung-Lu graphs of the same size stand in for them):
//   * node weights w_i = (i + i0)^(-1/(gamma-1)), i = 0..n-1;
//   * i0 is chosen so that the expected degree of the heaviest node equals
//     sqrt(2m), the structural cutoff below which Chung-Lu edge
//     probabilities w_i w_j / W stay below one;
//   * M endpoint pairs are drawn i.i.d. with P(i) = w_i / W using Walker's
//     alias method; randomness comes from the counter-based SplitMix64
//     generator (Steele, Lea & Flood, OOPSLA 2014), so every draw is a pure
//     function of (seed, counter) and threads need no shared state;
//   * self-loops are dropped, each pair becomes two arcs, duplicate arcs are
//     removed, nodes left without edges are dropped;
//   * M is corrected (secant steps) until the undirected edge count is
//     within 0.5% of the target;
//   * nodes are relabelled by a seeded random permutation (SNAP ids are not
//     degree-sorted) or kept in weight order (heaviest first).
// Rows come out sorted by column index.

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// Output number `ctr` (0-based) of a SplitMix64 stream whose state starts at
// `seed`: state advances by the golden gamma, the output is the mixer of the
// advanced state.
inline uint64_t splitmix64_at(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1) * kGolden;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

int pick_threads(int requested) {
  unsigned hw = std::thread::hardware_concurrency();
  int t = requested > 0 ? requested : (int)(hw ? hw : 1);
  return std::max(1, std::min(t, 16));
}

// Static partition of [0, total) into `nt` contiguous ranges.
void parallel_ranges(int64_t total, int nt,
                     const std::function<void(int, int64_t, int64_t)>& fn) {
  std::vector<std::thread> pool;
  int64_t chunk = (total + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t b = std::min<int64_t>(total, (int64_t)t * chunk);
    int64_t e = std::min<int64_t>(total, b + chunk);
    pool.emplace_back([=, &fn] { fn(t, b, e); });
  }
  for (auto& th : pool) th.join();
}

// Dynamic chunks over [0, total): used where per-item cost is skewed (rows).
void parallel_dynamic(int64_t total, int nt, int64_t grain,
                      const std::function<void(int64_t, int64_t)>& fn) {
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) {
    pool.emplace_back([&] {
      for (;;) {
        int64_t b = next.fetch_add(grain);
        if (b >= total) break;
        fn(b, std::min(total, b + grain));
      }
    });
  }
  for (auto& th : pool) th.join();
}

struct Alias {
  std::vector<double> prob;
  std::vector<int32_t> alias;
};

// Vose's variant of Walker's alias method.
Alias build_alias(const std::vector<double>& w) {
  const int64_t n = (int64_t)w.size();
  double total = 0.0;
  for (double x : w) total += x;
  Alias a;
  a.prob.assign(n, 0.0);
  a.alias.assign(n, 0);
  std::vector<double> scaled(n);
  std::vector<int32_t> small, large;
  small.reserve(n);
  large.reserve(n);
  for (int64_t i = 0; i < n; ++i) {
    scaled[i] = w[i] * (double)n / total;
    (scaled[i] < 1.0 ? small : large).push_back((int32_t)i);
  }
  while (!small.empty() && !large.empty()) {
    int32_t s = small.back(); small.pop_back();
    int32_t l = large.back(); large.pop_back();
    a.prob[s] = scaled[s];
    a.alias[s] = l;
    scaled[l] = (scaled[l] + scaled[s]) - 1.0;
    (scaled[l] < 1.0 ? small : large).push_back(l);
  }
  for (int32_t l : large) { a.prob[l] = 1.0; a.alias[l] = l; }
  for (int32_t s : small) { a.prob[s] = 1.0; a.alias[s] = s; }
  return a;
}

inline int32_t draw(const Alias& a, uint64_t n, uint64_t x_idx, uint64_t x_coin) {
  uint64_t i = mulhi64(x_idx, n);
  double u = (double)(x_coin >> 11) * 0x1.0p-53;
  return u < a.prob[i] ? (int32_t)i : a.alias[i];
}

// Endpoint pair number j of the stream: four SplitMix64 outputs.
inline bool pair_at(const Alias& al, uint64_t n, uint64_t seed, uint64_t j,
                    int32_t* a, int32_t* b) {
  *a = draw(al, n, splitmix64_at(seed, 4 * j + 0), splitmix64_at(seed, 4 * j + 1));
  *b = draw(al, n, splitmix64_at(seed, 4 * j + 2), splitmix64_at(seed, 4 * j + 3));
  return *a != *b;
}

// Sum_{i=0}^{n-1} (i+i0)^-a, exact for the first terms, midpoint integral
// for the smooth remainder (only used to pick i0, not for sampling).
double weight_sum_approx(int64_t n, double i0, double a) {
  const int64_t head = std::min<int64_t>(n, 2048);
  double s = 0.0;
  for (int64_t i = 0; i < head; ++i) s += std::pow((double)i + i0, -a);
  if (n > head) {
    double lo = (double)head - 0.5 + i0, hi = (double)n - 0.5 + i0;
    if (std::fabs(a - 1.0) < 1e-12) s += std::log(hi / lo);
    else s += (std::pow(hi, 1.0 - a) - std::pow(lo, 1.0 - a)) / (1.0 - a);
  }
  return s;
}

double solve_i0(int64_t n, double a, double m_target) {
  // Want E[deg(0)] = 2M w_0 / W = sqrt(2M)  <=>  w_0 / W = 1/sqrt(2M).
  const double target = 1.0 / std::sqrt(2.0 * m_target);
  if (target <= 1.0 / (double)n) return 1e12;  // degree cap unreachable: flat weights
  double lo = std::log(1e-9), hi = std::log(1e12);
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    double i0 = std::exp(mid);
    double r = std::pow(i0, -a) / weight_sum_approx(n, i0, a);
    if (r > target) lo = mid; else hi = mid;  // ratio falls as i0 grows
  }
  return std::exp(0.5 * (lo + hi));
}

struct RawCSR {
  std::vector<int64_t> off;  // n+1
  int32_t* adj = nullptr;    // off[n] entries (malloc'd)
  ~RawCSR() { std::free(adj); }
};

// Draw M pairs, symmetrize, dedup.  Returns false on allocation failure.
bool build_simple_graph(const Alias& al, int64_t n, uint64_t seed, int64_t M,
                        int nt, RawCSR* out, bool verbose) {
  auto stage = [&](const char* what) {
    if (verbose) { fprintf(stderr, "[synth]   %s\n", what); fflush(stderr); }
  };
  std::vector<std::atomic<uint32_t>> deg(n);
  for (auto& d : deg) d.store(0, std::memory_order_relaxed);
  parallel_ranges(M, nt, [&](int, int64_t b, int64_t e) {
    int32_t x, y;
    for (int64_t j = b; j < e; ++j)
      if (pair_at(al, (uint64_t)n, seed, (uint64_t)j, &x, &y)) {
        deg[x].fetch_add(1, std::memory_order_relaxed);
        deg[y].fetch_add(1, std::memory_order_relaxed);
      }
  });
  stage("degrees counted");
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i].load(std::memory_order_relaxed);
  const int64_t total = off[n];
  int32_t* adj = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
  if (!adj) return false;
  std::vector<std::atomic<int64_t>> cur(n);
  for (int64_t i = 0; i < n; ++i) cur[i].store(off[i], std::memory_order_relaxed);
  parallel_ranges(M, nt, [&](int, int64_t b, int64_t e) {
    int32_t x, y;
    for (int64_t j = b; j < e; ++j)
      if (pair_at(al, (uint64_t)n, seed, (uint64_t)j, &x, &y)) {
        adj[cur[x].fetch_add(1, std::memory_order_relaxed)] = y;
        adj[cur[y].fetch_add(1, std::memory_order_relaxed)] = x;
      }
  });
  stage("arcs scattered");
  // Sort and dedup each row (slot order from the scatter is nondeterministic,
  // the sorted unique row is not).
  std::vector<int64_t> ulen(n, 0);
  parallel_dynamic(n, nt, 4096, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t* r = adj + off[i];
      int64_t len = off[i + 1] - off[i];
      std::sort(r, r + len);
      ulen[i] = std::unique(r, r + len) - r;
    }
  });
  stage("rows sorted and deduplicated");
  // Compact in row order (left moves only, so sequential memmove is safe).
  out->off.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    out->off[i + 1] = out->off[i] + ulen[i];
    if (ulen[i] && out->off[i] != off[i])
      std::memmove(adj + out->off[i], adj + off[i], sizeof(int32_t) * (size_t)ulen[i]);
  }
  std::free(out->adj);
  out->adj = adj;
  return true;
}

}  // namespace

extern "C" {

typedef struct {
  int64_t n_target;     // nodes before isolated ones are dropped
  int64_t m_target;     // undirected edges wanted
  double gamma;         // degree exponent (> 2 for a finite mean)
  uint64_t seed;
  int32_t relabel;      // 0: weight order (heaviest first), 1: seeded random permutation
  int32_t threads;      // 0: all hardware threads, capped at 16
  int32_t tune_passes;  // extra M-correction passes (0: single pass with M = m_target)
  int32_t verbose;      // 1: one progress line per stage on stderr
} synth_cl_params;

typedef struct {
  int64_t n;            // nodes kept (no isolated nodes)
  int64_t nnz;          // arcs = 2 * undirected edges
  int64_t d_max;
  int64_t n_dropped;    // isolated nodes removed
  int64_t pairs_drawn;  // M of the final pass
  double i0;
} synth_cl_info;

typedef struct {
  int64_t* row_ptr;
  int32_t* col_idx;
  synth_cl_info info;
} synth_graph;

// Returns 0 on success, -1 on bad parameters, -2 on allocation failure.
int synth_chunglu(const synth_cl_params* p, synth_graph** out) {
  if (!p || !out || p->n_target < 2 || p->m_target < 1 || !(p->gamma > 1.0) ||
      p->n_target > INT32_MAX)
    return -1;
  try {
    const int nt = pick_threads(p->threads);
    const int64_t n = p->n_target;
    const double a = 1.0 / (p->gamma - 1.0);
    const double i0 = solve_i0(n, a, (double)p->m_target);
    std::vector<double> w(n);
    for (int64_t i = 0; i < n; ++i) w[i] = std::pow((double)i + i0, -a);
    Alias al = build_alias(w);
    w.clear();
    w.shrink_to_fit();

    RawCSR g;
    int64_t M = p->m_target;
    int64_t prevM = 0, prevm = 0;
    for (int pass = 0;; ++pass) {
      if (p->verbose) { fprintf(stderr, "[synth] pass %d: drawing %lld pairs\n", pass, (long long)M); fflush(stderr); }
      if (!build_simple_graph(al, n, p->seed, M, nt, &g, p->verbose != 0)) return -2;
      int64_t m = g.off[n] / 2;
      double rel = (double)m / (double)p->m_target - 1.0;
      if (pass >= p->tune_passes || std::fabs(rel) < 0.005) break;
      int64_t nextM;
      if (prevM > 0 && m != prevm) {
        double slope = (double)(m - prevm) / (double)(M - prevM);
        nextM = M + (int64_t)std::llround((double)(p->m_target - m) / slope);
      } else {
        nextM = (int64_t)std::llround((double)M * (double)p->m_target / (double)m);
      }
      prevM = M;
      prevm = m;
      M = std::max<int64_t>(1, nextM);
    }

    if (p->verbose) { fprintf(stderr, "[synth] relabelling %lld nodes\n", (long long)n); fflush(stderr); }
    // Drop isolated nodes and relabel.
    std::vector<int32_t> kept;
    kept.reserve(n);
    for (int64_t i = 0; i < n; ++i)
      if (g.off[i + 1] > g.off[i]) kept.push_back((int32_t)i);
    const int64_t nk = (int64_t)kept.size();
    if (p->relabel == 1) {
      const uint64_t pseed = p->seed ^ 0x5DEECE66DA3C1F27ull;
      for (int64_t i = nk - 1; i > 0; --i) {
        int64_t j = (int64_t)mulhi64(splitmix64_at(pseed, (uint64_t)i), (uint64_t)(i + 1));
        std::swap(kept[i], kept[j]);
      }
    }
    // kept[new] = old; invert.
    std::vector<int32_t> new_id(n, -1);
    for (int64_t v = 0; v < nk; ++v) new_id[kept[v]] = (int32_t)v;

    synth_graph* res = (synth_graph*)std::calloc(1, sizeof(synth_graph));
    if (!res) return -2;
    res->row_ptr = (int64_t*)std::malloc(sizeof(int64_t) * (size_t)(nk + 1));
    res->col_idx = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(g.off[n], 1));
    if (!res->row_ptr || !res->col_idx) {
      std::free(res->row_ptr); std::free(res->col_idx); std::free(res);
      return -2;
    }
    int64_t* rp = res->row_ptr;
    rp[0] = 0;
    int64_t dmax = 0;
    for (int64_t v = 0; v < nk; ++v) {
      int64_t d = g.off[kept[v] + 1] - g.off[kept[v]];
      rp[v + 1] = rp[v] + d;
      dmax = std::max(dmax, d);
    }
    int32_t* ci = res->col_idx;
    parallel_dynamic(nk, nt, 4096, [&](int64_t b, int64_t e) {
      for (int64_t v = b; v < e; ++v) {
        const int32_t* src = g.adj + g.off[kept[v]];
        int32_t* dst = ci + rp[v];
        int64_t d = rp[v + 1] - rp[v];
        for (int64_t q = 0; q < d; ++q) dst[q] = new_id[src[q]];
        std::sort(dst, dst + d);
      }
    });
    res->info.n = nk;
    res->info.nnz = rp[nk];
    res->info.d_max = dmax;
    res->info.n_dropped = n - nk;
    res->info.pairs_drawn = M;
    res->info.i0 = i0;
    *out = res;
    return 0;
  } catch (const std::bad_alloc&) {
    return -2;
  }
}

void synth_graph_free(synth_graph* g) {
  if (!g) return;
  std::free(g->row_ptr);
  std::free(g->col_idx);
  std::free(g);
}

// SplitMix64 output `ctr` for `seed` (exposed so Python-side draws of
// sources and tolerances use the same documented generator).
uint64_t synth_splitmix64_at(uint64_t seed, uint64_t ctr) { return splitmix64_at(seed, ctr); }

}  // extern "C"
