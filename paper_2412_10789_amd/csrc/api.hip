// C ABI of the ChebyPower library: graph objects, workspaces and queries.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "common.h"

namespace cp {

thread_local int32_t g_last_hip_error = 0;
void set_hip_error(hipError_t e) { g_last_hip_error = (int32_t)e; }

#define CP_HIP(call)                     \
  do {                                   \
    hipError_t e_ = (call);              \
    if (e_ != hipSuccess) {              \
      set_hip_error(e_);                 \
      return CP_EHIP;                    \
    }                                    \
  } while (0)

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t storage_bytes(int32_t prec) { return prec == CP_F64 ? 8 : prec == CP_BF16 ? 2 : 4; }
size_t acc_bytes(int32_t prec) { return prec == CP_F64 || prec == CP_F32 ? 8 : 4; }
bool valid_prec(int32_t prec) { return prec == CP_F64 || prec == CP_F32 || prec == CP_F32F || prec == CP_BF16; }

int host_threads() {
  unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h ? h : 1u, 16u));
}

// Wall-clock phases of cp_graph_create, printed to stderr when the
// environment variable CHEBYPROP_TRACE is set (diagnostics only).
struct PhaseClock {
  bool on = std::getenv("CHEBYPROP_TRACE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[chebyprop] graph create: %s %.1f ms\n", what,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

template <typename F>
void parallel_rows(int64_t n, F&& fn) {
  const int nt = host_threads();
  std::vector<std::thread> pool;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t b = std::min<int64_t>(n, t * chunk), e = std::min<int64_t>(n, b + chunk);
    pool.emplace_back([=, &fn] { fn(b, e); });
  }
  for (auto& th : pool) th.join();
}

// Rows [0, n) of a CSR in chunks of about equal work (arcs plus rows),
// taken by the threads in turn: degree-ordered graphs hold most arcs in
// their first rows, so equal row counts would leave one thread the hubs.
template <typename F>
void parallel_rows_balanced(const int64_t* rp, int64_t n, F&& fn) {
  const int nt = host_threads();
  const int64_t nchunks = std::min<int64_t>(n, (int64_t)nt * 8);
  if (nchunks <= 1 || nt == 1) {
    fn((int64_t)0, n);
    return;
  }
  const int64_t total = rp[n] + n;
  std::vector<int64_t> cut((size_t)nchunks + 1, n);
  cut[0] = 0;
  for (int64_t c = 1; c < nchunks; ++c) {
    const int64_t target = total / nchunks * c;
    int64_t lo = cut[(size_t)c - 1], hi = n;  // smallest v with rp[v] + v >= target
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (rp[mid] + mid >= target) hi = mid;
      else lo = mid + 1;
    }
    cut[(size_t)c] = lo;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&] {
      for (int64_t c = next++; c < nchunks; c = next++)
        if (cut[(size_t)c] < cut[(size_t)c + 1]) fn(cut[(size_t)c], cut[(size_t)c + 1]);
    });
  for (auto& th : pool) th.join();
}

// O(nnz) structural checks on host CSR (see CP_GRAPH_VALIDATE).
bool validate_csr(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci) {
  if (rp[0] != 0 || rp[n] != nnz) return false;
  for (int64_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) return false;
  std::vector<int32_t> sorted(ci, ci + nnz);
  std::atomic<bool> ok{true};
  parallel_rows(n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e && ok.load(std::memory_order_relaxed); ++v) {
      int32_t* r = sorted.data() + rp[v];
      const int64_t d = rp[v + 1] - rp[v];
      for (int64_t q = 0; q < d; ++q)
        if (r[q] < 0 || r[q] >= n || r[q] == v) { ok = false; return; }
      std::sort(r, r + d);
      for (int64_t q = 1; q < d; ++q)
        if (r[q] == r[q - 1]) { ok = false; return; }
    }
  });
  if (!ok) return false;
  // symmetry: every arc v->u has u->v
  parallel_rows(n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e && ok.load(std::memory_order_relaxed); ++v)
      for (int64_t q = rp[v]; q < rp[v + 1]; ++q) {
        const int32_t u = sorted[q];
        const int32_t* ub = sorted.data() + rp[u];
        const int32_t* ue = sorted.data() + rp[u + 1];
        if (!std::binary_search(ub, ue, (int32_t)v)) { ok = false; return; }
      }
  });
  return ok;
}

}  // namespace

struct StripeLayout {
  int32_t count = 0;          // S
  std::vector<int32_t> rp;    // [S][n+1]
  std::vector<int32_t> cols;  // stripe CSRs concatenated
  int64_t col_off[kMaxStripes] = {};
  int64_t base[kMaxStripes] = {};   // first node of each stripe
  bool packed = false;              // tile blocks in the packed form (common.h)
  std::vector<StripeBlock> blocks;  // [tiles][S]
  int64_t ntiles = 0, nlong = 0;
};

// Per-stripe CSRs of a graph already relabelled into S contiguous
// stripes, and the row tiles of the striped step (see common.h).  Stripe
// offsets are int32: returns false when one stripe holds 2^31 arcs or more.
bool build_stripes(const int64_t* rp, const int32_t* ci, int64_t n, int32_t S, StripeLayout& sl) {
  sl.count = S;
  int64_t start[kMaxStripes + 1] = {0};
  for (int j = 0; j < S; ++j) start[j + 1] = start[j] + (n - j + S - 1) / S;
  // per row, per stripe arc counts (rows are sorted by column)
  std::vector<int32_t> cnt((size_t)n * S);
  parallel_rows_balanced(rp, n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      const int32_t* r = ci + rp[v];
      const int32_t* re = ci + rp[v + 1];
      const int32_t* lo = r;
      for (int j = 0; j < S; ++j) {
        const int32_t* hi = std::lower_bound(lo, re, (int32_t)start[j + 1]);
        cnt[(size_t)v * S + j] = (int32_t)(hi - lo);
        lo = hi;
      }
    }
  });
  for (int j = 0; j < S; ++j) {
    int64_t arcs = 0;
    for (int64_t v = 0; v < n; ++v) arcs += cnt[(size_t)v * S + j];
    if (arcs > INT32_MAX) return false;
  }
  sl.rp.assign((size_t)S * (n + 1), 0);
  int64_t total = 0;
  for (int j = 0; j < S; ++j) {
    int32_t* rj = sl.rp.data() + (size_t)j * (n + 1);
    int64_t acc = 0;
    for (int64_t v = 0; v < n; ++v) {
      rj[v] = (int32_t)acc;
      acc += cnt[(size_t)v * S + j];
    }
    rj[n] = (int32_t)acc;
    sl.col_off[j] = total;
    total += acc;
  }
  sl.cols.resize((size_t)total);
  parallel_rows_balanced(rp, n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      const int32_t* src = ci + rp[v];
      for (int j = 0; j < S; ++j) {
        const int32_t c = cnt[(size_t)v * S + j];
        int32_t* dst = sl.cols.data() + sl.col_off[j] + sl.rp[(size_t)j * (n + 1) + v];
        std::copy(src, src + c, dst);
        src += c;
      }
    }
  });
  // row tiles: at most kStripeTileRows rows and kStripeTileNnz arcs per stripe
  int64_t r0 = -1;
  int64_t acc[kMaxStripes] = {0};
  auto emit = [&](int64_t a, int64_t b) {  // one tile = S blocks
    for (int j = 0; j < S; ++j) {
      const int32_t* rj = sl.rp.data() + (size_t)j * (n + 1);
      sl.blocks.push_back(StripeBlock{(int32_t)a, (int32_t)(b - a), rj[a], rj[b] - rj[a]});
    }
    ++sl.ntiles;
  };
  auto close = [&](int64_t r1) {
    if (r0 >= 0) emit(r0, r1);
    r0 = -1;
  };
  for (int64_t v = 0; v < n; ++v) {
    const int32_t* c = cnt.data() + (size_t)v * S;
    const int32_t cmax = *std::max_element(c, c + S);
    if (cmax > kStripeTileNnz) {
      close(v);
      emit(v, v + 1);  // stripes of this row above the tile size stream it whole
      ++sl.nlong;
      continue;
    }
    bool full = r0 >= 0 && v - r0 == kStripeTileRows;
    for (int j = 0; j < S && !full; ++j) full = r0 >= 0 && acc[j] + c[j] > kStripeTileNnz;
    if (full) close(v);
    if (r0 < 0) {
      r0 = v;
      for (int j = 0; j < S; ++j) acc[j] = 0;
    }
    for (int j = 0; j < S; ++j) acc[j] += c[j];
  }
  close(n);
  // packed form: each tile block's arcs sorted by column (ties in CSR
  // order), stored as local column << kPackPosBits | CSR position
  for (int j = 0; j < S; ++j) sl.base[j] = start[j];
  sl.packed = start[1] - start[0] <= ((int64_t)1 << kPackLocalBits);
  if (sl.packed) {
    const int64_t nb = (int64_t)sl.blocks.size();
    parallel_rows(nb, [&](int64_t b, int64_t e) {
      std::vector<uint64_t> key;
      for (int64_t q = b; q < e; ++q) {
        const StripeBlock& sb = sl.blocks[(size_t)q];
        if (sb.cnt > kStripeTileNnz || sb.cnt == 0) continue;
        const int j = (int)(q % S);
        int32_t* c = sl.cols.data() + sl.col_off[j] + sb.p0;
        key.resize((size_t)sb.cnt);
        for (int32_t i = 0; i < sb.cnt; ++i)
          key[(size_t)i] = ((uint64_t)(c[i] - start[j]) << kPackPosBits) | (uint64_t)i;
        std::sort(key.begin(), key.end());
        for (int32_t i = 0; i < sb.cnt; ++i) c[i] = (int32_t)(uint32_t)key[(size_t)i];
      }
    });
  }
  return true;
}

// Host image of the hot/cold split of the batched step (CP_GRAPH_HOT_SPLIT).
struct SplitHost {
  int64_t hot_nodes = 0;
  std::vector<int64_t> hrp, crp;   // [n+1] row offsets of the hot and cold CSRs
  std::vector<int32_t> hci, cci;   // their columns, each row in the graph's order
  Plan hot, cold;
};

// Hot nodes: CHEBYPROP_HOT_NODES if set, else a 16 MiB slice of 8-wide FP32
// rows (32 bytes a node, 524,288 nodes); at most n.
int64_t hot_nodes_for(int64_t n) {
  int64_t h = (int64_t(16) << 20) / 32;
  if (const char* env = std::getenv("CHEBYPROP_HOT_NODES")) {
    const long long v = std::atoll(env);
    if (v >= 0) h = v;
  }
  return std::min<int64_t>(h, n);
}

// Split each row of the (relabelled) CSR into its arcs into the H
// highest-degree nodes and the rest, keeping their order.  In degree order
// the hot nodes are ids [0, H); with S stripes (degree rank r at stripe
// r % S, position r / S) they are the first ceil((H - j) / S) ids of each
// stripe j.
void build_split(const int64_t* rp, const int32_t* ci, int64_t n, int32_t S, int64_t H, SplitHost& sp) {
  sp.hot_nodes = H;
  std::vector<uint8_t> hot((size_t)n, 0);
  if (S == 0) {
    std::fill(hot.begin(), hot.begin() + H, 1);
  } else {
    int64_t start = 0;
    for (int j = 0; j < S; ++j) {
      const int64_t size = (n - j + S - 1) / S;
      const int64_t nh = H > j ? (H - j + S - 1) / S : 0;
      std::fill(hot.begin() + start, hot.begin() + start + std::min(nh, size), 1);
      start += size;
    }
  }
  std::vector<int32_t> cnt((size_t)n);
  parallel_rows_balanced(rp, n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int32_t c = 0;
      for (int64_t q = rp[v]; q < rp[v + 1]; ++q) c += hot[(size_t)ci[q]];
      cnt[(size_t)v] = c;
    }
  });
  sp.hrp.assign((size_t)n + 1, 0);
  sp.crp.assign((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    sp.hrp[(size_t)v + 1] = sp.hrp[(size_t)v] + cnt[(size_t)v];
    sp.crp[(size_t)v + 1] = sp.crp[(size_t)v] + (rp[v + 1] - rp[v] - cnt[(size_t)v]);
  }
  sp.hci.resize((size_t)sp.hrp[(size_t)n]);
  sp.cci.resize((size_t)sp.crp[(size_t)n]);
  parallel_rows_balanced(rp, n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int32_t* h = sp.hci.data() + sp.hrp[(size_t)v];
      int32_t* c = sp.cci.data() + sp.crp[(size_t)v];
      for (int64_t q = rp[v]; q < rp[v + 1]; ++q) {
        const int32_t u = ci[q];
        if (hot[(size_t)u]) *h++ = u;
        else *c++ = u;
      }
    }
  });
  sp.hot = build_plan(sp.hrp.data(), n, PlanShape{kBatchLong});
  sp.cold = build_plan(sp.crp.data(), n, PlanShape{kBatchLong});
}

Plan build_plan(const int64_t* rp, int64_t n, const PlanShape& shape) {
  Plan p;
  p.shape = shape;
  const int64_t long_threshold = shape.long_cut;
  std::vector<int32_t> hubs, longs;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = rp[v + 1] - rp[v];
    if (d > shape.hub_cut) hubs.push_back((int32_t)v);
    else if (d > long_threshold) longs.push_back((int32_t)v);
  }
  auto by_degree = [&](int32_t a, int32_t b) {
    const int64_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
    return da != db ? da > db : a < b;
  };
  std::sort(hubs.begin(), hubs.end(), by_degree);
  std::sort(longs.begin(), longs.end(), by_degree);
  int32_t base = 0;
  for (size_t h = 0; h < hubs.size(); ++h) {
    const int64_t d = rp[hubs[h] + 1] - rp[hubs[h]];
    const int32_t nseg = (int32_t)((d + shape.hub_seg - 1) / shape.hub_seg);
    p.hubs.push_back(HubDesc{hubs[h], nseg, base, (int32_t)shape.hub_seg});
    for (int32_t s = 0; s < nseg; ++s) p.blocks.push_back(BlockDesc{hubs[h], (int32_t)h, kHub, s, 0, 0});
    base += nseg;
  }
  p.hub_segments = base;
  for (int32_t v : longs) p.blocks.push_back(BlockDesc{v, v + 1, kLong, 0, 0, 0});
  p.nlong = (int64_t)longs.size();
  p.nspecial = (int64_t)p.blocks.size();
  // greedy stream tiles over the remaining rows, in row order
  int64_t r0 = -1, nnz = 0;
  auto close = [&](int64_t r1) {
    if (r0 >= 0) p.blocks.push_back(BlockDesc{(int32_t)r0, (int32_t)r1, kStream, (int32_t)nnz, rp[r0], 0});
    r0 = -1;
    nnz = 0;
  };
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = rp[v + 1] - rp[v];
    if (d > long_threshold) { close(v); continue; }
    if (r0 >= 0 && (nnz + d > kTileNnz || v - r0 == kTileRows)) close(v);
    if (r0 < 0) r0 = v;
    nnz += d;
  }
  close(n);
  return p;
}

int64_t batch_hub_rows(const cp_graph* g) { return g->hub_rows_cap; }

int64_t batch_hub_segments(const cp_graph* g) { return g->hub_segs_cap; }

// Row-split shapes of hubs the autotuners try (the first is the default).
const PlanShape kHubShapes[3] = {{0, kHubThreshold, kHubSeg}, {0, 4096, 2048}, {0, 65536, 16384}};

// The most hub rows and segments any of those shapes makes of these rows (a
// split CSR's rows are no longer than the graph's, so this bounds them too).
void hub_caps(const int64_t* rp, int64_t n, int64_t* rows_cap, int64_t* segs_cap) {
  int64_t rc = 1, sc = 1;
  for (const PlanShape& sh : kHubShapes) {
    int64_t r = 0, sg = 0;
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = rp[v + 1] - rp[v];
      if (d > sh.hub_cut) {
        ++r;
        sg += (d + sh.hub_seg - 1) / sh.hub_seg;
      }
    }
    rc = std::max(rc, r);
    sc = std::max(sc, sg);
  }
  *rows_cap = rc;
  *segs_cap = sc;
}

void set_batch_plan(const cp_graph* g, BatchStepArgs& a, void* part) {
  a.row_ptr = g->row_ptr;
  a.col_idx = g->col_idx;
  a.blocks = g->batch.blocks;
  a.hubs = g->batch.hubs;
  a.nblocks = g->batch.nblocks;
  a.nspecial = g->batch.nspecial;
  a.split = g->hot_split ? &g->split : nullptr;
  a.deg_rp = nullptr;
  a.part = g->hot_split ? part : nullptr;
}

namespace {

struct WsLayout {
  size_t rA, rB, yacc, hub_count, hub_partial, mass, partial, total;
};

WsLayout ws_layout(const cp_graph* g, int32_t nq, int32_t prec) {
  WsLayout L{};
  const size_t vec = align256((size_t)g->n * (size_t)nq * storage_bytes(prec));
  const size_t yv = align256((size_t)g->n * (size_t)nq * acc_bytes(prec));
  size_t off = 0;
  L.rA = off; off += vec;
  L.rB = off; off += vec;
  L.yacc = off; off += yv;
  L.hub_count = off; off += align256((size_t)batch_hub_rows(g) * 4);
  L.hub_partial = off; off += align256((size_t)batch_hub_segments(g) * 8 * nq);
  L.mass = off; off += align256((1 + 1024) * 8);
  L.partial = off;
  if (g->striped) off += align256((size_t)g->s_count * (size_t)g->n * acc_bytes(prec));
  L.total = off;
  return L;
}

}  // namespace

size_t single_ws_bytes(const cp_graph* g, int32_t prec) { return ws_layout(g, 1, prec).total; }

cp_status plan_query(const cp_graph* g, const cp_query* q, int32_t K_max, QueryPlan* p) {
  if (!q || !p) return CP_EINVAL;
  if (q->kind != CP_PPR && q->kind != CP_HKPR) return CP_EINVAL;
  if (q->flags & ~(CP_Q_STATS | CP_Q_TIMING | CP_Q_PWMETHOD)) return CP_EINVAL;
  if (!(q->a >= 0.0 && q->a <= 1.0)) return CP_EINVAL;
  if (q->source < 0 || q->source >= g->n) return CP_ESOURCE;
  const int32_t ds = g->degree[q->source];
  if (ds == 0) return CP_EISOLATED;
  p->s_int = g->reordered ? g->ext2int[q->source] : q->source;
  p->oexp = 1.0 - q->a;
  p->oscale = q->a == 0.0 ? 1.0 : std::pow((double)ds, q->a);
  cp_status rc;
  if (q->flags & CP_Q_PWMETHOD) {
    // N terms zeta_0..zeta_{N-1}; the highest index N - 1 must fit K_max
    rc = choose_N_impl(q->kind, q->param, q->tol, q->kmode, q->K_fixed, K_max + 1, &p->K, &p->tail);
    if (rc != CP_OK) return rc;
    p->top = std::max(p->K - 1, 1);
    p->L = 1.0;
    p->rec = 1.0;
    p->c.assign((size_t)p->top + 1, 0.0);
    return taylor_impl(q->kind, q->param, p->K, p->c.data());
  }
  rc = choose_K_impl(q->kind, q->param, q->tol, q->kmode, q->K_fixed, (double)g->nnz, (double)ds, K_max,
                     &p->K, &p->tail);
  if (rc != CP_OK) return rc;
  p->top = p->K;
  p->L = std::sqrt((double)g->nnz / (double)ds);
  p->rec = 2.0;
  p->c.assign((size_t)p->K + 1, 0.0);
  return coeffs_impl(q->kind, q->param, p->K, p->c.data());
}

// Host image of the slot parameters (see kSlotParams): step factor 2,
// output exponent 1, output scale 1, ones.
std::vector<double> slot_params(int32_t nslots) {
  std::vector<double> sp((size_t)kSlotParams * nslots, 1.0);
  std::fill(sp.begin(), sp.begin() + nslots, 2.0);
  return sp;
}

namespace {

struct BatchLayout {
  int32_t bw = 0, nq_pad = 0, ntiles = 0;
  size_t rA = 0, rB = 0, yacc = 0, hub_count = 0, hub_partial = 0, coef = 0, src = 0, rec = 0, slotmap = 0,
         part = 0, total = 0;
};

int32_t round_up(int32_t a, int32_t b) { return (a + b - 1) / b * b; }

BatchLayout batch_layout(const cp_graph* g, int32_t nq, int32_t prec, int32_t bw) {
  BatchLayout L;
  L.bw = bw;
  L.nq_pad = round_up(nq, bw);
  L.ntiles = L.nq_pad / bw;
  const size_t vec = align256((size_t)g->n * (size_t)L.nq_pad * storage_bytes(prec));
  const size_t yv = align256((size_t)g->n * (size_t)L.nq_pad * acc_bytes(prec));
  size_t off = 0;
  L.rA = off; off += vec;
  L.rB = off; off += vec;
  L.yacc = off; off += yv;
  L.hub_count = off; off += align256((size_t)batch_hub_rows(g) * L.ntiles * 4);
  L.hub_partial = off; off += align256((size_t)batch_hub_segments(g) * L.nq_pad * 8);
  L.coef = off; off += align256((size_t)(kBatchKCap + 1) * L.nq_pad * 8);
  L.src = off; off += align256((size_t)L.nq_pad * 8);
  L.rec = off; off += align256((size_t)kSlotParams * L.nq_pad * 8);
  L.slotmap = off; off += align256((size_t)nq * 4);
  L.part = off;
  if (g->hot_split) off += yv;  // partial row sums of the hot pass
  L.total = off;
  return L;
}

const int32_t kBatchWidths[] = {8, 16, 32, 64};

bool width_allowed(int32_t nq, int32_t bw) {
  int32_t cap = 8;
  while (cap < nq && cap < 64) cap *= 2;
  return bw <= cap;
}

size_t batch_ws_bytes(const cp_graph* g, int32_t nq, int32_t prec) {
  size_t m = 0;
  for (int32_t bw : kBatchWidths)
    if (width_allowed(nq, bw)) m = std::max(m, batch_layout(g, nq, prec, bw).total);
  return m;
}

int64_t tune_key(int32_t nq, int32_t prec) { return ((int64_t)nq << 4) | prec; }

int32_t choose_bw(cp_graph* g, int32_t nq, int32_t prec) {
  {
    std::lock_guard<std::mutex> lk(g->tune_mu);
    auto it = g->tuned_bw.find(tune_key(nq, prec));
    if (it != g->tuned_bw.end()) return it->second;
  }
  int32_t bw = 8;
  while (bw < nq && bw < 32) bw *= 2;
  return bw;
}

}  // namespace
}  // namespace cp

using namespace cp;

namespace {

// Free every device allocation a (possibly partially built) graph holds.
hipError_t release_graph(cp_graph* g) {
  if (!g) return hipSuccess;
  hipError_t e = hipSuccess;
  for (void* p : {g->owned_csr, g->plan_mem, static_cast<void*>(g->s_rp), g->split_mem, g->tuned_plan_mem[0],
                  g->tuned_plan_mem[1]}) {
    if (!p) continue;
    const hipError_t x = hipFree(p);
    if (e == hipSuccess) e = x;
  }
  delete g;
  return e;
}

}  // namespace

// Workspace of cp_power_noalloc: one array per device, held until the
// process ends.  Host code never uses this name as an address (on the host
// it stands for the symbol); noalloc_scratch looks up the device address.
static __device__ __align__(256) unsigned char scratch[CP_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};  // device address of `scratch`, per device id

// The device address of `scratch` on device dev (the current device),
// looked up on the first call for that device.
cp_status noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= 64) return CP_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_hip_error(e);
      return CP_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CP_OK;
}

cp_status power_impl(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws, size_t ws_bytes,
                     void* stream, cp_info* info);

}  // namespace

extern "C" {

const char* cp_version(void) { return "chebyprop 0.1 (gfx950)"; }

int32_t cp_last_hip_error(void) { return g_last_hip_error; }

const char* cp_status_str(int32_t st) {
  switch (st) {
    case CP_OK: return "ok";
    case CP_EINVAL: return "invalid argument";
    case CP_ESOURCE: return "source out of range";
    case CP_EISOLATED: return "source has degree 0";
    case CP_ENOMEM: return "out of memory";
    case CP_EHIP: return "HIP runtime error";
    case CP_EKMAX: return "tolerance needs too many terms";
    case CP_EBUSY: return "admission refused";
    case CP_ECANCELLED: return "query cancelled";
    case CP_ENOTFOUND: return "unknown ticket";
    case CP_EGRAPH: return "graph validation failed";
    case CP_EPENDING: return "query pending";
    case CP_EWORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
  }
}

cp_status cp_coeffs(int32_t kind, double param, int32_t K, double* c_out) {
  return coeffs_impl(kind, param, K, c_out);
}

cp_status cp_choose_K(int32_t kind, double param, double tol, int32_t kmode, int32_t K_fixed,
                      double vol, double d_s, int32_t K_max, int32_t* K_out, double* tail_out) {
  return choose_K_impl(kind, param, tol, kmode, K_fixed, vol, d_s, K_max, K_out, tail_out);
}

cp_status cp_taylor(int32_t kind, double param, int32_t N, double* zeta_out) {
  return taylor_impl(kind, param, N, zeta_out);
}

cp_status cp_choose_N(int32_t kind, double param, double tol, int32_t kmode, int32_t N_fixed, int32_t N_max,
                      int32_t* N_out, double* tail_out) {
  return choose_N_impl(kind, param, tol, kmode, N_fixed, N_max, N_out, tail_out);
}

cp_status cp_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          int32_t flags, void* stream, cp_graph** out) {
  if (!out || !row_ptr || n < 1 || n >= INT32_MAX || nnz < 0 || (nnz > 0 && !col_idx))
    return CP_EINVAL;
  *out = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool host_in = flags & CP_GRAPH_HOST;
  const bool striped = flags & CP_GRAPH_XCD_STRIPES;
  const int32_t S = stripe_count(n);  // stripes, if striped
  const bool hot_split = flags & CP_GRAPH_HOT_SPLIT;
  const bool reorder = (flags & CP_GRAPH_REORDER) || striped || hot_split;
  const bool borrow = (flags & CP_GRAPH_BORROW) && !host_in && !reorder;
  cp_graph* g = nullptr;
#define CP_HIP_G(call)      \
  do {                      \
    hipError_t e_ = (call); \
    if (e_ != hipSuccess) { \
      set_hip_error(e_);    \
      (void)release_graph(g); \
      return CP_EHIP;       \
    }                       \
  } while (0)
  try {
    g = new cp_graph();
    g->n = n;
    g->nnz = nnz;
    CP_HIP_G(hipGetDevice(&g->device));
    PhaseClock clock;
    // host copy of the row offsets; host view of the columns when needed:
    // the caller's array (CP_GRAPH_HOST) or a copy from the device
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> ci;
    const int32_t* hci = host_in ? col_idx : nullptr;
    const bool need_cols = (flags & CP_GRAPH_VALIDATE) || reorder;
    if (host_in) {
      std::memcpy(rp.data(), row_ptr, sizeof(int64_t) * (n + 1));
    } else {
      CP_HIP_G(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
      if (need_cols) {
        ci.resize(nnz);
        if (nnz)
          CP_HIP_G(hipMemcpyAsync(ci.data(), col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
        hci = ci.data();
      }
    }
    CP_HIP_G(hipStreamSynchronize(st));
    clock.mark("host copy");
    if (rp[0] != 0 || rp[n] != nnz) { (void)release_graph(g); return CP_EINVAL; }
    if ((flags & CP_GRAPH_VALIDATE) && !validate_csr(n, nnz, rp.data(), hci)) {
      (void)release_graph(g);
      return CP_EGRAPH;
    }
    g->degree.resize(n);
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = rp[v + 1] - rp[v];
      if (d < 0 || d > INT32_MAX) {  // non-monotone offsets would make negative-length tiles
        (void)release_graph(g);
        return CP_EINVAL;
      }
      g->degree[v] = (int32_t)d;
      g->d_max = std::max(g->d_max, d);
    }
    // internal order
    std::vector<int32_t> perm;  // internal -> caller
    if (reorder) {
      // decreasing degree, ties in caller order: a counting sort on degrees
      perm.resize(n);
      {
        std::vector<int64_t> first((size_t)g->d_max + 1, 0);
        for (int64_t v = 0; v < n; ++v) ++first[(size_t)g->degree[v]];
        int64_t acc = 0;
        for (int64_t d = g->d_max; d >= 0; --d) {
          const int64_t c = first[(size_t)d];
          first[(size_t)d] = acc;
          acc += c;
        }
        for (int64_t v = 0; v < n; ++v) perm[(size_t)first[(size_t)g->degree[v]]++] = (int32_t)v;
      }
      if (striped) {
        // degree rank r -> stripe r % S, position r / S (stripes contiguous)
        std::vector<int32_t> by_rank(perm);
        int64_t start[kMaxStripes + 1] = {0};
        for (int j = 0; j < S; ++j) start[j + 1] = start[j] + (n - j + S - 1) / S;
        for (int64_t r = 0; r < n; ++r) perm[start[r % S] + r / S] = by_rank[r];
      }
      g->ext2int.resize(n);
      for (int64_t i = 0; i < n; ++i) g->ext2int[perm[i]] = (int32_t)i;
      std::vector<int64_t> rp2(n + 1, 0);
      for (int64_t i = 0; i < n; ++i) rp2[i + 1] = rp2[i] + g->degree[perm[i]];
      clock.mark("order");
      std::vector<int32_t> ci2(nnz);
      parallel_rows_balanced(rp2.data(), n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
          const int32_t v = perm[i];
          int32_t* dst = ci2.data() + rp2[i];
          for (int64_t q = rp[v]; q < rp[v + 1]; ++q) *dst++ = g->ext2int[hci[q]];
          std::sort(ci2.data() + rp2[i], dst);
        }
      });
      rp.swap(rp2);
      ci.swap(ci2);
      hci = ci.data();
      g->reordered = true;
      clock.mark("relabel");
    }
    const Plan plans[2] = {build_plan(rp.data(), n, PlanShape{kTileNnz}), build_plan(rp.data(), n, PlanShape{kBatchLong})};
    hub_caps(rp.data(), n, &g->hub_rows_cap, &g->hub_segs_cap);
    clock.mark("plans");
    StripeLayout sl;
    if (striped && !build_stripes(rp.data(), hci, n, S, sl)) {
      (void)release_graph(g);
      return CP_EINVAL;
    }
    if (striped) clock.mark("stripes");
    SplitHost sp;
    if (hot_split) {
      build_split(rp.data(), hci, n, striped ? S : 0, hot_nodes_for(n), sp);
      clock.mark("hot split");
    }

    // device copies: [row_ptr | col_idx | perm] in one allocation, plans in another
    const size_t b_rp = borrow ? 0 : align256(sizeof(int64_t) * (n + 1));
    const size_t b_ci = borrow ? 0 : align256(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    const size_t b_pm = reorder ? align256(sizeof(int32_t) * n) : 0;
    const size_t total = b_rp + b_ci + b_pm;
    char* base = nullptr;
    if (total) {
      hipError_t e = hipMalloc(&base, total);
      if (e != hipSuccess) {
        (void)release_graph(g);
        return e == hipErrorOutOfMemory ? CP_ENOMEM : (set_hip_error(e), CP_EHIP);
      }
      g->owned_csr = base;
    }
    size_t b_plans = 0;
    for (const Plan& pl : plans)
      b_plans += align256(sizeof(BlockDesc) * std::max<size_t>(pl.blocks.size(), 1)) +
                 align256(sizeof(HubDesc) * std::max<size_t>(pl.hubs.size(), 1));
    char* pbase = nullptr;
    {
      hipError_t e = hipMalloc(&pbase, b_plans);
      if (e != hipSuccess) {
        (void)release_graph(g);
        return e == hipErrorOutOfMemory ? CP_ENOMEM : (set_hip_error(e), CP_EHIP);
      }
      g->plan_mem = pbase;
    }
    size_t b_stripes = 0;
    if (striped) {
      b_stripes = align256(sizeof(int32_t) * (size_t)S * (n + 1)) +
                  align256(sizeof(int32_t) * std::max<size_t>(sl.cols.size(), 1)) +
                  align256(sizeof(StripeBlock) * std::max<size_t>(sl.blocks.size(), 1));
      char* sb = nullptr;
      hipError_t e = hipMalloc(&sb, b_stripes);
      if (e != hipSuccess) {
        (void)release_graph(g);
        return e == hipErrorOutOfMemory ? CP_ENOMEM : (set_hip_error(e), CP_EHIP);
      }
      g->striped = true;
      g->s_rp = reinterpret_cast<int32_t*>(sb);
      sb += align256(sizeof(int32_t) * (size_t)S * (n + 1));
      g->s_cols = reinterpret_cast<int32_t*>(sb);
      sb += align256(sizeof(int32_t) * std::max<size_t>(sl.cols.size(), 1));
      g->s_blocks = reinterpret_cast<StripeBlock*>(sb);
      g->s_ntiles = sl.ntiles;
      g->s_nlong = sl.nlong;
      g->s_count = S;
      for (int j = 0; j < S; ++j) g->s_col_off[j] = sl.col_off[j];
      for (int j = 0; j < S; ++j) g->s_base[j] = sl.base[j];
      g->s_packed = sl.packed;
      CP_HIP_G(hipMemcpyAsync(g->s_rp, sl.rp.data(), sizeof(int32_t) * sl.rp.size(), hipMemcpyHostToDevice, st));
      if (!sl.cols.empty())
        CP_HIP_G(hipMemcpyAsync(g->s_cols, sl.cols.data(), sizeof(int32_t) * sl.cols.size(), hipMemcpyHostToDevice,
                              st));
      if (!sl.blocks.empty())
        CP_HIP_G(hipMemcpyAsync(g->s_blocks, sl.blocks.data(), sizeof(StripeBlock) * sl.blocks.size(),
                              hipMemcpyHostToDevice, st));
    }
    size_t b_split = 0;
    if (hot_split) {
      const size_t b_rps = align256(sizeof(int64_t) * (n + 1));
      const size_t b_hci = align256(sizeof(int32_t) * std::max<size_t>(sp.hci.size(), 1));
      const size_t b_cci = align256(sizeof(int32_t) * std::max<size_t>(sp.cci.size(), 1));
      size_t b_pl = 0;
      for (const Plan* pl : {&sp.hot, &sp.cold})
        b_pl += align256(sizeof(BlockDesc) * std::max<size_t>(pl->blocks.size(), 1)) +
                align256(sizeof(HubDesc) * std::max<size_t>(pl->hubs.size(), 1));
      b_split = 2 * b_rps + b_hci + b_cci + b_pl;
      char* m = nullptr;
      hipError_t e = hipMalloc(&m, b_split);
      if (e != hipSuccess) {
        (void)release_graph(g);
        return e == hipErrorOutOfMemory ? CP_ENOMEM : (set_hip_error(e), CP_EHIP);
      }
      g->split_mem = m;
      g->hot_split = true;
      g->split.hot_nodes = sp.hot_nodes;
      g->hot_arcs = (int64_t)sp.hci.size();
      int64_t* drh = reinterpret_cast<int64_t*>(m); m += b_rps;
      int64_t* drc = reinterpret_cast<int64_t*>(m); m += b_rps;
      int32_t* dch = reinterpret_cast<int32_t*>(m); m += b_hci;
      int32_t* dcc = reinterpret_cast<int32_t*>(m); m += b_cci;
      CP_HIP_G(hipMemcpyAsync(drh, sp.hrp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
      CP_HIP_G(hipMemcpyAsync(drc, sp.crp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
      if (!sp.hci.empty())
        CP_HIP_G(hipMemcpyAsync(dch, sp.hci.data(), sizeof(int32_t) * sp.hci.size(), hipMemcpyHostToDevice, st));
      if (!sp.cci.empty())
        CP_HIP_G(hipMemcpyAsync(dcc, sp.cci.data(), sizeof(int32_t) * sp.cci.size(), hipMemcpyHostToDevice, st));
      DevPlan* dps[2] = {&g->hot_plan, &g->cold_plan};
      const Plan* pls[2] = {&sp.hot, &sp.cold};
      for (int i = 0; i < 2; ++i) {
        DevPlan& dp = *dps[i];
        const Plan& pl = *pls[i];
        dp.nblocks = (int64_t)pl.blocks.size();
        dp.nspecial = pl.nspecial;
        dp.nlong = pl.nlong;
        dp.nhubs = (int64_t)pl.hubs.size();
        dp.hub_segments = pl.hub_segments;
        dp.shape = pl.shape;
        dp.blocks = reinterpret_cast<BlockDesc*>(m);
        m += align256(sizeof(BlockDesc) * std::max<size_t>(pl.blocks.size(), 1));
        dp.hubs = reinterpret_cast<HubDesc*>(m);
        m += align256(sizeof(HubDesc) * std::max<size_t>(pl.hubs.size(), 1));
        if (dp.nblocks)
          CP_HIP_G(hipMemcpyAsync(dp.blocks, pl.blocks.data(), sizeof(BlockDesc) * dp.nblocks,
                                  hipMemcpyHostToDevice, st));
        if (dp.nhubs)
          CP_HIP_G(hipMemcpyAsync(dp.hubs, pl.hubs.data(), sizeof(HubDesc) * dp.nhubs, hipMemcpyHostToDevice, st));
      }
      g->split.hot = BatchPass{drh, dch, g->hot_plan.blocks, g->hot_plan.hubs, g->hot_plan.nblocks,
                               g->hot_plan.nspecial};
      g->split.cold = BatchPass{drc, dcc, g->cold_plan.blocks, g->cold_plan.hubs, g->cold_plan.nblocks,
                                g->cold_plan.nspecial};
    }
    g->device_bytes = (int64_t)(total + b_plans + b_stripes + b_split);
    char* p = base;
    if (borrow) {
      g->row_ptr = row_ptr;
      g->col_idx = col_idx;
      g->borrowed = true;
    } else {
      int64_t* drp = reinterpret_cast<int64_t*>(p); p += b_rp;
      int32_t* dci = reinterpret_cast<int32_t*>(p); p += b_ci;
      CP_HIP_G(hipMemcpyAsync(drp, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
      if (nnz) {
        if (hci)
          CP_HIP_G(hipMemcpyAsync(dci, hci, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
        else
          CP_HIP_G(hipMemcpyAsync(dci, col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st));
      }
      g->row_ptr = drp;
      g->col_idx = dci;
    }
    if (reorder) {
      g->perm = reinterpret_cast<int32_t*>(p); p += b_pm;
      CP_HIP_G(hipMemcpyAsync(g->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    }
    DevPlan* dps[2] = {&g->single, &g->batch};
    char* q = pbase;
    for (int i = 0; i < 2; ++i) {
      const Plan& pl = plans[i];
      DevPlan& dp = *dps[i];
      dp.nblocks = (int64_t)pl.blocks.size();
      dp.nspecial = pl.nspecial;
      dp.nlong = pl.nlong;
      dp.nhubs = (int64_t)pl.hubs.size();
      dp.hub_segments = pl.hub_segments;
      dp.shape = pl.shape;
      dp.blocks = reinterpret_cast<BlockDesc*>(q);
      q += align256(sizeof(BlockDesc) * std::max<size_t>(pl.blocks.size(), 1));
      dp.hubs = reinterpret_cast<HubDesc*>(q);
      q += align256(sizeof(HubDesc) * std::max<size_t>(pl.hubs.size(), 1));
      if (dp.nblocks)
        CP_HIP_G(hipMemcpyAsync(dp.blocks, pl.blocks.data(), sizeof(BlockDesc) * dp.nblocks,
                              hipMemcpyHostToDevice, st));
      if (dp.nhubs)
        CP_HIP_G(hipMemcpyAsync(dp.hubs, pl.hubs.data(), sizeof(HubDesc) * dp.nhubs,
                              hipMemcpyHostToDevice, st));
    }
    CP_HIP_G(hipStreamSynchronize(st));
    clock.mark("upload");
    g->host_rp.swap(rp);
    *out = g;
    return CP_OK;
  } catch (const std::bad_alloc&) {
    (void)release_graph(g);
    return CP_ENOMEM;
  }
#undef CP_HIP_G
}

cp_status cp_graph_destroy(cp_graph* g) {
  if (!g) return CP_EINVAL;
  const hipError_t e = release_graph(g);
  if (e != hipSuccess) { set_hip_error(e); return CP_EHIP; }
  return CP_OK;
}

cp_status cp_graph_get_stats(const cp_graph* g, cp_graph_stats* out) {
  if (!g || !out) return CP_EINVAL;
  out->n = g->n;
  out->nnz = g->nnz;
  out->d_max = g->d_max;
  out->blocks = g->single.nblocks;
  out->long_rows = g->single.nlong;
  out->hub_rows = g->single.nhubs;
  out->device_bytes = g->device_bytes;
  out->reordered = g->reordered;
  out->borrowed = g->borrowed;
  out->stripe_tiles = g->s_ntiles;
  out->stripe_packed = g->s_packed ? 1 : 0;
  out->stripe_count = g->striped ? g->s_count : 0;
  out->hot_nodes = g->hot_split ? g->split.hot_nodes : 0;
  out->single_long_cut = g->single.shape.long_cut;
  out->single_hub_cut = g->single.shape.hub_cut;
  out->single_hub_seg = g->single.shape.hub_seg;
  out->batch_long_cut = g->batch.shape.long_cut;
  out->batch_hub_cut = g->batch.shape.hub_cut;
  out->batch_hub_seg = g->batch.shape.hub_seg;
  out->hot_arcs = g->hot_split ? g->hot_arcs : 0;
  return CP_OK;
}

size_t cp_workspace_bytes(const cp_graph* g, int32_t nq, int32_t prec) {
  if (!g || nq < 1 || !valid_prec(prec)) return 0;
  if (nq == 1) return std::max(ws_layout(g, 1, prec).total, batch_ws_bytes(g, 1, prec));
  return batch_ws_bytes(g, nq, prec);
}

cp_status cp_power(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws,
                   size_t ws_bytes, void* stream, cp_info* info) {
  return power_impl(g, q, prec, y, ws, ws_bytes, stream, info);
}

cp_status cp_power_noalloc(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* stream,
                           cp_info* info) {
  if (!g || !q || !y || !valid_prec(prec)) return CP_EINVAL;
  if (q->flags & CP_Q_TIMING) return CP_EINVAL;
  int dev = -1;
  CP_HIP(hipGetDevice(&dev));
  if (dev != g->device) return CP_EINVAL;
  if (ws_layout(g, 1, prec).total > CP_NOALLOC_SCRATCH_BYTES) return CP_EWORKSPACE;
  void* ws = nullptr;
  const cp_status rc = noalloc_scratch(dev, &ws);
  if (rc != CP_OK) return rc;
  return power_impl(g, q, prec, y, ws, CP_NOALLOC_SCRATCH_BYTES, stream, info);
}

}  // extern "C"

namespace {

cp_status power_impl(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws, size_t ws_bytes,
                     void* stream, cp_info* info) {
  if (!g || !q || !y || !valid_prec(prec)) return CP_EINVAL;
  QueryPlan qp;
  cp_status rc = plan_query(g, q, kDefaultKMax, &qp);
  if (rc != CP_OK) return rc;
  const WsLayout W = ws_layout(g, 1, prec);
  if (!ws || ws_bytes < W.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return CP_EWORKSPACE;
  const int64_t s = qp.s_int;
  const int32_t top = qp.top;
  const std::vector<double>& c = qp.c;
  const bool power = q->flags & CP_Q_PWMETHOD;

  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  void* rA = w + W.rA;
  void* rB = w + W.rB;
  void* yacc = w + W.yacc;
  const bool timing = q->flags & CP_Q_TIMING;
  const bool stats = q->flags & CP_Q_STATS;
  std::vector<hipEvent_t> ev;
  auto cleanup = [&] {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  };
  if (timing) {
    ev.resize(2 + 2 * (size_t)std::max(top - 1, 0));
    for (auto& e : ev) {
      hipError_t he = hipEventCreate(&e);
      if (he != hipSuccess) { set_hip_error(he); cleanup(); return CP_EHIP; }
    }
  }
#define CP_HIP_C(call)                             \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) {                        \
      set_hip_error(e_);                           \
      cleanup();                                   \
      return CP_EHIP;                              \
    }                                              \
  } while (0)

  if (timing) CP_HIP_C(hipEventRecord(ev[0], st));
  // zero r~ buffers, estimate and hub counters (one contiguous range)
  CP_HIP_C(launch_zero(w, W.hub_partial, st));
  InitArgs ia{g->row_ptr, g->col_idx, s, rA, rB, yacc, c[0], c[1]};
  CP_HIP_C(launch_init(prec, ia, st));
  StepArgs sa{};
  sa.row_ptr = g->row_ptr;
  sa.col_idx = g->col_idx;
  sa.blocks = g->single.blocks;
  sa.hubs = g->single.hubs;
  sa.nblocks = g->single.nblocks;
  sa.nspecial = g->single.nspecial;
  sa.yacc = yacc;
  sa.hub_partial = w + W.hub_partial;
  sa.hub_count = reinterpret_cast<int32_t*>(w + W.hub_count);
  for (int32_t k = 1; k < top; ++k) {
    // x = r~_k, z = r~_{k-1} -> r~_{k+1} (Alg. 1: z <- r~_{k+1})
    sa.x = (k & 1) ? rB : rA;
    sa.z = (k & 1) ? rA : rB;
    sa.c = c[k + 1];
    if (timing) CP_HIP_C(hipEventRecord(ev[2 * k], st));
    if (g->striped) {
      StripeArgs ga{};
      ga.rp = g->s_rp;
      ga.cols = g->s_cols;
      for (int j = 0; j < g->s_count; ++j) ga.col_off[j] = g->s_col_off[j];
      for (int j = 0; j < g->s_count; ++j) ga.base[j] = g->s_base[j];
      ga.packed = g->s_packed;
      ga.nstripes = g->s_count;
      ga.blocks = g->s_blocks;
      ga.ntiles = g->s_ntiles;
      ga.n = g->n;
      ga.x = sa.x;
      ga.partial = w + W.partial;
      CP_HIP_C(launch_stripe_gather(prec, ga, st));
      CombineArgs ca{g->row_ptr, g->n, w + W.partial, g->s_count, sa.z, yacc, sa.c};
      CP_HIP_C(launch_stripe_combine(prec, ca, power ? kStepPower : kStepCheb, st));
    } else {
      CP_HIP_C(launch_step(prec, sa, power ? kStepPower : kStepCheb, st));
    }
    if (timing) CP_HIP_C(hipEventRecord(ev[2 * k + 1], st));
  }
  double* mass = stats ? reinterpret_cast<double*>(w + W.mass) : nullptr;
  FinalArgs fa{g->row_ptr, g->perm, g->n, yacc, y, mass, qp.oexp, qp.oscale};
  CP_HIP_C(launch_finalize(prec, fa, st));
  if (timing) CP_HIP_C(hipEventRecord(ev[1], st));

  if (info) {
    info->K = qp.K;
    info->steps = top - 1;
    info->tail = qp.tail;
    info->tail_bound_l1 = qp.tail * qp.L;
    info->mass = NAN;
    info->elapsed_ms = NAN;
    info->step_ms = NAN;
    info->latency_ms = NAN;
    info->wait_ms = NAN;
    info->pushes = 0;
    info->arcs = (int64_t)(top - 1) * g->nnz;
    info->walks = 0;
    info->walk_steps = 0;
  }
  if (stats || timing) {
    CP_HIP_C(hipStreamSynchronize(st));
    if (info && stats) {
      double m = 0;
      CP_HIP_C(hipMemcpy(&m, mass, sizeof(double), hipMemcpyDeviceToHost));
      info->mass = m;
    }
    if (info && timing) {
      float ms = 0;
      CP_HIP_C(hipEventElapsedTime(&ms, ev[0], ev[1]));
      info->elapsed_ms = ms;
      double sum = 0;
      for (int32_t k = 1; k < top; ++k) {
        CP_HIP_C(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
        sum += ms;
      }
      info->step_ms = sum;
    }
  }
  cleanup();
#undef CP_HIP_C
  return CP_OK;
}

}  // namespace

namespace cp {
namespace {

// Build the plan of `shape` from the graph's host row offsets and make it
// the graph's plan `which` (0 single-source, 1 batched), freeing the plan a
// previous call installed there.  Synchronizes st.
cp_status install_plan(cp_graph* g, int which, const PlanShape& shape, hipStream_t st) {
  const Plan pl = build_plan(g->host_rp.data(), g->n, shape);
  const size_t b_blocks = align256(sizeof(BlockDesc) * std::max<size_t>(pl.blocks.size(), 1));
  const size_t b_hubs = align256(sizeof(HubDesc) * std::max<size_t>(pl.hubs.size(), 1));
  char* m = nullptr;
  hipError_t e = hipMalloc(&m, b_blocks + b_hubs);
  if (e != hipSuccess) {
    set_hip_error(e);
    return e == hipErrorOutOfMemory ? CP_ENOMEM : CP_EHIP;
  }
  DevPlan dp;
  dp.nblocks = (int64_t)pl.blocks.size();
  dp.nspecial = pl.nspecial;
  dp.nlong = pl.nlong;
  dp.nhubs = (int64_t)pl.hubs.size();
  dp.hub_segments = pl.hub_segments;
  dp.shape = pl.shape;
  dp.blocks = reinterpret_cast<BlockDesc*>(m);
  dp.hubs = reinterpret_cast<HubDesc*>(m + b_blocks);
  if (dp.nblocks) e = hipMemcpyAsync(dp.blocks, pl.blocks.data(), sizeof(BlockDesc) * dp.nblocks,
                                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess && dp.nhubs)
    e = hipMemcpyAsync(dp.hubs, pl.hubs.data(), sizeof(HubDesc) * dp.nhubs, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_hip_error(e);
    (void)hipFree(m);
    return CP_EHIP;
  }
  if (g->tuned_plan_mem[which]) (void)hipFree(g->tuned_plan_mem[which]);
  g->tuned_plan_mem[which] = m;
  (which == 0 ? g->single : g->batch) = dp;
  return CP_OK;
}

// Row-split shapes the autotuners try, each against the best so far: long
// cuts first, then hub cut and segment size.
const int64_t kLongCuts[2][5] = {{256, 512, 1024, 2048, 0}, {64, 128, 256, 512, 1024}};

// Time `run` (which reports its device time in ms) for each candidate shape of
// plan `which`, install the fastest, and return it.
template <typename Run>
cp_status tune_shape(cp_graph* g, int which, hipStream_t st, Run&& run, PlanShape* best_out) {
  PlanShape best = (which == 0 ? g->single : g->batch).shape;
  double best_ms = 1e300;
  auto trial = [&](const PlanShape& sh) -> cp_status {
    cp_status rc = install_plan(g, which, sh, st);
    if (rc != CP_OK) return rc;
    double ms = 0;
    for (int rep = 0; rep < 2; ++rep) {  // the first run warms caches
      rc = run(&ms);
      if (rc != CP_OK) return rc;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = sh;
    }
    return CP_OK;
  };
  for (int64_t cut : kLongCuts[which]) {
    if (cut <= 0) continue;
    PlanShape sh = best;
    sh.long_cut = cut;
    cp_status rc = trial(sh);
    if (rc != CP_OK) return rc;
  }
  for (const PlanShape& hs : kHubShapes) {
    PlanShape sh = best;
    sh.hub_cut = hs.hub_cut;
    sh.hub_seg = hs.hub_seg;
    cp_status rc = trial(sh);
    if (rc != CP_OK) return rc;
  }
  cp_status rc = install_plan(g, which, best, st);
  if (rc == CP_OK && best_out) *best_out = best;
  return rc;
}

cp_status power_batch_bw(cp_graph* g, int32_t nq, const cp_query* q, int32_t prec, void* Y, void* ws,
                         size_t ws_bytes, hipStream_t st, cp_info* infos, int32_t bw) {
  std::vector<QueryPlan> P(nq);
  for (int32_t j = 0; j < nq; ++j) {
    cp_status rc = plan_query(g, &q[j], kBatchKCap, &P[j]);
    if (rc != CP_OK) return rc;
  }
  const BatchLayout W = batch_layout(g, nq, prec, bw);
  if (!ws || ws_bytes < W.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return CP_EWORKSPACE;
  // slots in decreasing number of steps (stable), tiles of bw slots
  std::vector<int32_t> order(nq);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P[a].top > P[b].top; });
  std::vector<int32_t> slot_of_query(nq);
  for (int32_t i = 0; i < nq; ++i) slot_of_query[order[i]] = i;
  const int32_t Kmax = P[order[0]].top;
  std::vector<double> coef((size_t)(Kmax + 1) * W.nq_pad, 0.0);
  std::vector<int64_t> src(W.nq_pad, -1);
  std::vector<double> sp = slot_params(W.nq_pad);
  for (int32_t i = 0; i < nq; ++i) {
    const QueryPlan& p = P[order[i]];
    for (int32_t k = 0; k <= p.top; ++k) coef[(size_t)k * W.nq_pad + i] = p.c[k];
    src[i] = p.s_int;
    sp[i] = p.rec;
    sp[(size_t)W.nq_pad + i] = p.oexp;
    sp[2 * (size_t)W.nq_pad + i] = p.oscale;
  }
  std::vector<int32_t> tileK(W.ntiles);
  for (int32_t t = 0; t < W.ntiles; ++t) tileK[t] = P[order[t * bw]].top;

  char* w = static_cast<char*>(ws);
  double* dcoef = reinterpret_cast<double*>(w + W.coef);
  const bool timing = q[0].flags & CP_Q_TIMING;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  auto cleanup = [&] {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
#define CP_HIP_B(call)        \
  do {                        \
    hipError_t e_ = (call);   \
    if (e_ != hipSuccess) {   \
      set_hip_error(e_);      \
      cleanup();              \
      return CP_EHIP;         \
    }                         \
  } while (0)
  if (timing)
    for (auto& e : ev) CP_HIP_B(hipEventCreate(&e));
  if (timing) CP_HIP_B(hipEventRecord(ev[0], st));
  CP_HIP_B(launch_zero(w, W.hub_partial, st));
  CP_HIP_B(launch_upload(dcoef, coef.data(), coef.size() * sizeof(double), st));
  CP_HIP_B(launch_upload(w + W.src, src.data(), src.size() * sizeof(int64_t), st));
  CP_HIP_B(launch_upload(w + W.slotmap, slot_of_query.data(), slot_of_query.size() * sizeof(int32_t), st));
  CP_HIP_B(launch_upload(w + W.rec, sp.data(), sp.size() * sizeof(double), st));
  void* rA = w + W.rA;
  void* rB = w + W.rB;
  BatchInitArgs ia{g->row_ptr, g->col_idx, reinterpret_cast<const int64_t*>(w + W.src), g->n, bw,
                   W.nq_pad, rA, rB, w + W.yacc, dcoef};
  CP_HIP_B(launch_batch_init(prec, ia, nq, st));
  BatchStepArgs sa{};
  set_batch_plan(g, sa, w + W.part);
  sa.n = g->n;
  sa.bw = bw;
  sa.nq_pad = W.nq_pad;
  sa.yacc = w + W.yacc;
  sa.rec = reinterpret_cast<const double*>(w + W.rec);
  sa.hub_partial = w + W.hub_partial;
  sa.hub_count = reinterpret_cast<int32_t*>(w + W.hub_count);
  sa.ntiles_total = W.ntiles;
  if (timing) CP_HIP_B(hipEventRecord(ev[1], st));
  for (int32_t k = 1; k < Kmax; ++k) {
    int32_t active = 0;
    while (active < W.ntiles && tileK[active] > k) ++active;
    if (active == 0) break;
    sa.ntiles = active;
    sa.x = (k & 1) ? rB : rA;
    sa.z = (k & 1) ? rA : rB;
    sa.coef_row = dcoef + (size_t)(k + 1) * W.nq_pad;
    CP_HIP_B(launch_batch_step(prec, sa, st));
  }
  if (timing) CP_HIP_B(hipEventRecord(ev[2], st));
  const double* dsp = reinterpret_cast<const double*>(w + W.rec);
  BatchFinalArgs fa{g->row_ptr, g->perm, reinterpret_cast<const int32_t*>(w + W.slotmap), g->n, bw, nq,
                    w + W.yacc, Y, dsp + W.nq_pad, dsp + 2 * (size_t)W.nq_pad};
  CP_HIP_B(launch_batch_finalize(prec, fa, st));
  if (timing) CP_HIP_B(hipEventRecord(ev[3], st));
  float ms_all = NAN, ms_steps = NAN;
  if (timing) {
    CP_HIP_B(hipStreamSynchronize(st));
    CP_HIP_B(hipEventElapsedTime(&ms_all, ev[0], ev[3]));
    CP_HIP_B(hipEventElapsedTime(&ms_steps, ev[1], ev[2]));
  }
  if (infos)
    for (int32_t j = 0; j < nq; ++j) {
      infos[j].K = P[j].K;
      infos[j].steps = P[j].top - 1;
      infos[j].tail = P[j].tail;
      infos[j].tail_bound_l1 = P[j].tail * P[j].L;
      infos[j].mass = NAN;
      infos[j].elapsed_ms = ms_all;
      infos[j].step_ms = ms_steps;
      infos[j].latency_ms = NAN;
      infos[j].wait_ms = NAN;
      infos[j].pushes = 0;
      infos[j].arcs = (int64_t)(P[j].top - 1) * g->nnz;
      infos[j].walks = 0;
      infos[j].walk_steps = 0;
    }
  cleanup();
#undef CP_HIP_B
  return CP_OK;
}

}  // namespace
}  // namespace cp

extern "C" {

cp_status cp_power_batch(const cp_graph* g, int32_t nq, const cp_query* q, int32_t prec, void* Y,
                         void* ws, size_t ws_bytes, void* stream, cp_info* infos) {
  if (!g || nq < 1 || !q || !Y || !valid_prec(prec)) return CP_EINVAL;
  cp_graph* gm = const_cast<cp_graph*>(g);  // only the tuning cache is mutable
  const int32_t bw = choose_bw(gm, nq, prec);
  if (ws_bytes < batch_ws_bytes(g, nq, prec)) return CP_EWORKSPACE;
  return power_batch_bw(gm, nq, q, prec, Y, ws, ws_bytes, static_cast<hipStream_t>(stream), infos, bw);
}

cp_status cp_propagate(const cp_graph* g, const cp_query* q, int32_t k, int32_t prec, const void* X, void* Z,
                       void* ws, size_t ws_bytes, void* stream, cp_info* info) {
  if (!g || !q || k < 1 || !X || !Z || !valid_prec(prec)) return CP_EINVAL;
  if (q->kind != CP_PPR && q->kind != CP_HKPR) return CP_EINVAL;
  if (q->flags & ~(CP_Q_TIMING | CP_Q_PWMETHOD | CP_Q_CLENSHAW)) return CP_EINVAL;
  const bool clenshaw = q->flags & CP_Q_CLENSHAW;
  if (clenshaw && (q->flags & CP_Q_PWMETHOD)) return CP_EINVAL;
  if (!(q->a >= 0.0 && q->a <= 1.0)) return CP_EINVAL;
  if (q->kmode == CP_K_CERTIFIED) return CP_EINVAL;  // the certified rule needs norms of X
  const bool power = q->flags & CP_Q_PWMETHOD;
  int32_t K = 0, top = 0;
  double tail = 0;
  std::vector<double> c;
  cp_status rc;
  if (power) {
    rc = choose_N_impl(q->kind, q->param, q->tol, q->kmode, q->K_fixed, kBatchKCap + 1, &K, &tail);
    if (rc != CP_OK) return rc;
    top = std::max(K - 1, 1);
    c.assign((size_t)top + 1, 0.0);
    rc = taylor_impl(q->kind, q->param, K, c.data());
  } else {
    rc = choose_K_impl(q->kind, q->param, q->tol, q->kmode, q->K_fixed, (double)g->nnz, 1.0, kBatchKCap, &K,
                       &tail);
    if (rc != CP_OK) return rc;
    top = K;
    c.assign((size_t)K + 1, 0.0);
    rc = coeffs_impl(q->kind, q->param, K, c.data());
  }
  if (rc != CP_OK) return rc;
  cp_graph* gm = const_cast<cp_graph*>(g);  // only the tuning cache is mutable
  const int32_t bw = choose_bw(gm, k, prec);
  if (!ws || ws_bytes < batch_ws_bytes(g, k, prec) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return CP_EWORKSPACE;
  const BatchLayout W = batch_layout(g, k, prec, bw);
  const size_t np = (size_t)W.nq_pad;
  std::vector<double> coef((size_t)(top + 1) * np, 0.0);
  for (int32_t kk = 0; kk <= top; ++kk)
    for (int32_t j = 0; j < k; ++j) coef[kk * np + j] = c[kk];
  std::vector<double> sp = slot_params(W.nq_pad);
  for (int32_t j = 0; j < k; ++j) {
    sp[j] = power ? 1.0 : 2.0;
    sp[np + j] = 1.0 - q->a;
  }
  std::vector<int32_t> slotmap(k);
  std::iota(slotmap.begin(), slotmap.end(), 0);

  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  double* dcoef = reinterpret_cast<double*>(w + W.coef);
  const double* dsp = reinterpret_cast<const double*>(w + W.rec);
  const bool timing = q->flags & CP_Q_TIMING;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  auto cleanup = [&] {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
#define CP_HIP_P(call)        \
  do {                        \
    hipError_t e_ = (call);   \
    if (e_ != hipSuccess) {   \
      set_hip_error(e_);      \
      cleanup();              \
      return CP_EHIP;         \
    }                         \
  } while (0)
  if (timing)
    for (auto& e : ev) CP_HIP_P(hipEventCreate(&e));
  if (timing) CP_HIP_P(hipEventRecord(ev[0], st));
  CP_HIP_P(launch_zero(w, W.hub_partial, st));
  CP_HIP_P(launch_upload(dcoef, coef.data(), coef.size() * sizeof(double), st));
  CP_HIP_P(launch_upload(w + W.slotmap, slotmap.data(), slotmap.size() * sizeof(int32_t), st));
  CP_HIP_P(launch_upload(w + W.rec, sp.data(), sp.size() * sizeof(double), st));
  void* rA = w + W.rA;
  void* rB = w + W.rB;
  DenseInitArgs ia{g->row_ptr, g->perm, g->n, bw, k, X, q->a, clenshaw ? c[K] : 1.0, clenshaw ? 1.0 : c[0], rA,
                   w + W.yacc};
  CP_HIP_P(launch_dense_init(prec, ia, st));
  BatchStepArgs sa{};
  set_batch_plan(g, sa, w + W.part);
  sa.n = g->n;
  sa.bw = bw;
  sa.nq_pad = W.nq_pad;
  sa.ntiles = W.ntiles;
  sa.yacc = w + W.yacc;
  sa.hub_partial = w + W.hub_partial;
  sa.hub_count = reinterpret_cast<int32_t*>(w + W.hub_count);
  sa.ntiles_total = W.ntiles;
  if (timing) CP_HIP_P(hipEventRecord(ev[1], st));
  if (clenshaw) {
    // b~_K = c_K x~ in rA, b~_{K+1} = 0 in rB; b~_k for k = K-1 .. 1 over
    // the older buffer, then c_0 x~ + D^{-1} P b_1 - b~_2 into yacc
    void* cur = rA;   // b~_{k+1}
    void* prev = rB;  // b~_{k+2}
    sa.mode = kClenshawStep;
    sa.rec = dsp;
    for (int32_t kk = K - 1; kk >= 1; --kk) {
      sa.x = cur;
      sa.z = prev;
      sa.coef_row = dcoef + (size_t)kk * np;
      CP_HIP_P(launch_batch_step(prec, sa, st));
      std::swap(cur, prev);
    }
    sa.mode = kClenshawLast;
    sa.rec = dsp + 3 * np;
    sa.x = cur;
    sa.z = prev;
    sa.coef_row = dcoef;
    CP_HIP_P(launch_batch_step(prec, sa, st));
  } else {
    // r~_1 = D^{-1} P r_0: a power step from r~_0 into the zeroed second buffer
    sa.x = rA;
    sa.z = rB;
    sa.coef_row = dcoef + np;
    sa.rec = dsp + 3 * np;
    CP_HIP_P(launch_batch_step(prec, sa, st));
    sa.rec = dsp;
    for (int32_t kk = 1; kk < top; ++kk) {
      sa.x = (kk & 1) ? rB : rA;
      sa.z = (kk & 1) ? rA : rB;
      sa.coef_row = dcoef + (size_t)(kk + 1) * np;
      CP_HIP_P(launch_batch_step(prec, sa, st));
    }
  }
  if (timing) CP_HIP_P(hipEventRecord(ev[2], st));
  BatchFinalArgs fa{g->row_ptr, g->perm, reinterpret_cast<const int32_t*>(w + W.slotmap), g->n, bw, k,
                    w + W.yacc, Z, dsp + np, dsp + 2 * np};
  CP_HIP_P(launch_batch_finalize(prec, fa, st));
  if (timing) CP_HIP_P(hipEventRecord(ev[3], st));
  float ms_all = NAN, ms_steps = NAN;
  if (timing) {
    CP_HIP_P(hipStreamSynchronize(st));
    CP_HIP_P(hipEventElapsedTime(&ms_all, ev[0], ev[3]));
    CP_HIP_P(hipEventElapsedTime(&ms_steps, ev[1], ev[2]));
  }
  if (info) {
    info->K = K;
    info->steps = top;
    info->tail = tail;
    info->tail_bound_l1 = NAN;
    info->mass = NAN;
    info->elapsed_ms = ms_all;
    info->step_ms = ms_steps;
    info->latency_ms = NAN;
    info->wait_ms = NAN;
    info->pushes = 0;
    info->arcs = (int64_t)top * g->nnz;
    info->walks = 0;
    info->walk_steps = 0;
  }
  cleanup();
#undef CP_HIP_P
  return CP_OK;
}

cp_status cp_set_batch_width(cp_graph* g, int32_t nq, int32_t prec, int32_t bw) {
  if (!g || nq < 1 || !valid_prec(prec)) return CP_EINVAL;
  std::lock_guard<std::mutex> lk(g->tune_mu);
  if (bw == 0) {
    g->tuned_bw.erase(tune_key(nq, prec));
    return CP_OK;
  }
  if (!(bw == 8 || bw == 16 || bw == 32 || bw == 64) || !width_allowed(nq, bw)) return CP_EINVAL;
  g->tuned_bw[tune_key(nq, prec)] = bw;
  return CP_OK;
}

cp_status cp_autotune_batch(cp_graph* g, int32_t nq, const cp_query* q, int32_t prec, void* Y, void* ws,
                            size_t ws_bytes, void* stream, int32_t* bw_out) {
  if (!g || nq < 1 || !q || !Y || !valid_prec(prec)) return CP_EINVAL;
  if (ws_bytes < batch_ws_bytes(g, nq, prec)) return CP_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<cp_query> qq(q, q + nq);
  for (auto& x : qq) x.flags = CP_Q_TIMING;
  std::vector<cp_info> infos(nq);
  int32_t best = 0;
  double best_ms = 1e300;
  for (int32_t bw : kBatchWidths) {
    if (!width_allowed(nq, bw)) continue;
    double ms = 1e300;
    for (int rep = 0; rep < 2; ++rep) {  // first run warms caches and code objects
      cp_status rc = power_batch_bw(g, nq, qq.data(), prec, Y, ws, ws_bytes, st, infos.data(), bw);
      if (rc != CP_OK) return rc;
      ms = infos[0].elapsed_ms;
    }
    if (ms < best_ms) { best_ms = ms; best = bw; }
  }
  {
    std::lock_guard<std::mutex> lk(g->tune_mu);
    g->tuned_bw[tune_key(nq, prec)] = best;
  }
  // the batched plan's row splits at that width (the hot/cold split keeps its own plans)
  if (!g->hot_split) {
    auto run = [&](double* ms) {
      cp_status rc = power_batch_bw(g, nq, qq.data(), prec, Y, ws, ws_bytes, st, infos.data(), best);
      *ms = infos[0].step_ms;
      return rc;
    };
    cp_status rc = tune_shape(g, 1, st, run, nullptr);
    if (rc != CP_OK) return rc;
  }
  if (bw_out) *bw_out = best;
  return CP_OK;
}

cp_status cp_autotune_single(cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!g || !q || !y || !valid_prec(prec)) return CP_EINVAL;
  if (g->striped) return CP_OK;  // striped steps run fixed stripe tiles, not the plan
  hipStream_t st = static_cast<hipStream_t>(stream);
  cp_query qq = *q;
  qq.flags = (q->flags & CP_Q_PWMETHOD) | CP_Q_TIMING;
  auto run = [&](double* ms) {
    cp_info info{};
    cp_status rc = cp_power(g, &qq, prec, y, ws, ws_bytes, stream, &info);
    *ms = info.step_ms;
    return rc;
  };
  return tune_shape(g, 0, st, run, nullptr);
}

}  // extern "C"
