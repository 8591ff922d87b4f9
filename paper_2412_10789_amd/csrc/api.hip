// C ABI of the ChebyPower library: graph objects, workspaces and queries.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
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

size_t storage_bytes(int32_t prec) { return prec == CP_F64 ? 8 : prec == CP_F32 ? 4 : 2; }
size_t acc_bytes(int32_t prec) { return prec == CP_F64 ? 8 : 4; }
bool valid_prec(int32_t prec) { return prec == CP_F64 || prec == CP_F32 || prec == CP_BF16; }

int host_threads() {
  unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h ? h : 1u, 16u));
}

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

Plan build_plan(const int64_t* rp, int64_t n) {
  Plan p;
  std::vector<int32_t> hubs, longs;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = rp[v + 1] - rp[v];
    if (d > kHubThreshold) hubs.push_back((int32_t)v);
    else if (d > kTileNnz) longs.push_back((int32_t)v);
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
    const int32_t nseg = (int32_t)((d + kHubSeg - 1) / kHubSeg);
    p.hubs.push_back(HubDesc{hubs[h], nseg, base, 0});
    for (int32_t s = 0; s < nseg; ++s) p.blocks.push_back(BlockDesc{hubs[h], (int32_t)h, kHub, s});
    base += nseg;
  }
  p.hub_segments = base;
  for (int32_t v : longs) p.blocks.push_back(BlockDesc{v, v + 1, kLong, 0});
  p.nlong = (int64_t)longs.size();
  p.nspecial = (int64_t)p.blocks.size();
  // greedy stream tiles over the remaining rows, in row order
  int64_t r0 = -1, nnz = 0;
  auto close = [&](int64_t r1) {
    if (r0 >= 0) p.blocks.push_back(BlockDesc{(int32_t)r0, (int32_t)r1, kStream, 0});
    r0 = -1;
    nnz = 0;
  };
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = rp[v + 1] - rp[v];
    if (d > kTileNnz) { close(v); continue; }
    if (r0 >= 0 && (nnz + d > kTileNnz || v - r0 == kTileRows)) close(v);
    if (r0 < 0) r0 = v;
    nnz += d;
  }
  close(n);
  return p;
}

namespace {

struct WsLayout {
  size_t rA, rB, yacc, hub_count, hub_partial, mass, total;
};

WsLayout ws_layout(const cp_graph* g, int32_t nq, int32_t prec) {
  WsLayout L{};
  const size_t vec = align256((size_t)g->n * (size_t)nq * storage_bytes(prec));
  const size_t yv = align256((size_t)g->n * (size_t)nq * acc_bytes(prec));
  size_t off = 0;
  L.rA = off; off += vec;
  L.rB = off; off += vec;
  L.yacc = off; off += yv;
  L.hub_count = off; off += align256((size_t)std::max<int64_t>(g->nhubs, 1) * 4);
  L.hub_partial = off; off += align256((size_t)std::max<int64_t>(g->hub_segments, 1) * 8 * nq);
  L.mass = off; off += align256((1 + 1024) * 8);
  L.total = off;
  return L;
}

cp_status check_query(const cp_graph* g, const cp_query* q, int64_t* s_int, int32_t* K,
                      double* tail, double* L) {
  if (!q) return CP_EINVAL;
  if (q->kind != CP_PPR && q->kind != CP_HKPR) return CP_EINVAL;
  if (q->source < 0 || q->source >= g->n) return CP_ESOURCE;
  const int32_t ds = g->degree[q->source];
  if (ds == 0) return CP_EISOLATED;
  *s_int = g->reordered ? g->ext2int[q->source] : q->source;
  *L = std::sqrt((double)g->nnz / (double)ds);
  return choose_K_impl(q->kind, q->param, q->tol, q->kmode, q->K_fixed, (double)g->nnz, (double)ds,
                       kDefaultKMax, K, tail);
}

}  // namespace
}  // namespace cp

using namespace cp;

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

cp_status cp_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          int32_t flags, void* stream, cp_graph** out) {
  if (!out || !row_ptr || n < 1 || n >= INT32_MAX || nnz < 0 || (nnz > 0 && !col_idx))
    return CP_EINVAL;
  *out = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool host_in = flags & CP_GRAPH_HOST;
  const bool reorder = flags & CP_GRAPH_REORDER;
  const bool borrow = (flags & CP_GRAPH_BORROW) && !host_in && !reorder;
  cp_graph* g = nullptr;
  try {
    g = new cp_graph();
    g->n = n;
    g->nnz = nnz;
    CP_HIP(hipGetDevice(&g->device));
    // host copies of the CSR (row offsets always; columns when needed)
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> ci;
    const bool need_cols = (flags & CP_GRAPH_VALIDATE) || reorder || host_in;
    if (host_in) {
      std::memcpy(rp.data(), row_ptr, sizeof(int64_t) * (n + 1));
    } else {
      CP_HIP(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
    }
    if (need_cols) {
      ci.resize(nnz);
      if (host_in) std::memcpy(ci.data(), col_idx, sizeof(int32_t) * nnz);
      else if (nnz)
        CP_HIP(hipMemcpyAsync(ci.data(), col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
    }
    CP_HIP(hipStreamSynchronize(st));
    if (rp[0] != 0 || rp[n] != nnz) { delete g; return CP_EINVAL; }
    if ((flags & CP_GRAPH_VALIDATE) && !validate_csr(n, nnz, rp.data(), ci.data())) {
      delete g;
      return CP_EGRAPH;
    }
    g->degree.resize(n);
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = rp[v + 1] - rp[v];
      g->degree[v] = (int32_t)d;
      g->d_max = std::max(g->d_max, d);
    }
    // internal order
    std::vector<int32_t> perm;  // internal -> caller
    if (reorder) {
      perm.resize(n);
      std::iota(perm.begin(), perm.end(), 0);
      std::stable_sort(perm.begin(), perm.end(),
                       [&](int32_t a, int32_t b) { return g->degree[a] > g->degree[b]; });
      g->ext2int.resize(n);
      for (int64_t i = 0; i < n; ++i) g->ext2int[perm[i]] = (int32_t)i;
      std::vector<int64_t> rp2(n + 1, 0);
      for (int64_t i = 0; i < n; ++i) rp2[i + 1] = rp2[i] + g->degree[perm[i]];
      std::vector<int32_t> ci2(nnz);
      parallel_rows(n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
          const int32_t v = perm[i];
          int32_t* dst = ci2.data() + rp2[i];
          for (int64_t q = rp[v]; q < rp[v + 1]; ++q) *dst++ = g->ext2int[ci[q]];
          std::sort(ci2.data() + rp2[i], dst);
        }
      });
      rp.swap(rp2);
      ci.swap(ci2);
      g->reordered = true;
    }
    const Plan plan = build_plan(rp.data(), n);
    g->nblocks = (int64_t)plan.blocks.size();
    g->nspecial = plan.nspecial;
    g->nlong = plan.nlong;
    g->nhubs = (int64_t)plan.hubs.size();
    g->hub_segments = plan.hub_segments;

    // device copies: [row_ptr | col_idx | perm | blocks | hubs] in one allocation
    const size_t b_rp = borrow ? 0 : align256(sizeof(int64_t) * (n + 1));
    const size_t b_ci = borrow ? 0 : align256(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    const size_t b_pm = reorder ? align256(sizeof(int32_t) * n) : 0;
    const size_t b_bl = align256(sizeof(BlockDesc) * std::max<int64_t>(g->nblocks, 1));
    const size_t b_hb = align256(sizeof(HubDesc) * std::max<int64_t>(g->nhubs, 1));
    const size_t total = b_rp + b_ci + b_pm + b_bl + b_hb;
    char* base = nullptr;
    hipError_t e = hipMalloc(&base, total);
    if (e != hipSuccess) {
      delete g;
      return e == hipErrorOutOfMemory ? CP_ENOMEM : (set_hip_error(e), CP_EHIP);
    }
    g->owned_csr = base;
    g->device_bytes = (int64_t)total;
    char* p = base;
    if (borrow) {
      g->row_ptr = row_ptr;
      g->col_idx = col_idx;
      g->borrowed = true;
    } else {
      int64_t* drp = reinterpret_cast<int64_t*>(p); p += b_rp;
      int32_t* dci = reinterpret_cast<int32_t*>(p); p += b_ci;
      CP_HIP(hipMemcpyAsync(drp, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
      if (nnz) {
        if (need_cols)
          CP_HIP(hipMemcpyAsync(dci, ci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
        else
          CP_HIP(hipMemcpyAsync(dci, col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st));
      }
      g->row_ptr = drp;
      g->col_idx = dci;
    }
    if (reorder) {
      g->perm = reinterpret_cast<int32_t*>(p); p += b_pm;
      CP_HIP(hipMemcpyAsync(g->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    }
    g->blocks = reinterpret_cast<BlockDesc*>(p); p += b_bl;
    g->hubs = reinterpret_cast<HubDesc*>(p); p += b_hb;
    if (g->nblocks)
      CP_HIP(hipMemcpyAsync(g->blocks, plan.blocks.data(), sizeof(BlockDesc) * g->nblocks,
                            hipMemcpyHostToDevice, st));
    if (g->nhubs)
      CP_HIP(hipMemcpyAsync(g->hubs, plan.hubs.data(), sizeof(HubDesc) * g->nhubs,
                            hipMemcpyHostToDevice, st));
    CP_HIP(hipStreamSynchronize(st));
    *out = g;
    return CP_OK;
  } catch (const std::bad_alloc&) {
    if (g && g->owned_csr) (void)hipFree(g->owned_csr);
    delete g;
    return CP_ENOMEM;
  }
}

cp_status cp_graph_destroy(cp_graph* g) {
  if (!g) return CP_EINVAL;
  if (g->owned_csr) {
    hipError_t e = hipFree(g->owned_csr);
    if (e != hipSuccess) { set_hip_error(e); delete g; return CP_EHIP; }
  }
  delete g;
  return CP_OK;
}

cp_status cp_graph_get_stats(const cp_graph* g, cp_graph_stats* out) {
  if (!g || !out) return CP_EINVAL;
  out->n = g->n;
  out->nnz = g->nnz;
  out->d_max = g->d_max;
  out->blocks = g->nblocks;
  out->long_rows = g->nlong;
  out->hub_rows = g->nhubs;
  out->device_bytes = g->device_bytes;
  out->reordered = g->reordered;
  out->borrowed = g->borrowed;
  return CP_OK;
}

size_t cp_workspace_bytes(const cp_graph* g, int32_t nq, int32_t prec) {
  if (!g || nq < 1 || !valid_prec(prec)) return 0;
  return ws_layout(g, nq, prec).total;
}

cp_status cp_power(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws,
                   size_t ws_bytes, void* stream, cp_info* info) {
  if (!g || !q || !y || !valid_prec(prec)) return CP_EINVAL;
  int64_t s = 0;
  int32_t K = 0;
  double tail = 0, L = 1;
  cp_status rc = check_query(g, q, &s, &K, &tail, &L);
  if (rc != CP_OK) return rc;
  const WsLayout W = ws_layout(g, 1, prec);
  if (!ws || ws_bytes < W.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return CP_EWORKSPACE;
  std::vector<double> c(K + 1);
  rc = coeffs_impl(q->kind, q->param, K, c.data());
  if (rc != CP_OK) return rc;

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
    ev.resize(2 + 2 * (size_t)std::max(K - 1, 0));
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
  sa.blocks = g->blocks;
  sa.hubs = g->hubs;
  sa.nblocks = g->nblocks;
  sa.nspecial = g->nspecial;
  sa.yacc = yacc;
  sa.hub_partial = w + W.hub_partial;
  sa.hub_count = reinterpret_cast<int32_t*>(w + W.hub_count);
  for (int32_t k = 1; k < K; ++k) {
    // x = r~_k, z = r~_{k-1} -> r~_{k+1}
    sa.x = (k & 1) ? rB : rA;
    sa.z = (k & 1) ? rA : rB;
    sa.c = c[k + 1];
    if (timing) CP_HIP_C(hipEventRecord(ev[2 * k], st));
    CP_HIP_C(launch_step(prec, sa, st));
    if (timing) CP_HIP_C(hipEventRecord(ev[2 * k + 1], st));
  }
  double* mass = stats ? reinterpret_cast<double*>(w + W.mass) : nullptr;
  FinalArgs fa{g->row_ptr, g->perm, g->n, yacc, y, mass};
  CP_HIP_C(launch_finalize(prec, fa, st));
  if (timing) CP_HIP_C(hipEventRecord(ev[1], st));

  if (info) {
    info->K = K;
    info->steps = K - 1;
    info->tail = tail;
    info->tail_bound_l1 = tail * L;
    info->mass = NAN;
    info->elapsed_ms = NAN;
    info->step_ms = NAN;
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
      for (int32_t k = 1; k < K; ++k) {
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

cp_status cp_power_batch(const cp_graph* g, int32_t nq, const cp_query* q, int32_t prec, void* Y,
                         void* ws, size_t ws_bytes, void* stream, cp_info* infos) {
  (void)g; (void)nq; (void)q; (void)prec; (void)Y; (void)ws; (void)ws_bytes; (void)stream; (void)infos;
  return CP_EINVAL;
}

}  // extern "C"
