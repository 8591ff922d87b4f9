// Batched ChebyPower kernels: Alg. 3 for many sources at once.
//
// The recurrence vectors of bw sources form a tile-major matrix [n][bw]
// (D^{-1} basis, as in the single-source kernels), so for every arc u -> v
// one gather reads the bw contiguous values x[u][0..bw) and all bw
// sources share one pass over the column ids.  A workgroup of 256 threads
// splits into 256/bw lane groups; each lane owns one source of the tile.
// Each source carries its own coefficient row, so sources with different
// truncation steps share the launches (a finished source gets c = 0).

#include <hip/hip_runtime.h>

#include "common.h"

namespace cp {
namespace {

struct bf16 {
  uint16_t bits;
};
struct f32f {  // CP_F32F storage: a float whose arithmetic stays in float
  float v;
};

template <typename T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = double; };  // FP32 storage, FP64 arithmetic
template <> struct Acc<f32f> { using type = float; };    // FP32 storage, FP32 arithmetic

template <typename T> struct Out { using type = float; };  // result type handed to the caller
template <> struct Out<double> { using type = double; };
template <> struct Acc<bf16> { using type = float; };

__device__ __forceinline__ double to_acc(double v) { return v; }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ float to_acc(f32f v) { return v.v; }
__device__ __forceinline__ float to_acc(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }

template <typename T> __device__ __forceinline__ T from_acc(typename Acc<T>::type v);
template <> __device__ __forceinline__ double from_acc<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_acc<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ f32f from_acc<f32f>(float v) { return f32f{v}; }
template <> __device__ __forceinline__ bf16 from_acc<bf16>(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}

template <typename T> __device__ __forceinline__ T ld_nt(const T* p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ bf16 ld_nt<bf16>(const bf16* p) {
  return bf16{__builtin_nontemporal_load(&p->bits)};
}
template <> __device__ __forceinline__ f32f ld_nt<f32f>(const f32f* p) {
  return f32f{__builtin_nontemporal_load(&p->v)};
}
template <typename T> __device__ __forceinline__ void st_nt(T* p, T v) { __builtin_nontemporal_store(v, p); }
template <> __device__ __forceinline__ void st_nt<bf16>(bf16* p, bf16 v) {
  __builtin_nontemporal_store(v.bits, &p->bits);
}
template <> __device__ __forceinline__ void st_nt<f32f>(f32f* p, f32f v) {
  __builtin_nontemporal_store(v.v, &p->v);
}

__device__ __forceinline__ int64_t logical_block(int64_t w, int64_t nblocks, int64_t nspecial) {
  if (w < nspecial) return w;
  const int64_t m = nblocks - nspecial, i = w - nspecial;
  const int64_t q = m >> 3, r = m & 7, x = i & 7, j = i >> 3;
  return nspecial + x * q + (x < r ? x : r) + j;
}

// Forward: zn = u acc / d - (u - 1) z, u = 2 the Chebyshev step (Eq. 6),
// u = 1 the power step of Alg. 1 (the old value is read but weighted by
// zero), then y += c zn.  Clenshaw (y holds x~): bn = c x~ + u acc / d - z,
// written over z (a step) or over y (the last one).
template <typename T, typename A>
__device__ __forceinline__ void row_update(T* z, A* y, size_t e, A acc, int32_t d, A c, A u, int32_t mode) {
  if (mode == kBatchForward) {
    const A zn = (u * acc) / A(d) - (u - A(1)) * to_acc(ld_nt(z + e));
    st_nt(z + e, from_acc<T>(zn));
    st_nt(y + e, ld_nt(y + e) + c * zn);
    return;
  }
  const A bn = c * ld_nt(y + e) + (u * acc) / A(d) - to_acc(ld_nt(z + e));
  if (mode == kClenshawStep) st_nt(z + e, from_acc<T>(bn));
  else st_nt(y + e, bn);
}

// Gathers in flight per lane: a lane issues U gathers (then 4, then 1)
// before it adds any of them; U = 16 in the DEEP form of the step kernel,
// else 4 (8 in stream rows of 64-wide tiles).  A wavefront holds 64 / bw
// lane groups, so with 4 gathers a lane a wavefront has 32 rows in flight
// at bw = 8 but only 8 at bw = 32.  The
// launcher takes the DEEP form for tiles of 32 or more sources on graphs
// whose stream tiles average fewer than 64 rows (more than 32 arcs a row,
// enough to fill 16-deep chunks): 3% faster a launch on an Orkut-sized
// degree-ordered graph (78 arcs a row), while on a LiveJournal-sized one
// (17.5 arcs a row) the 16-deep form was 5% slower, its larger register
// footprint costing a wavefront per SIMD.  At bw = 8 on a Friendster-sized
// graph it was 1% slower.
constexpr int kDeepGathers = 16;
constexpr int kDeepRowsPerTile = 64;

// Running sum of a long chain of terms.  A float chain uses Kahan's
// compensated summation (Kahan, 1965), so its rounding does not grow with
// the chain's length (a lane group's share of a hub segment is hundreds of
// terms); double chains are plain sums.
template <typename A> struct ChainSum {
  A s = A(0);
  __device__ __forceinline__ void add(A v) { s += v; }
  __device__ __forceinline__ A value() const { return s; }
};
template <> struct ChainSum<float> {
  float s = 0.0f, c = 0.0f;  // c: what the last add lost, with its sign
  __device__ __forceinline__ void add(float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ float value() const { return s - c; }
};

// Pairwise sum of v[0..U) (a fixed order).
template <typename A, int U>
__device__ __forceinline__ A tree_sum(const A* v) {
  if constexpr (U == 1) {
    return v[0];
  } else {
    return tree_sum<A, U / 2>(v) + tree_sum<A, U / 2>(v + U / 2);
  }
}

// Sum over arcs [p0, p1) of x[col[p]][lane]; the workgroup's lane groups
// take interleaved arcs, partial sums are combined in group order.
// Result valid in group 0.
template <typename T, typename A, int BW, int NL, bool DEEP>
__device__ __forceinline__ A wg_row_sum(const int32_t* __restrict__ col, const T* __restrict__ x,
                                        int64_t p0, int64_t p1, int grp, int lane, A (*part)[NL]) {
  constexpr int G = kThreads / NL;
  constexpr int U = DEEP ? kDeepGathers : 4;
  ChainSum<A> chain;
  int64_t p = p0 + grp;
  if constexpr (U > 4) {
    for (; p + (U - 1) * G < p1; p += U * G) {
      A v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) v[q] = to_acc(x[(size_t)col[p + q * G] * BW + lane]);
      chain.add(tree_sum<A, U>(v));
    }
  }
  for (; p + 3 * G < p1; p += 4 * G) {
    A v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = to_acc(x[(size_t)col[p + q * G] * BW + lane]);
    chain.add(tree_sum<A, 4>(v));
  }
  for (; p < p1; p += G) chain.add(to_acc(x[(size_t)col[p] * BW + lane]));
  part[grp][lane] = chain.value();
  __syncthreads();
  A total = A(0);
  if (grp == 0) {
    for (int g = 0; g < G; ++g) total += part[g][lane];
  }
  return total;
}

// NL: lanes per group, one per slot the launch updates; NL = BW except in a
// narrow launch (8 or 16 lanes over rows BW apart).
template <typename T, int BW, bool DEEP, int NL = BW>
__global__ void __launch_bounds__(kThreads) batch_step_kernel(BatchStepArgs a) {
  using A = typename Acc<T>::type;
  constexpr int G = kThreads / NL;
  __shared__ int32_t cols[kTileNnz];
  __shared__ int32_t rpl[kTileRows + 1];
  __shared__ int32_t dgl[kTileRows];
  __shared__ A part[G][NL];
  __shared__ int32_t last_flag;

  const int tid = threadIdx.x, grp = tid / NL, lane = tid % NL;
  const int tile = blockIdx.y;
  const size_t toff = (size_t)tile * (size_t)a.n * BW;
  const T* __restrict__ x = static_cast<const T*>(a.x) + toff;
  T* __restrict__ z = static_cast<T*>(a.z) + toff;
  A* __restrict__ y = static_cast<A*>(a.yacc) + toff;
  // split step: the hot pass writes its row sums here, the cold pass starts from them
  A* __restrict__ hp_row = a.part ? static_cast<A*>(a.part) + toff : nullptr;
  const bool hot = a.mode == kBatchHot;
  const A c = (A)a.coef_row[tile * BW + lane];
  const A u = (A)a.rec[tile * BW + lane];
  const int64_t* __restrict__ rp = a.row_ptr;
  const int64_t* __restrict__ drp = a.deg_rp ? a.deg_rp : a.row_ptr;
  const int32_t* __restrict__ col = a.col_idx;
  const int64_t b = logical_block(blockIdx.x, a.nblocks, a.nspecial);
  const BlockDesc bd = a.blocks[b];

  // the end of a row: the hot pass stores the sum; otherwise the partial of
  // the hot pass (if any) is added and the row update applied with the full degree
  auto finish_row = [&](int64_t v, A acc, int32_t d) {
    const size_t e = (size_t)v * BW + lane;
    if (hot) {
      st_nt(hp_row + e, acc);
      return;
    }
    if (hp_row) acc += ld_nt(hp_row + e);
    if (d > 0) row_update<T, A>(z, y, e, acc, d, c, u, a.mode);
  };

  if (bd.kind == kStream) {
    const int32_t r0 = bd.r0, nr = bd.r1 - bd.r0;
    const int64_t p0 = bd.p0;
    const int32_t cnt = bd.aux;
    for (int i = tid; i < cnt; i += kThreads) cols[i] = ld_nt(col + p0 + i);
    for (int j = tid; j <= nr; j += kThreads) rpl[j] = (int32_t)(rp[r0 + j] - p0);
    if (a.deg_rp)
      for (int j = tid; j < nr; j += kThreads) dgl[j] = (int32_t)(drp[r0 + j + 1] - drp[r0 + j]);
    __syncthreads();
    // the groups own consecutive row ranges of about equal work, counting a
    // row's arcs plus one for the row itself (in a split step every row is
    // finished, also those without arcs of this pass): group g takes the
    // rows j whose rpl[j] + j falls in [g tot / G, (g + 1) tot / G)
    const int tot = cnt + nr;
    auto first_row_at = [&](int target) {  // smallest j with rpl[j] + j >= target
      int lo = 0, hi = nr;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rpl[mid] + mid >= target) hi = mid; else lo = mid + 1;
      }
      return lo;
    };
    const int rlo = grp == 0 ? 0 : first_row_at((grp * tot + G - 1) / G);
    const int rhi = grp == G - 1 ? nr : first_row_at(((grp + 1) * tot + G - 1) / G);
    for (int r = rlo; r < rhi; ++r) {
      const int pb = rpl[r], pe = rpl[r + 1];
      if (pe == pb && !hp_row) continue;
      A acc = A(0);
      int p = pb;
      // shallow form with one lane group per wavefront (bw 64): chunks of 8
      constexpr int U = DEEP ? kDeepGathers : NL >= 64 ? 8 : 4;
      if constexpr (U > 4) {
        for (; p + U <= pe; p += U) {
          A v[U];
#pragma unroll
          for (int q = 0; q < U; ++q) v[q] = to_acc(x[(size_t)cols[p + q] * BW + lane]);
          acc += tree_sum<A, U>(v);
        }
      }
      for (; p + 4 <= pe; p += 4) {
        A v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = to_acc(x[(size_t)cols[p + q] * BW + lane]);
        acc += tree_sum<A, 4>(v);
      }
      for (; p < pe; ++p) acc += to_acc(x[(size_t)cols[p] * BW + lane]);
      finish_row(r0 + r, acc, a.deg_rp ? dgl[r] : pe - pb);
    }
    return;
  }

  if (bd.kind == kLong) {
    const int64_t v = bd.r0;
    const int64_t p0 = rp[v], p1 = rp[v + 1];
    const A total = wg_row_sum<T, A, BW, NL, DEEP>(col, x, p0, p1, grp, lane, part);
    if (grp == 0) finish_row(v, total, (int32_t)(drp[v + 1] - drp[v]));
    return;
  }

  // hub segment: partial per (segment, slot); last workgroup of (hub, tile) combines
  const HubDesc h = a.hubs[bd.r1];
  const int64_t rb = rp[h.row], re = rp[h.row + 1];
  const int64_t p0 = rb + (int64_t)bd.aux * h.seg;
  const int64_t p1 = p0 + h.seg < re ? p0 + h.seg : re;
  const A total = wg_row_sum<T, A, BW, NL, DEEP>(col, x, p0, p1, grp, lane, part);
  A* hp = static_cast<A*>(a.hub_partial);
  const int slot = tile * BW + lane;
  if (grp == 0) {
    __hip_atomic_store(hp + (size_t)(h.base + bd.aux) * a.nq_pad + slot, total, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
  __syncthreads();
  int32_t* counter = a.hub_count + (size_t)bd.r1 * a.ntiles_total + tile;
  if (tid == 0) {
    const int32_t prev = __hip_atomic_fetch_add(counter, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last_flag = prev == h.nseg - 1;
  }
  __syncthreads();
  if (last_flag && grp == 0) {
    __threadfence();
    A s = A(0);
    for (int q = 0; q < h.nseg; ++q)
      s += __hip_atomic_load(hp + (size_t)(h.base + q) * a.nq_pad + slot, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    finish_row(h.row, s, (int32_t)(drp[h.row + 1] - drp[h.row]));
    if (lane == 0) __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One workgroup per slot: r~_0 = e_s/d_s, r~_1 = D^{-1} P e_s, estimate.
template <typename T>
__global__ void __launch_bounds__(kThreads) batch_init_kernel(BatchInitArgs a) {
  using A = typename Acc<T>::type;
  const int slot = blockIdx.x;
  const int64_t s = a.src[slot];
  if (s < 0) return;
  const int tile = slot / a.bw, lane = slot % a.bw;
  const size_t toff = (size_t)tile * (size_t)a.n * a.bw;
  T* r0 = static_cast<T*>(a.r0) + toff;
  T* r1 = static_cast<T*>(a.r1) + toff;
  A* y = static_cast<A*>(a.yacc) + toff;
  const double c0 = a.coef[slot], c1 = a.coef[a.nq_pad + slot];
  const int64_t p0 = a.row_ptr[s], ds = a.row_ptr[s + 1] - p0;
  for (int64_t i = threadIdx.x; i < ds; i += blockDim.x) {
    const int32_t u = a.col_idx[p0 + i];
    const int64_t du = a.row_ptr[u + 1] - a.row_ptr[u];
    const double val = 1.0 / ((double)ds * (double)du);
    r1[(size_t)u * a.bw + lane] = from_acc<T>((A)val);
    y[(size_t)u * a.bw + lane] = (A)(c1 * val);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    r0[(size_t)s * a.bw + lane] = from_acc<T>((A)(1.0 / (double)ds));
    y[(size_t)s * a.bw + lane] = y[(size_t)s * a.bw + lane] + (A)(c0 / (double)ds);
  }
}

// Output of one slot at row v: y = d_v yacc, or oscale d_v^oexp yacc for
// the generalized output of Def. 8 (exact d_v yacc when oexp = 1, oscale = 1).
template <typename A>
__device__ __forceinline__ A slot_output(A yv, int64_t d, double oexp, double oscale) {
  if (oexp == 1.0 && oscale == 1.0) return A(d) * yv;
  return (A)(oscale * pow((double)d, oexp) * (double)yv);
}

// Y[perm(v)][q] = output of yacc[tile(slot)][v][lane(slot)]
template <typename A, typename O>
__global__ void __launch_bounds__(kThreads) batch_finalize_kernel(BatchFinalArgs a) {
  const A* y = static_cast<const A*>(a.yacc);
  O* out = static_cast<O*>(a.Y);
  const int64_t total = a.n * a.nq;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t v = i / a.nq;
    const int q = (int)(i - v * a.nq);
    const int slot = a.slot_of_query[q];
    const int tile = slot / a.bw, lane = slot % a.bw;
    const A val = y[((size_t)tile * a.n + v) * a.bw + lane];
    const int64_t d = a.row_ptr[v + 1] - a.row_ptr[v];
    const int64_t vo = a.perm ? a.perm[v] : v;
    out[vo * a.nq + q] = (O)slot_output<A>(val, d, a.oexp[slot], a.oscale[slot]);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) slot_finish_kernel(SlotFinishArgs a) {
  using A = typename Acc<T>::type;
  using O = typename Out<T>::type;
  const int f = blockIdx.y;
  const int slot = a.slots[f];
  const int tile = slot / a.bw, lane = slot % a.bw;
  O* out = static_cast<O*>(a.outs[f]);
  const double oexp = a.oexp[slot], oscale = a.oscale[slot];
  T* rA = static_cast<T*>(a.rA);
  T* rB = static_cast<T*>(a.rB);
  A* y = static_cast<A*>(a.yacc);
  const T zero = from_acc<T>(A(0));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const size_t e = ((size_t)tile * a.n + v) * a.bw + lane;
    if (out) {
      const int64_t d = a.row_ptr[v + 1] - a.row_ptr[v];
      out[a.perm ? a.perm[v] : v] = (O)slot_output<A>(y[e], d, oexp, oscale);
    }
    y[e] = A(0);
    rA[e] = zero;
    rB[e] = zero;
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) dense_init_kernel(DenseInitArgs a) {
  using A = typename Acc<T>::type;
  using O = typename Out<T>::type;
  const O* X = static_cast<const O*>(a.X);
  T* r0 = static_cast<T*>(a.r0);
  A* y = static_cast<A*>(a.yacc);
  const int64_t total = a.n * a.k;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t v = i / a.k;
    const int j = (int)(i - v * a.k);
    const int64_t d = a.row_ptr[v + 1] - a.row_ptr[v];
    double f = 0.0;  // d^{a-1}: the D^{a} rescaling in the D^{-1} basis
    if (d > 0) f = a.a == 0.0 ? 1.0 / (double)d : a.a == 1.0 ? 1.0 : pow((double)d, a.a - 1.0);
    const int64_t vo = a.perm ? a.perm[v] : v;
    const double x = f * (double)X[vo * a.k + j];
    const size_t e = ((size_t)(j / a.bw) * a.n + v) * a.bw + (j % a.bw);
    r0[e] = from_acc<T>((A)(a.cr * x));
    y[e] = (A)(a.cy * x);
  }
}

struct UploadArgs {
  uint32_t* dst;
  int32_t count;  // 32-bit words
  uint32_t vals[kMaxUploadWords];
};

__global__ void upload_kernel(UploadArgs a) {
  for (int i = threadIdx.x; i < a.count; i += blockDim.x) a.dst[i] = a.vals[i];
}

template <typename T>
hipError_t launch_bs(const BatchStepArgs& a, hipStream_t st) {
  dim3 grid((unsigned)a.nblocks, (unsigned)a.ntiles), block(kThreads);
  // stream tiles hold at most kTileNnz arcs, so fewer than kDeepRowsPerTile
  // rows a tile on average means rows of more than kTileNnz / kDeepRowsPerTile arcs
  const int64_t nstream = a.nblocks - a.nspecial;
  const bool deep = nstream > 0 && a.n < kDeepRowsPerTile * nstream;
  if (a.lanes != 0 && a.lanes < a.bw) {
    if (a.ntiles != 1) return hipErrorInvalidValue;
    switch (a.lanes * 1000 + a.bw) {
      case 8016: hipLaunchKernelGGL((batch_step_kernel<T, 16, false, 8>), grid, block, 0, st, a); break;
      case 8032: hipLaunchKernelGGL((batch_step_kernel<T, 32, false, 8>), grid, block, 0, st, a); break;
      case 8064: hipLaunchKernelGGL((batch_step_kernel<T, 64, false, 8>), grid, block, 0, st, a); break;
      case 16032: hipLaunchKernelGGL((batch_step_kernel<T, 32, false, 16>), grid, block, 0, st, a); break;
      case 16064: hipLaunchKernelGGL((batch_step_kernel<T, 64, false, 16>), grid, block, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (a.bw) {
    case 8: hipLaunchKernelGGL((batch_step_kernel<T, 8, false>), grid, block, 0, st, a); break;
    case 16: hipLaunchKernelGGL((batch_step_kernel<T, 16, false>), grid, block, 0, st, a); break;
    case 32:
      if (deep) hipLaunchKernelGGL((batch_step_kernel<T, 32, true>), grid, block, 0, st, a);
      else hipLaunchKernelGGL((batch_step_kernel<T, 32, false>), grid, block, 0, st, a);
      break;
    case 64:
      if (deep) hipLaunchKernelGGL((batch_step_kernel<T, 64, true>), grid, block, 0, st, a);
      else hipLaunchKernelGGL((batch_step_kernel<T, 64, false>), grid, block, 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

namespace {

hipError_t launch_bs_prec(int32_t prec, const BatchStepArgs& a, hipStream_t st) {
  if (a.nblocks <= 0 || a.ntiles <= 0) return hipSuccess;
  switch (prec) {
    case CP_F64: return launch_bs<double>(a, st);
    case CP_F32: return launch_bs<float>(a, st);
    case CP_F32F: return launch_bs<f32f>(a, st);
    case CP_BF16: return launch_bs<bf16>(a, st);
    default: return hipErrorInvalidValue;
  }
}

BatchStepArgs with_pass(const BatchStepArgs& a, const BatchPass& p) {
  BatchStepArgs b = a;
  b.row_ptr = p.row_ptr;
  b.col_idx = p.col_idx;
  b.blocks = p.blocks;
  b.hubs = p.hubs;
  b.nblocks = p.nblocks;
  b.nspecial = p.nspecial;
  b.split = nullptr;
  return b;
}

}  // namespace

hipError_t launch_batch_step(int32_t prec, const BatchStepArgs& a, hipStream_t st) {
  if (a.ntiles <= 0) return hipSuccess;
  if (!a.split) {
    BatchStepArgs b = a;
    b.deg_rp = nullptr;
    b.part = nullptr;
    return launch_bs_prec(prec, b, st);
  }
  // hot pass: sums over the hot columns into part; cold pass: part + the
  // rest, then the row update with the degree from the full row offsets
  BatchStepArgs h = with_pass(a, a.split->hot);
  h.mode = kBatchHot;
  h.deg_rp = nullptr;  // the hot pass applies no row update
  hipError_t e = launch_bs_prec(prec, h, st);
  if (e != hipSuccess) return e;
  BatchStepArgs c = with_pass(a, a.split->cold);
  c.deg_rp = a.row_ptr;
  return launch_bs_prec(prec, c, st);
}

hipError_t launch_batch_init(int32_t prec, const BatchInitArgs& a, int32_t nslots, hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  dim3 grid((unsigned)nslots), block(kThreads);
  switch (prec) {
    case CP_F64: hipLaunchKernelGGL(batch_init_kernel<double>, grid, block, 0, st, a); break;
    case CP_F32: hipLaunchKernelGGL(batch_init_kernel<float>, grid, block, 0, st, a); break;
    case CP_F32F: hipLaunchKernelGGL(batch_init_kernel<f32f>, grid, block, 0, st, a); break;
    case CP_BF16: hipLaunchKernelGGL(batch_init_kernel<bf16>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_finalize(int32_t prec, const BatchFinalArgs& a, hipStream_t st) {
  dim3 grid(2048), block(kThreads);
  if (prec == CP_F64) hipLaunchKernelGGL((batch_finalize_kernel<double, double>), grid, block, 0, st, a);
  else if (prec == CP_F32) hipLaunchKernelGGL((batch_finalize_kernel<double, float>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((batch_finalize_kernel<float, float>), grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dense_init(int32_t prec, const DenseInitArgs& a, hipStream_t st) {
  if (a.n * a.k <= 0) return hipSuccess;
  dim3 grid(2048), block(kThreads);
  switch (prec) {
    case CP_F64: hipLaunchKernelGGL(dense_init_kernel<double>, grid, block, 0, st, a); break;
    case CP_F32: hipLaunchKernelGGL(dense_init_kernel<float>, grid, block, 0, st, a); break;
    case CP_F32F: hipLaunchKernelGGL(dense_init_kernel<f32f>, grid, block, 0, st, a); break;
    case CP_BF16: hipLaunchKernelGGL(dense_init_kernel<bf16>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_slot_finish(int32_t prec, const SlotFinishArgs& a, int32_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  dim3 grid(1024, (unsigned)count), block(kThreads);
  switch (prec) {
    case CP_F64: hipLaunchKernelGGL(slot_finish_kernel<double>, grid, block, 0, st, a); break;
    case CP_F32: hipLaunchKernelGGL(slot_finish_kernel<float>, grid, block, 0, st, a); break;
    case CP_F32F: hipLaunchKernelGGL(slot_finish_kernel<f32f>, grid, block, 0, st, a); break;
    case CP_BF16: hipLaunchKernelGGL(slot_finish_kernel<bf16>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_upload(void* dst, const void* host, size_t bytes, hipStream_t st) {
  if (bytes % 4) return hipErrorInvalidValue;
  uint32_t* d = static_cast<uint32_t*>(dst);
  const uint32_t* h = static_cast<const uint32_t*>(host);
  size_t words = bytes / 4;
  while (words > 0) {
    UploadArgs u;
    u.dst = d;
    u.count = (int32_t)(words < (size_t)kMaxUploadWords ? words : (size_t)kMaxUploadWords);
    for (int i = 0; i < u.count; ++i) u.vals[i] = h[i];
    hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, st, u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    d += u.count;
    h += u.count;
    words -= (size_t)u.count;
  }
  return hipSuccess;
}

}  // namespace cp
