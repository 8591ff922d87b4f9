// Device kernels of the single-source ChebyPower path (gfx950, wave64).
//
// Precision: CP_F64 stores and computes in double; CP_F32 stores the
// recurrence vectors in float (the gathered bytes) but sums, updates and
// accumulates the estimate in double; CP_F32F stores float and sums,
// updates and accumulates in float (estimate and partial sums in float
// too); CP_BF16 stores bfloat16 and computes in float.
//
// Vectors live in the D^{-1} basis: x = D^{-1} r_k, z = D^{-1} r_{k-1},
// yacc = D^{-1} y.  Then (P r_k)(v) = sum_{u in N(v)} r_k(u)/d_u is a pure
// gather-sum of x over row v, and the Chebyshev recurrence of Eq. (6),
// r_{k+1} = 2 P r_k - r_{k-1}, becomes, per row,
//   z_new(v) = 2 (sum_{u in N(v)} x(u)) / d_v - z(v).
// This is T_k(D^{-1/2} A D^{-1/2}) applied to D^{-1/2} e_s and rescaled
// (the similarity P = D^{1/2} A~ D^{-1/2} of the Lemma 1 proof), so the
// symmetric normalisation costs one per-row divide and no per-arc degree
// reads.  Alg. 3 adds c_k r_k at the top of iteration k; here each term is
// added as soon as it is produced, which sums the same c_0..c_K terms.
//
// Summation order is fixed by the block plan, never by timing, so every
// result is bitwise reproducible run to run (no floating-point atomics).

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
template <> struct Acc<bf16> { using type = float; };

__device__ __forceinline__ double to_acc(double v) { return v; }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ float to_acc(f32f v) { return v.v; }
__device__ __forceinline__ float to_acc(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }

template <typename T> __device__ __forceinline__ T from_acc(typename Acc<T>::type v);
template <> __device__ __forceinline__ double from_acc<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_acc<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ f32f from_acc<f32f>(float v) { return f32f{v}; }
// float -> bfloat16, round to nearest even (finite inputs)
template <> __device__ __forceinline__ bf16 from_acc<bf16>(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}

template <typename T> __device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <> __device__ __forceinline__ bf16 ld_stream<bf16>(const bf16* p) {
  return bf16{__builtin_nontemporal_load(&p->bits)};
}
template <> __device__ __forceinline__ f32f ld_stream<f32f>(const f32f* p) {
  return f32f{__builtin_nontemporal_load(&p->v)};
}
template <typename T> __device__ __forceinline__ void st_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
template <> __device__ __forceinline__ void st_stream<bf16>(bf16* p, bf16 v) {
  __builtin_nontemporal_store(v.bits, &p->bits);
}
template <> __device__ __forceinline__ void st_stream<f32f>(f32f* p, f32f v) {
  __builtin_nontemporal_store(v.v, &p->v);
}

template <typename A> __device__ __forceinline__ A wave_sum(A v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Logical block for workgroup w.  Workgroups are dispatched round-robin over
// the 8 XCDs; inside the stream region consecutive logical blocks are given
// to workgroups of the same XCD so neighbouring tiles share L2 lines.
__device__ __forceinline__ int64_t logical_block(int64_t w, int64_t nblocks, int64_t nspecial) {
  if (w < nspecial) return w;
  const int64_t m = nblocks - nspecial, i = w - nspecial;
  const int64_t q = m >> 3, r = m & 7, x = i & 7, j = i >> 3;
  return nspecial + x * q + (x < r ? x : r) + j;
}

// Chebyshev step (Eq. 6): z(v) <- 2 acc / d - z(v);  power step (Alg. 1):
// z(v) <- acc / d.  Then yacc(v) += c z_new.  Push pull (Alg. 4):
// z(v) <- z(v) + acc, no estimate.
template <typename T, typename A, int MODE>
__device__ __forceinline__ void row_update(T* z, A* yacc, int64_t v, A acc, int32_t d, A c) {
  A zn;
  if constexpr (MODE == kStepAdd) {
    st_stream(z + v, from_acc<T>(to_acc(ld_stream(z + v)) + acc));
    return;
  }
  if constexpr (MODE == kStepPower) zn = acc / A(d);
  else zn = (A(2) * acc) / A(d) - to_acc(ld_stream(z + v));
  st_stream(z + v, from_acc<T>(zn));
  st_stream(yacc + v, ld_stream(yacc + v) + c * zn);
}

// row_update with z(v) and yacc(v) already loaded (as zold, yold).
template <typename T, typename A, int MODE>
__device__ __forceinline__ void row_update_loaded(T* z, A* yacc, int64_t v, A acc, int32_t d, A c, A zold, A yold) {
  A zn;
  if constexpr (MODE == kStepAdd) {
    st_stream(z + v, from_acc<T>(zold + acc));
    return;
  }
  if constexpr (MODE == kStepPower) zn = acc / A(d);
  else zn = (A(2) * acc) / A(d) - zold;
  st_stream(z + v, from_acc<T>(zn));
  st_stream(yacc + v, yold + c * zn);
}

// Running sum of a long chain of terms.  A float chain uses Kahan's
// compensated summation (Kahan, 1965): the low-order part lost by each add
// is carried into the next, so the chain's rounding does not grow with its
// length (a hub row's stripe segment can be tens of thousands of arcs, one
// chain of d / 256 terms per thread).  Double chains are plain sums.
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

// Whole-workgroup gather-sum of x over arcs [p0, p1); result valid in thread 0.
template <typename T, typename A>
__device__ __forceinline__ A block_gather_sum(const int32_t* __restrict__ col, const T* __restrict__ x,
                                              int64_t p0, int64_t p1, A* wsum) {
  const int tid = threadIdx.x;
  ChainSum<A> chain;
  for (int64_t base = p0; base < p1; base += kTileNnz) {
    int32_t idx[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
      const int64_t i = base + tid + u * kThreads;
      idx[u] = i < p1 ? ld_stream(col + i) : -1;
    }
    A v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) v[u] = idx[u] >= 0 ? to_acc(x[idx[u]]) : A(0);
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) chain.add(v[u]);
  }
  A acc = wave_sum(chain.value());
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  A total = A(0);
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) total += wsum[q];
  }
  return total;
}

// LDS slot of arc p of a tile: the CH arcs a thread scans keep their chunk
// but are rotated by an XOR with bits of the thread's wave position, so at
// every step of the scan the 64 lanes of a wavefront read 64 different
// banks (4-byte values; 8-byte values: two lanes per bank pair).
template <int CH> __device__ __forceinline__ int lds_slot(int p) {
  static_assert(CH > 0 && CH <= 64 && (CH & (CH - 1)) == 0, "chunk must be a power of two up to 64");
  return p ^ ((p >> 6) & (CH - 1));
}

// Row sums of an LDS tile: vals[lds_slot(p)] holds the gathered value of arc
// p of the tile, rpl[0..nr] the tile-relative row offsets (cnt <= kTileNnz).
// Thread t owns arcs [CH t, CH t + CH); heads are row starts.  (F, V) = (chunk holds
// a head, sum since the last head) is scanned over threads (wavefront
// shuffles, then wavefront totals in LDS) to give each thread the partial
// sum of the row still open at its chunk start; the thread holding a row's
// last arc writes rowsum[row].  Caller: vals/rpl staged, rowsum zeroed,
// barrier passed.  Ends with a barrier.
template <int CH, typename VT, typename A>
__device__ __forceinline__ void tile_rowsums(const VT* vals, const int32_t* rpl, int nr, int cnt, A* rowsum,
                                             A* wsum, int32_t* wflag) {
  const int tid = threadIdx.x;
  const int start = tid * CH;
  const int end = start + CH < cnt ? start + CH : cnt;
  int row = 0;
  int32_t F = 0;
  A V = A(0);
  if (start < cnt) {
    int lo = 0, hi = nr - 1;  // largest j with rpl[j] <= start
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rpl[mid] <= start) lo = mid; else hi = mid - 1;
    }
    row = lo;
    int r = row;
    for (int p = start; p < end; ++p) {
      while (rpl[r + 1] <= p) ++r;
      if (rpl[r] == p) { F = 1; V = A(0); }
      V += (A)vals[lds_slot<CH>(p)];
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const A Vp = __shfl_up(V, off, 64);
    const int32_t Fp = __shfl_up(F, off, 64);
    if (lane >= off) {
      if (!F) V = Vp + V;
      F |= Fp;
    }
  }
  if (lane == 63) { wsum[wv] = V; wflag[wv] = F; }
  __syncthreads();
  A Vex = __shfl_up(V, 1, 64);
  int32_t Fex = __shfl_up(F, 1, 64);
  if (lane == 0) { Vex = A(0); Fex = 0; }
  A Cw = A(0);
  for (int q = 0; q < wv; ++q) Cw = wflag[q] ? wsum[q] : Cw + wsum[q];
  const A carry = Fex ? Vex : Cw + Vex;
  if (start < cnt) {
    int r = row;
    A acc = carry;
    for (int p = start; p < end; ++p) {
      while (rpl[r + 1] <= p) ++r;
      if (rpl[r] == p) acc = A(0);
      acc += (A)vals[lds_slot<CH>(p)];
      if (p + 1 == rpl[r + 1]) rowsum[r] = acc;
    }
  }
  __syncthreads();
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) step_kernel(StepArgs a) {
  using A = typename Acc<T>::type;
  __shared__ A vals[kTileNnz];
  __shared__ int32_t rpl[kTileRows + 1];
  __shared__ A rowsum[kTileRows];
  __shared__ A wsum[kThreads / 64];
  __shared__ int32_t wflag[kThreads / 64];
  if (a.gate && *a.gate == 0) return;

  const int tid = threadIdx.x;
  const int64_t b = logical_block(blockIdx.x, a.nblocks, a.nspecial);
  const BlockDesc bd = a.blocks[b];
  const int64_t* __restrict__ rp = a.row_ptr;
  const int32_t* __restrict__ col = a.col_idx;
  const T* __restrict__ x = static_cast<const T*>(a.x);
  T* __restrict__ z = static_cast<T*>(a.z);
  A* __restrict__ yacc = static_cast<A*>(a.yacc);
  const A c = (A)a.c;

  if (bd.kind == kStream) {
    static_assert(kTileRows <= kThreads, "one row of a stream tile per thread");
    const int32_t r0 = bd.r0, nr = bd.r1 - bd.r0;
    const int64_t p0 = bd.p0;
    const int32_t cnt = bd.aux;
    // Thread j's row: its old z and estimate are loaded now, beside the
    // column stream and the gathers, not after the row sums.
    const bool own = tid < nr;
    A zold = A(0), yold = A(0);
    if (own) {
      if constexpr (MODE != kStepPower) zold = to_acc(ld_stream(z + r0 + tid));
      if constexpr (MODE != kStepAdd) yold = ld_stream(yacc + r0 + tid);
    }
    for (int j = tid; j <= nr; j += kThreads) rpl[j] = (int32_t)(rp[r0 + j] - p0);
    if (own) rowsum[tid] = A(0);

    // Phase 1: coalesced stream of the tile's column ids, gather, stage in LDS.
    int32_t idx[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
      const int i = tid + u * kThreads;
      idx[u] = i < cnt ? ld_stream(col + p0 + i) : -1;
    }
    A v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) v[u] = idx[u] >= 0 ? to_acc(x[idx[u]]) : A(0);
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
      const int i = tid + u * kThreads;
      if (i < cnt) vals[lds_slot<kPerThread>(i)] = v[u];
    }
    __syncthreads();

    tile_rowsums<kPerThread, A, A>(vals, rpl, nr, cnt, rowsum, wsum, wflag);

    // Phase 3: row-parallel recurrence and accumulation.
    if (own) {
      const int32_t d = rpl[tid + 1] - rpl[tid];
      if (d > 0) row_update_loaded<T, A, MODE>(z, yacc, (int64_t)r0 + tid, rowsum[tid], d, c, zold, yold);
    }
    return;
  }

  if (bd.kind == kLong) {
    const int64_t v = bd.r0;
    const int64_t p0 = rp[v], p1 = rp[v + 1];
    const A total = block_gather_sum<T, A>(col, x, p0, p1, wsum);
    if (tid == 0) row_update<T, A, MODE>(z, yacc, v, total, (int32_t)(p1 - p0), c);
    return;
  }

  // Hub segment.
  const HubDesc h = a.hubs[bd.r1];
  const int64_t rb = rp[h.row], re = rp[h.row + 1];
  const int64_t p0 = rb + (int64_t)bd.aux * h.seg;
  const int64_t p1 = p0 + h.seg < re ? p0 + h.seg : re;
  const A total = block_gather_sum<T, A>(col, x, p0, p1, wsum);
  if (tid == 0) {
    A* part = static_cast<A*>(a.hub_partial);
    __hip_atomic_store(part + h.base + bd.aux, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t prev =
        __hip_atomic_fetch_add(a.hub_count + bd.r1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == h.nseg - 1) {
      A s = A(0);
      for (int q = 0; q < h.nseg; ++q)
        s += __hip_atomic_load(part + h.base + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      row_update<T, A, MODE>(z, yacc, h.row, s, (int32_t)(re - rb), c);
      __hip_atomic_store(a.hub_count + bd.r1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}


// LDS copy of gathered values: the stored precision (exact), float for bf16.
template <typename T> struct Lds { using type = T; };
template <> struct Lds<bf16> { using type = float; };
template <> struct Lds<f32f> { using type = float; };

// One (row tile, stripe) block of an XCD-striped step: partial row sums of
// the tile's rows over the stripe's columns.  Workgroup w handles tile
// w / S and stripe w % S, so the workgroups of stripe j run on the XCDs
// j, j + S, ... (workgroups go round-robin over the 8 XCDs, S divides 8).
template <typename T, bool PACKED>
__global__ void __launch_bounds__(kThreads) stripe_gather_kernel(StripeArgs a) {
  using A = typename Acc<T>::type;
  using L = typename Lds<T>::type;
  if (a.gate && *a.gate == 0) return;
  __shared__ L vals[kStripeTileNnz];
  __shared__ int32_t rpl[kStripeTileRows + 1];
  __shared__ A rowsum[kStripeTileRows];
  __shared__ A wsum[kThreads / 64];
  __shared__ int32_t wflag[kThreads / 64];

  const int tid = threadIdx.x;
  const int j = (int)(blockIdx.x % (unsigned)a.nstripes);
  const StripeBlock sb = a.blocks[blockIdx.x];
  const int32_t* __restrict__ rpj = a.rp + (size_t)j * (size_t)(a.n + 1);
  const int32_t* __restrict__ cols = a.cols + a.col_off[j];
  const T* __restrict__ x = static_cast<const T*>(a.x);
  A* __restrict__ part = static_cast<A*>(a.partial) + (size_t)j * (size_t)a.n;
  const int32_t r0 = sb.r0, nr = sb.nr, p0 = sb.p0, cnt = sb.cnt;

  if (cnt <= kStripeTileNnz) {
    // column ids and row offsets only depend on the descriptor: issue both
    constexpr int CH = kStripeTileNnz / kThreads;
    uint32_t w[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = tid + u * kThreads;
      w[u] = i < cnt ? (uint32_t)ld_stream(cols + p0 + i) : 0u;
    }
    for (int i = tid; i <= nr; i += kThreads) rpl[i] = rpj[r0 + i] - p0;
    for (int i = tid; i < nr; i += kThreads) rowsum[i] = A(0);
    const T* __restrict__ xs = PACKED ? x + a.base[j] : x;
    L v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = tid + u * kThreads;
      v[u] = i < cnt ? (L)to_acc(xs[PACKED ? (w[u] >> kPackPosBits) : w[u]]) : L(0);
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = tid + u * kThreads;
      if (i < cnt) vals[lds_slot<CH>(PACKED ? (int)(w[u] & ((1u << kPackPosBits) - 1u)) : i)] = v[u];
    }
    __syncthreads();
    tile_rowsums<CH, L, A>(vals, rpl, nr, cnt, rowsum, wsum, wflag);
    for (int i = tid; i < nr; i += kThreads) st_stream(part + r0 + i, rowsum[i]);
    return;
  }
  // one row whose stripe segment exceeds the LDS tile: whole-workgroup stream
  const A total = block_gather_sum<T, A>(cols, x, p0, (int64_t)p0 + cnt, wsum);
  if (tid == 0) st_stream(part + r0, total);
}

// Combine the S stripe partials of every row (in stripe order) and apply the
// recurrence and estimate update.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) stripe_combine_kernel(CombineArgs a) {
  using A = typename Acc<T>::type;
  if (a.gate && *a.gate == 0) return;
  const A* __restrict__ part = static_cast<const A*>(a.partial);
  T* __restrict__ z = static_cast<T*>(a.z);
  A* __restrict__ yacc = static_cast<A*>(a.yacc);
  const A c = (A)a.c;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int64_t d = a.row_ptr[v + 1] - a.row_ptr[v];
    if (d == 0) continue;
    A acc = A(0);
    for (int j = 0; j < a.nstripes; ++j) acc += ld_stream(part + (size_t)j * (size_t)a.n + v);
    row_update<T, A, MODE>(z, yacc, v, acc, (int32_t)d, c);
  }
}

__global__ void zero_kernel(uint4* p, size_t n16, uint32_t* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0)
    for (size_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) init_kernel(InitArgs a) {
  using A = typename Acc<T>::type;
  T* r0 = static_cast<T*>(a.r0);
  T* r1 = static_cast<T*>(a.r1);
  A* yacc = static_cast<A*>(a.yacc);
  const int64_t s = a.s;
  const int64_t p0 = a.row_ptr[s], ds = a.row_ptr[s + 1] - p0;
  // r~_1(u) = (P e_s)(u) / d_u = 1 / (d_s d_u) for u in N(s)
  for (int64_t i = threadIdx.x; i < ds; i += blockDim.x) {
    const int32_t u = a.col_idx[p0 + i];
    const int64_t du = a.row_ptr[u + 1] - a.row_ptr[u];
    const double val = 1.0 / ((double)ds * (double)du);
    r1[u] = from_acc<T>((A)val);
    yacc[u] = (A)(a.c1 * val);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    r0[s] = from_acc<T>((A)(1.0 / (double)ds));
    yacc[s] = yacc[s] + (A)(a.c0 / (double)ds);
  }
}

template <typename A, typename O>
__global__ void __launch_bounds__(kThreads) finalize_kernel(FinalArgs a, double* block_sums) {
  const A* yacc = static_cast<const A*>(a.yacc);
  O* out = static_cast<O*>(a.y_out);
  double local = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int64_t d = a.row_ptr[v + 1] - a.row_ptr[v];
    const A yv = a.oexp == 1.0 && a.oscale == 1.0 ? A(d) * yacc[v]
                                                  : (A)(a.oscale * pow((double)d, a.oexp) * (double)yacc[v]);
    out[a.perm ? a.perm[v] : v] = (O)yv;
    local += (double)(O)yv;
  }
  if (block_sums) {
    __shared__ double ws[kThreads / 64];
    local = wave_sum(local);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < kThreads / 64; ++q) t += ws[q];
      block_sums[blockIdx.x] = t;
    }
  }
}

__global__ void sum_blocks_kernel(const double* block_sums, int nb, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < nb; ++i) t += block_sums[i];
    *out = t;
  }
}

constexpr int kFinalBlocks = 1024;

}  // namespace

template <int MODE>
hipError_t launch_step_t(int32_t prec, const StepArgs& a, hipStream_t st) {
  dim3 grid((unsigned)a.nblocks), block(kThreads);
  switch (prec) {
    case CP_F64: hipLaunchKernelGGL((step_kernel<double, MODE>), grid, block, 0, st, a); break;
    case CP_F32: hipLaunchKernelGGL((step_kernel<float, MODE>), grid, block, 0, st, a); break;
    case CP_F32F: hipLaunchKernelGGL((step_kernel<f32f, MODE>), grid, block, 0, st, a); break;
    case CP_BF16: hipLaunchKernelGGL((step_kernel<bf16, MODE>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step(int32_t prec, const StepArgs& a, StepMode mode, hipStream_t st) {
  if (a.nblocks <= 0) return hipSuccess;
  switch (mode) {
    case kStepCheb: return launch_step_t<kStepCheb>(prec, a, st);
    case kStepPower: return launch_step_t<kStepPower>(prec, a, st);
    case kStepAdd:  // the push pull runs in FP64 only
      if (prec != CP_F64) return hipErrorInvalidValue;
      hipLaunchKernelGGL((step_kernel<double, kStepAdd>), dim3((unsigned)a.nblocks), dim3(kThreads), 0, st, a);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stripe_gather(int32_t prec, const StripeArgs& a, hipStream_t st) {
  if (a.ntiles <= 0) return hipSuccess;
  if (a.nstripes < 1 || a.nstripes > kMaxStripes || kMaxStripes % a.nstripes) return hipErrorInvalidValue;
  dim3 grid((unsigned)(a.ntiles * a.nstripes)), block(kThreads);
  switch (prec * 2 + (a.packed ? 1 : 0)) {
    case CP_F64 * 2: hipLaunchKernelGGL((stripe_gather_kernel<double, false>), grid, block, 0, st, a); break;
    case CP_F64 * 2 + 1: hipLaunchKernelGGL((stripe_gather_kernel<double, true>), grid, block, 0, st, a); break;
    case CP_F32 * 2: hipLaunchKernelGGL((stripe_gather_kernel<float, false>), grid, block, 0, st, a); break;
    case CP_F32 * 2 + 1: hipLaunchKernelGGL((stripe_gather_kernel<float, true>), grid, block, 0, st, a); break;
    case CP_F32F * 2: hipLaunchKernelGGL((stripe_gather_kernel<f32f, false>), grid, block, 0, st, a); break;
    case CP_F32F * 2 + 1: hipLaunchKernelGGL((stripe_gather_kernel<f32f, true>), grid, block, 0, st, a); break;
    case CP_BF16 * 2: hipLaunchKernelGGL((stripe_gather_kernel<bf16, false>), grid, block, 0, st, a); break;
    case CP_BF16 * 2 + 1: hipLaunchKernelGGL((stripe_gather_kernel<bf16, true>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_stripe_combine_t(int32_t prec, const CombineArgs& a, hipStream_t st) {
  int64_t blocks = (a.n + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  dim3 grid((unsigned)blocks), block(kThreads);
  switch (prec) {
    case CP_F64: hipLaunchKernelGGL((stripe_combine_kernel<double, MODE>), grid, block, 0, st, a); break;
    case CP_F32:
      if constexpr (MODE == kStepAdd) return hipErrorInvalidValue;
      else hipLaunchKernelGGL((stripe_combine_kernel<float, MODE>), grid, block, 0, st, a);
      break;
    case CP_F32F:
      if constexpr (MODE == kStepAdd) return hipErrorInvalidValue;
      else hipLaunchKernelGGL((stripe_combine_kernel<f32f, MODE>), grid, block, 0, st, a);
      break;
    case CP_BF16:
      if constexpr (MODE == kStepAdd) return hipErrorInvalidValue;
      else hipLaunchKernelGGL((stripe_combine_kernel<bf16, MODE>), grid, block, 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stripe_combine(int32_t prec, const CombineArgs& a, StepMode mode, hipStream_t st) {
  switch (mode) {
    case kStepCheb: return launch_stripe_combine_t<kStepCheb>(prec, a, st);
    case kStepPower: return launch_stripe_combine_t<kStepPower>(prec, a, st);
    case kStepAdd: return launch_stripe_combine_t<kStepAdd>(prec, a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16, ntail = (bytes % 16) / 4;
  unsigned grid = (unsigned)((n16 + kThreads - 1) / kThreads);
  if (grid > 2048) grid = 2048;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(kThreads), 0, st, static_cast<uint4*>(p), n16,
                     reinterpret_cast<uint32_t*>(static_cast<char*>(p) + n16 * 16), ntail);
  return hipGetLastError();
}

hipError_t launch_init(int32_t prec, const InitArgs& a, hipStream_t st) {
  switch (prec) {
    case CP_F64: hipLaunchKernelGGL(init_kernel<double>, dim3(1), dim3(kThreads), 0, st, a); break;
    case CP_F32: hipLaunchKernelGGL(init_kernel<float>, dim3(1), dim3(kThreads), 0, st, a); break;
    case CP_F32F: hipLaunchKernelGGL(init_kernel<f32f>, dim3(1), dim3(kThreads), 0, st, a); break;
    case CP_BF16: hipLaunchKernelGGL(init_kernel<bf16>, dim3(1), dim3(kThreads), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(int32_t prec, const FinalArgs& a, hipStream_t st) {
  double* block_sums = a.mass ? a.mass + 1 : nullptr;  // mass[0] result, mass[1..] scratch
  if (prec == CP_F64)
    hipLaunchKernelGGL((finalize_kernel<double, double>), dim3(kFinalBlocks), dim3(kThreads), 0, st, a, block_sums);
  else if (prec == CP_F32)
    hipLaunchKernelGGL((finalize_kernel<double, float>), dim3(kFinalBlocks), dim3(kThreads), 0, st, a, block_sums);
  else  // float estimate: CP_F32F, CP_BF16
    hipLaunchKernelGGL((finalize_kernel<float, float>), dim3(kFinalBlocks), dim3(kThreads), 0, st, a, block_sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.mass) return e;
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(64), 0, st, block_sums, kFinalBlocks, a.mass);
  return hipGetLastError();
}

}  // namespace cp
