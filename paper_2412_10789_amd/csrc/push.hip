// ChebyPush (Alg. 4, Sec. 4.2) on the GPU: the subset Chebyshev recurrence
// of Def. 7 in its push form, computed without floating-point atomics.
// Residuals stay in the paper's space (FP64): r_cur starts as P e_s, r_new
// as -e_s, and iteration k
//   1. select (one pass over the nodes): every u with |r_cur(u)| > eps_k d_u
//      adds c_k r_cur(u) to y(u), stores its push value pv(u) = 2 r_cur(u)
//      / d_u, flips the sign of r_cur(u) and is stamped sel(u) = k; the push
//      values of the previous iteration are cleared in the same pass, and
//      per-block counts and degree sums give |S_k| and vol(S_k), which
//      decide whether the iteration is sparse or dense;
//   2. the stamped nodes are listed in node order (S_k) and their arcs mark
//      every neighbour with mark(v) = k (plain stores);
//   3. the marked rows are listed in node order, short and long rows apart;
//   4. pull: every marked row adds sum_{u in N(v)} pv(u) to r_new(v), summed
//      in CSR order (a long row: one workgroup, thread-strided partial sums
//      combined in a fixed order), gathering pv(u) only where u's bit is set
//      in a bitmap of S_k (every other pv is zero);
//   5. the host swaps r_cur and r_new.
// Step 4 is r_new += 2 P (r_cur|S_k) restricted to the rows it changes, so
// the iteration is exactly the push form of Sec. 4.2.  In a dense
// iteration (see kDenseDiv, kDenseVolDiv) steps 2-4 are skipped and the tiled
// single-source step kernels (or their XCD-striped form) pull every row in
// their add mode, r_new += sum of pv over the row (a row with no pushed
// neighbour adds an exact zero).  The choice is made on the device: every
// launch of both paths is queued and reads the dense flag, so the host never
// waits.  Nothing depends on timing, so results are bitwise reproducible run
// to run.  The arcs of the pushed nodes are visited twice (marks, then the
// pulls of their neighbours' rows), both at gather speed; the listing passes
// cost O(n) per iteration in coalesced reads.

#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

namespace cp {
namespace {

constexpr int kRangeBlocks = 1024;  // fixed node ranges of the listing passes
constexpr int kEdgeBlocks = 1024;
constexpr int kChunk = kThreads;    // selected nodes expanded together by one workgroup
constexpr int32_t kShortRow = 32;   // rows up to this degree are pulled by one thread

struct PushLayout {
  size_t r[2], y, pv, deg, sel, mark, slist, tshort, tlong, bits, bcount, bvol, counts, hubc, sums, part, total;
};

// counts (int64): [0] |S_k|, [1] short marked rows, [2] long marked rows,
// [3] pushes (sum of |S_k|), [4] arcs (sum of vol(S_k)), [5] dense flag of
// the current iteration
constexpr int kCounts = 6;
// An iteration that pushes more than n / kDenseDiv nodes, or nodes with
// more than nnz / kDenseVolDiv arcs, pulls every row with the tiled step
// kernels (no marks, no row lists).  Neighbours of pushed nodes lean to
// high degrees, so the marked rows hold many more arcs than the pushed
// ones: on power-law graphs the sparse form only pays for small volumes
// (nnz / 128 was the best of 8 ... 4096 on a 4M-node, 70M-arc graph).
constexpr int64_t kDenseDiv = 8;
constexpr int64_t kDenseVolDiv = 128;

PushLayout push_layout(const cp_graph* g) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t n = (size_t)g->n;
  PushLayout L{};
  size_t off = 0;
  for (int i = 0; i < 2; ++i) { L.r[i] = off; off += al(n * 8); }
  L.y = off; off += al(n * 8);
  L.pv = off; off += al(n * 8);
  L.deg = off; off += al(n * 4);
  L.sel = off; off += al(n * 4);
  L.mark = off; off += al(n * 4);
  L.slist = off; off += al(n * 4);
  L.tshort = off; off += al(n * 4);
  L.tlong = off; off += al(n * 4);
  L.bits = off; off += al((n + 31) / 32 * 4);
  L.bcount = off; off += al((size_t)3 * kRangeBlocks * 4);
  L.bvol = off; off += al((size_t)kRangeBlocks * 8);
  L.counts = off; off += al((size_t)kCounts * 8);
  // hub row counters of the dense step (zero between launches)
  L.hubc = off; off += al((size_t)batch_hub_rows(g) * 4);
  L.sums = off; off += al((size_t)(1 + kRangeBlocks) * 8);
  // dense step partial sums: [S][n] (striped) or one per hub segment
  L.part = off;
  off += al(g->striped ? (size_t)g->s_count * n * 8 : (size_t)batch_hub_segments(g) * 8);
  L.total = off;
  return L;
}

// Node range [lo, hi) of listing block blockIdx.x (grid of kRangeBlocks).
__device__ __forceinline__ void block_range(int64_t n, int64_t& lo, int64_t& hi) {
  const int64_t span = (n + kRangeBlocks - 1) / kRangeBlocks;
  lo = (int64_t)blockIdx.x * span;
  hi = lo + span < n ? lo + span : n;
}

__device__ __forceinline__ long long block_sum_ll(long long v, long long* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  long long t = 0;
  for (int q = 0; q < kThreads / 64; ++q) t += red[q];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int block_sum_int(int v, int* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
  for (int q = 0; q < kThreads / 64; ++q) t += red[q];
  __syncthreads();
  return t;
}

// Ordered compaction step of a block: among this round's kThreads
// candidates (one per thread, in thread order) the takers get consecutive
// positions after `base`, which advances by their number.  All threads
// call it; returns the taker's position or -1.
__device__ __forceinline__ int64_t block_place(bool take, int* wcnt, int64_t& base) {
  const unsigned long long mask = __ballot(take);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wcnt[wv] = __popcll(mask);
  __syncthreads();
  int before = 0, total = 0;
  for (int q = 0; q < kThreads / 64; ++q) {
    if (q < wv) before += wcnt[q];
    total += wcnt[q];
  }
  __syncthreads();
  const int64_t pos = base + before + __popcll(mask & ((1ull << lane) - 1ull));
  base += total;
  return take ? pos : -1;
}

struct DegreeArgs {
  const int64_t* row_ptr;
  int64_t n;
  int32_t* deg;
};

__global__ void __launch_bounds__(kThreads) push_degree_kernel(DegreeArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride)
    a.deg[v] = (int32_t)(a.row_ptr[v + 1] - a.row_ptr[v]);
}

struct SeedArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  int64_t s;
  double c0;
  double* r_cur;  // P e_s
  double* r_new;  // -e_s
  double* y;
};

__global__ void __launch_bounds__(kThreads) push_seed_kernel(SeedArgs a) {
  const int64_t p0 = a.row_ptr[a.s], ds = a.row_ptr[a.s + 1] - p0;
  const double w = 1.0 / (double)ds;
  for (int64_t i = threadIdx.x; i < ds; i += blockDim.x) a.r_cur[a.col_idx[p0 + i]] = w;
  if (threadIdx.x == 0) {
    a.r_new[a.s] = -1.0;
    a.y[a.s] = a.c0;
  }
}

struct SelectArgs {
  int64_t n;
  const int32_t* deg;
  double* r;  // r_cur
  double* y;
  double* pv;
  int32_t* sel;
  int32_t k;
  double eps, c;
  int32_t* bcount;  // per range block: selected nodes
  long long* bvol;  // per range block: their degree sum
};

__global__ void __launch_bounds__(kThreads) push_select_kernel(SelectArgs a) {
  __shared__ int red[kThreads / 64];
  __shared__ long long redl[kThreads / 64];
  int64_t lo, hi;
  block_range(a.n, lo, hi);
  int cnt = 0;
  long long vol = 0;
  for (int64_t v = lo + threadIdx.x; v < hi; v += kThreads) {
    const double val = a.r[v];
    const int32_t d = a.deg[v];
    if (d > 0 && fabs(val) > a.eps * (double)d) {
      a.y[v] += a.c * val;
      a.pv[v] = 2.0 * val / (double)d;
      a.r[v] = -val;
      a.sel[v] = a.k;
      ++cnt;
      vol += d;
    } else if (a.k > 1 && a.sel[v] == a.k - 1) {
      a.pv[v] = 0.0;  // pushed in the previous iteration only
    }
  }
  const int t = block_sum_int(cnt, red);
  const long long tv = block_sum_ll(vol, redl);
  if (threadIdx.x == 0) {
    a.bcount[blockIdx.x] = t;
    a.bvol[blockIdx.x] = tv;
  }
}

// After the select pass: |S_k| and vol(S_k) from the per-block sums, the
// push and arc counters, and the dense decision of the iteration.
struct DecideArgs {
  int64_t n, nnz;
  const int32_t* bcount;
  const long long* bvol;
  long long* counts;  // [0] |S_k| (set), [3] pushes, [4] arcs (accumulated), [5] dense flag (set)
};

__global__ void __launch_bounds__(kThreads) push_decide_kernel(DecideArgs a) {
  __shared__ long long red[kThreads / 64];
  long long m = 0, vol = 0;
  for (int b = threadIdx.x; b < kRangeBlocks; b += kThreads) {
    m += a.bcount[b];
    vol += a.bvol[b];
  }
  m = block_sum_ll(m, red);
  vol = block_sum_ll(vol, red);
  if (threadIdx.x == 0) {
    a.counts[0] = m;
    a.counts[3] += m;
    a.counts[4] += vol;
    a.counts[5] = m * kDenseDiv > a.n || vol * kDenseVolDiv > a.nnz ? 1 : 0;
  }
}

// Lists of the nodes stamped k, in node order.  With split_long, rows
// longer than kShortRow go to list1, the others to list0.
struct ListArgs {
  int64_t n;
  const int32_t* stamp;
  const int32_t* deg;
  int32_t k;
  int32_t split_long;
  int32_t* bcount0;  // per range block counts (written by the count pass)
  int32_t* bcount1;
  int32_t* list0;
  int32_t* list1;
  long long* count0;
  long long* count1;
  const long long* dense;  // set: the iteration is dense, nothing to list
};

__device__ __forceinline__ bool listed(const ListArgs& a, int64_t v) { return a.stamp[v] == a.k; }

__global__ void __launch_bounds__(kThreads) push_count_kernel(ListArgs a) {
  __shared__ int red[kThreads / 64];
  if (*a.dense) return;
  int64_t lo, hi;
  block_range(a.n, lo, hi);
  int c0 = 0, c1 = 0;
  for (int64_t v = lo + threadIdx.x; v < hi; v += kThreads) {
    if (!listed(a, v)) continue;
    if (a.split_long && a.deg[v] > kShortRow) ++c1; else ++c0;
  }
  const int t0 = block_sum_int(c0, red);
  const int t1 = block_sum_int(c1, red);
  if (threadIdx.x == 0) {
    a.bcount0[blockIdx.x] = t0;
    a.bcount1[blockIdx.x] = t1;
  }
}

__global__ void __launch_bounds__(kThreads) push_list_kernel(ListArgs a) {
  __shared__ int wcnt[kThreads / 64];
  __shared__ int red[kThreads / 64];
  __shared__ long long off[2];
  if (*a.dense) return;
  // block offsets: the counts of the blocks before this one (block-wide sums)
  int p0 = 0, p1 = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kThreads) {
    p0 += a.bcount0[b];
    if (a.split_long) p1 += a.bcount1[b];
  }
  const int o0 = block_sum_int(p0, red);
  const int o1 = block_sum_int(p1, red);
  if (threadIdx.x == 0) {
    off[0] = o0;
    off[1] = o1;
    if (blockIdx.x == gridDim.x - 1) {
      *a.count0 = (long long)o0 + a.bcount0[blockIdx.x];
      if (a.split_long) *a.count1 = (long long)o1 + a.bcount1[blockIdx.x];
    }
  }
  __syncthreads();
  int64_t lo, hi;
  block_range(a.n, lo, hi);
  int64_t b0 = off[0], b1 = off[1];
  for (int64_t v0 = lo; v0 < hi; v0 += kThreads) {  // rounds are uniform across the block
    const int64_t v = v0 + threadIdx.x;
    const bool hit = v < hi && listed(a, v);
    const bool longrow = hit && a.split_long && a.deg[v] > kShortRow;
    const int64_t p0 = block_place(hit && !longrow, wcnt, b0);
    const int64_t p1 = block_place(longrow, wcnt, b1);
    if (p0 >= 0) a.list0[p0] = (int32_t)v;
    if (p1 >= 0) a.list1[p1] = (int32_t)v;
  }
}

struct MarkArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* slist;
  const long long* scount;
  int32_t* mark;
  int32_t k;
  const long long* dense;  // set: no marks
};

__global__ void __launch_bounds__(kThreads) push_mark_kernel(MarkArgs a) {
  __shared__ long long pre[kChunk];  // inclusive prefix sum of the chunk's degrees
  __shared__ int64_t off[kChunk];
  if (*a.dense) return;
  const long long m = *a.scount;
  const int tid = threadIdx.x;
  for (long long chunk = blockIdx.x; chunk * kChunk < m; chunk += gridDim.x) {
    const long long i = chunk * kChunk + tid;
    long long d = 0;
    if (i < m) {
      const int32_t u = a.slist[i];
      off[tid] = a.row_ptr[u];
      d = a.row_ptr[u + 1] - off[tid];
    }
    pre[tid] = d;
    __syncthreads();
    for (int step = 1; step < kChunk; step <<= 1) {  // Hillis-Steele scan in LDS
      const long long add = tid >= step ? pre[tid - step] : 0;
      __syncthreads();
      pre[tid] += add;
      __syncthreads();
    }
    const long long total = pre[kChunk - 1];
    for (long long e = tid; e < total; e += kChunk) {
      int lo = 0, hi = kChunk - 1;  // first entry whose inclusive prefix exceeds e
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] > e) hi = mid; else lo = mid + 1;
      }
      const long long before = lo ? pre[lo - 1] : 0;
      a.mark[a.col_idx[off[lo] + (e - before)]] = a.k;
    }
    __syncthreads();
  }
}

// Bitmap of S_k (bit u of word u / 32), for the sparse pulls.
struct BitsArgs {
  int64_t n;
  const int32_t* sel;
  int32_t k;
  uint32_t* bits;
  const long long* dense;
};

__global__ void __launch_bounds__(kThreads) push_bits_kernel(BitsArgs a) {
  if (*a.dense) return;
  // each wavefront turns 64 consecutive nodes into two bitmap words
  const int lane = threadIdx.x & 63;
  const int64_t chunks = (a.n + 63) / 64;
  const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
  for (int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); c < chunks; c += waves) {
    const int64_t v = c * 64 + lane;
    const unsigned long long m = __ballot(v < a.n && a.sel[v] == a.k);
    const int64_t w = 2 * c + lane;
    if (lane < 2 && w * 32 < a.n) a.bits[w] = (uint32_t)(m >> (32 * lane));
  }
}

__device__ __forceinline__ bool in_set(const uint32_t* bits, int32_t u) { return (bits[u >> 5] >> (u & 31)) & 1u; }

// The pulls add pv(u) only for u in S_k: every other pv is zero, so the
// sum over the row is the same, and the bit test reads a bitmap that stays
// in L2 instead of gathering pv.
struct PullArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* pv;
  const uint32_t* bits;  // S_k
  double* r;  // r_new
  const int32_t* list;  // marked rows of the class
  const long long* count;
  const long long* dense;  // set: the dense step pulls this iteration instead
};

// Short rows: one thread per row, arcs summed in CSR order (four loads in
// flight, added in order).
__global__ void __launch_bounds__(kThreads) push_pull_short_kernel(PullArgs a) {
  if (*a.dense) return;
  const int32_t* list = a.list;
  const long long m = *a.count;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int32_t v = list[i];
    const int64_t pe = a.row_ptr[v + 1];
    int64_t p = a.row_ptr[v];
    double acc = 0.0;
    for (; p + 4 <= pe; p += 4) {
      const int32_t u0 = a.col_idx[p], u1 = a.col_idx[p + 1], u2 = a.col_idx[p + 2], u3 = a.col_idx[p + 3];
      const bool b0 = in_set(a.bits, u0), b1 = in_set(a.bits, u1), b2 = in_set(a.bits, u2), b3 = in_set(a.bits, u3);
      if (b0) acc += a.pv[u0];
      if (b1) acc += a.pv[u1];
      if (b2) acc += a.pv[u2];
      if (b3) acc += a.pv[u3];
    }
    for (; p < pe; ++p) {
      const int32_t u = a.col_idx[p];
      if (in_set(a.bits, u)) acc += a.pv[u];
    }
    a.r[v] += acc;
  }
}

// Long rows: one workgroup per row; thread t sums arcs t, t + 256, ... in
// order (four loads in flight), then a fixed wave butterfly and an ordered
// sum of the four wave totals.
__global__ void __launch_bounds__(kThreads) push_pull_long_kernel(PullArgs a) {
  __shared__ double wsum[kThreads / 64];
  if (*a.dense) return;
  const int32_t* list = a.list;
  const long long m = *a.count;
  const int tid = threadIdx.x;
  for (long long i = blockIdx.x; i < m; i += gridDim.x) {
    const int32_t v = list[i];
    const int64_t pb = a.row_ptr[v], pe = a.row_ptr[v + 1];
    double acc = 0.0;
    int64_t p = pb + tid;
    for (; p + 3 * kThreads < pe; p += 4 * kThreads) {
      const int32_t u0 = a.col_idx[p], u1 = a.col_idx[p + kThreads];
      const int32_t u2 = a.col_idx[p + 2 * kThreads], u3 = a.col_idx[p + 3 * kThreads];
      const bool b0 = in_set(a.bits, u0), b1 = in_set(a.bits, u1), b2 = in_set(a.bits, u2), b3 = in_set(a.bits, u3);
      if (b0) acc += a.pv[u0];
      if (b1) acc += a.pv[u1];
      if (b2) acc += a.pv[u2];
      if (b3) acc += a.pv[u3];
    }
    for (; p < pe; p += kThreads) {
      const int32_t u = a.col_idx[p];
      if (in_set(a.bits, u)) acc += a.pv[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int q = 0; q < kThreads / 64; ++q) t += wsum[q];
      a.r[v] += t;
    }
    __syncthreads();
  }
}

struct PushFinalArgs {
  const int64_t* row_ptr;
  const int32_t* perm;
  int64_t n;
  const double* y;
  double* out;
  double oexp, oscale;  // out = oscale d^oexp y (Def. 8 output space: -a, d_s^a)
  double* block_sums;   // or null
};

__global__ void __launch_bounds__(kThreads) push_final_kernel(PushFinalArgs a) {
  double local = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int64_t d = a.row_ptr[v + 1] - a.row_ptr[v];
    double z = 0.0;
    if (d > 0) z = a.oexp == 0.0 && a.oscale == 1.0 ? a.y[v] : a.oscale * pow((double)d, a.oexp) * a.y[v];
    a.out[a.perm ? a.perm[v] : v] = z;
    local += z;
  }
  if (a.block_sums) {
    __shared__ double ws[kThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < kThreads / 64; ++q) t += ws[q];
      a.block_sums[1 + blockIdx.x] = t;
    }
  }
}

__global__ void push_sum_kernel(double* sums, int nb) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < nb; ++i) t += sums[1 + i];
    sums[0] = t;
  }
}

__global__ void rw_zero_counts_kernel(long long* c) {
  if (threadIdx.x < 8) c[threadIdx.x] = 0;
}

// ---------------------------------------------------------------- Alg. 5

// SplitMix64 (Steele, Lea & Flood, 2014): output c (0-based) of the stream
// whose state starts at `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int64_t kMaxWalkSteps = 1ll << 20;

// pv(u) = pi^(u) / d_u written as (1 / d_u) * pi^(u), the entry of P times
// pi^, for every node (the dense step then forms P pi^).
struct ScaleArgs {
  int64_t n;
  const int32_t* deg;
  const double* y;
  double* pv;
  double* acc;  // zeroed: receives P pi^
};

__global__ void __launch_bounds__(kThreads) rw_scale_kernel(ScaleArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int32_t d = a.deg[v];
    a.pv[v] = d > 0 ? (1.0 / (double)d) * a.y[v] : 0.0;
    a.acc[v] = 0.0;
  }
}

// r(v) = [v = s] - (pi^(v) - (1 - alpha) (P pi^)(v)) / alpha, the walk count
// W_v = ceil(|r(v)| W) and its per-block sums (nodes, walks).
struct ResidualArgs {
  int64_t n;
  int64_t s;
  double alpha, W;
  const double* y;
  const double* acc;
  double* res;
  long long* wv;
  int32_t* bnodes;
  long long* bwalks;
};

__global__ void __launch_bounds__(kThreads) rw_residual_kernel(ResidualArgs a) {
  __shared__ int red[kThreads / 64];
  __shared__ long long redl[kThreads / 64];
  int64_t lo, hi;
  block_range(a.n, lo, hi);
  int nodes = 0;
  long long walks = 0;
  for (int64_t v = lo + threadIdx.x; v < hi; v += kThreads) {
    const double r = (v == a.s ? 1.0 : 0.0) - (a.y[v] - (1.0 - a.alpha) * a.acc[v]) / a.alpha;
    a.res[v] = r;
    long long c = 0;
    if (r != 0.0) {
      c = (long long)ceil(fabs(r) * a.W);
      ++nodes;
    }
    a.wv[v] = c;
    walks += c;
  }
  const int tn = block_sum_int(nodes, red);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) walks += __shfl_xor(walks, o, 64);
  if ((threadIdx.x & 63) == 0) redl[threadIdx.x >> 6] = walks;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int q = 0; q < kThreads / 64; ++q) t += redl[q];
    a.bnodes[blockIdx.x] = tn;
    a.bwalks[blockIdx.x] = t;
  }
}

// Start nodes in node order with the exclusive prefix of their walk counts.
struct WalkListArgs {
  int64_t n;
  const long long* wv;
  const int32_t* bnodes;
  const long long* bwalks;
  int32_t* starts;
  long long* first;   // first walk index of each start node
  long long* nstart;  // number of start nodes
  long long* nwalks;  // total walks
};

__global__ void __launch_bounds__(kThreads) rw_list_kernel(WalkListArgs a) {
  __shared__ int wcnt[kThreads / 64];
  __shared__ int red[kThreads / 64];
  __shared__ long long redl[kThreads / 64];
  __shared__ long long wscan[kThreads];
  int p0 = 0;
  long long q0 = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kThreads) {
    p0 += a.bnodes[b];
    q0 += a.bwalks[b];
  }
  const int node_off = block_sum_int(p0, red);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) q0 += __shfl_xor(q0, o, 64);
  if ((threadIdx.x & 63) == 0) redl[threadIdx.x >> 6] = q0;
  __syncthreads();
  long long walk_off = 0;
  for (int q = 0; q < kThreads / 64; ++q) walk_off += redl[q];
  __syncthreads();
  if (threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) {
    *a.nstart = (long long)node_off + a.bnodes[blockIdx.x];
    *a.nwalks = walk_off + a.bwalks[blockIdx.x];
  }
  int64_t lo, hi;
  block_range(a.n, lo, hi);
  int64_t base = node_off;
  for (int64_t v0 = lo; v0 < hi; v0 += kThreads) {  // rounds are uniform across the block
    const int64_t v = v0 + threadIdx.x;
    const long long c = v < hi ? a.wv[v] : 0;
    // inclusive scan of the round's walk counts in thread order
    wscan[threadIdx.x] = c;
    __syncthreads();
    for (int step = 1; step < kThreads; step <<= 1) {
      const long long add = threadIdx.x >= step ? wscan[threadIdx.x - step] : 0;
      __syncthreads();
      wscan[threadIdx.x] += add;
      __syncthreads();
    }
    const long long incl = wscan[threadIdx.x], round_total = wscan[kThreads - 1];
    const int64_t pos = block_place(c > 0, wcnt, base);
    if (pos >= 0) {
      a.starts[pos] = (int32_t)v;
      a.first[pos] = walk_off + incl - c;
    }
    walk_off += round_total;
    __syncthreads();
  }
}

struct WalkArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* perm;    // internal -> caller id (the walk streams are keyed by caller id), or null
  const int32_t* starts;
  const long long* first;
  const long long* nstart;
  const long long* nwalks;
  const long long* wv;
  const double* res;
  double alpha;
  uint64_t seed;
  double* y;
  long long* steps;
};

__global__ void __launch_bounds__(kThreads) rw_walk_kernel(WalkArgs a) {
  const long long T = *a.nwalks, S = *a.nstart;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long my_steps = 0;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += stride) {
    long long lo = 0, hi = S - 1;  // last start whose first walk is <= t
    while (lo < hi) {
      const long long mid = (lo + hi + 1) >> 1;
      if (a.first[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int32_t v = a.starts[lo];
    const uint64_t j = (uint64_t)(t - a.first[lo]);
    const uint64_t key = splitmix64(a.seed, (uint64_t)(a.perm ? a.perm[v] : v));
    int32_t cur = v;
    for (int64_t step = 0; step < kMaxWalkSteps; ++step) {
      const uint64_t x = splitmix64(key, (j << 32) + 2ull * (uint64_t)step);
      if ((double)(x >> 11) * 0x1.0p-53 < a.alpha) break;
      const int64_t p0 = a.row_ptr[cur], d = a.row_ptr[cur + 1] - p0;
      const uint64_t x2 = splitmix64(key, (j << 32) + 2ull * (uint64_t)step + 1ull);
      cur = a.col_idx[p0 + (int64_t)__umul64hi(x2, (uint64_t)d)];
      ++my_steps;
    }
    unsafeAtomicAdd(a.y + cur, a.res[v] / (double)a.wv[v]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) my_steps += __shfl_xor(my_steps, o, 64);
  if ((threadIdx.x & 63) == 0 && my_steps) atomicAdd((unsigned long long*)a.steps, (unsigned long long)my_steps);
}

struct RwLayout {
  PushLayout push;
  size_t res, wv, starts, first, bnodes, bwalks, counts, total;
};

RwLayout rw_layout(const cp_graph* g) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t n = (size_t)g->n;
  RwLayout L{};
  L.push = push_layout(g);
  size_t off = L.push.total;
  L.res = off; off += al(n * 8);
  L.wv = off; off += al(n * 8);
  L.starts = off; off += al(n * 4);
  L.first = off; off += al(n * 8);
  L.bnodes = off; off += al((size_t)kRangeBlocks * 4);
  L.bwalks = off; off += al((size_t)kRangeBlocks * 8);
  L.counts = off; off += al(8 * 8);  // [0] start nodes, [1] walks, [2] walk steps
  L.total = off;
  return L;
}

// r += sum over each row of pv (every row), by the single-source step
// kernels in their add mode; with a gate, only while *gate != 0.
hipError_t dense_pull(const cp_graph* g, const double* pv, double* r, char* w, const PushLayout& L,
                      const long long* gate, hipStream_t st) {
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
    ga.x = pv;
    ga.partial = w + L.part;
    ga.gate = gate;
    hipError_t e = launch_stripe_gather(CP_F64, ga, st);
    if (e != hipSuccess) return e;
    const CombineArgs ca{g->row_ptr, g->n, w + L.part, g->s_count, r, nullptr, 0.0, gate};
    return launch_stripe_combine(CP_F64, ca, kStepAdd, st);
  }
  StepArgs sa{};
  sa.row_ptr = g->row_ptr;
  sa.col_idx = g->col_idx;
  sa.blocks = g->single.blocks;
  sa.hubs = g->single.hubs;
  sa.nblocks = g->single.nblocks;
  sa.nspecial = g->single.nspecial;
  sa.x = pv;
  sa.z = r;
  sa.hub_partial = w + L.part;
  sa.hub_count = reinterpret_cast<int32_t*>(w + L.hubc);
  sa.gate = gate;
  return launch_step(CP_F64, sa, kStepAdd, st);
}

// The push phase of Alg. 4 into the workspace: y (internal order, paper
// space) and the push counters.  Launches only; errors as hipError_t.
hipError_t push_phase(const cp_graph* g, const QueryPlan& qp, double eps_a, char* w, const PushLayout& L,
                      hipStream_t st) {
  const int32_t K = qp.K;
  const std::vector<double>& c = qp.c;
  // eps_k = eps_a / (4 K sum_{l=k}^{K} |c_l|), Alg. 4 (a zero tail: nothing
  // left to weight, so nothing is pushed)
  std::vector<double> eps(K + 1, 0.0);
  {
    double tail = 0.0;
    for (int32_t l = K; l >= 1; --l) {
      tail += std::fabs(c[l]);
      eps[l] = tail > 0.0 ? eps_a / (4.0 * K * tail) : std::numeric_limits<double>::infinity();
    }
  }
  hipError_t e = launch_zero(w, L.sums, st);
  if (e != hipSuccess) return e;
  double* rbuf[2] = {reinterpret_cast<double*>(w + L.r[0]), reinterpret_cast<double*>(w + L.r[1])};
  double* yv = reinterpret_cast<double*>(w + L.y);
  double* pv = reinterpret_cast<double*>(w + L.pv);
  int32_t* deg = reinterpret_cast<int32_t*>(w + L.deg);
  int32_t* sel = reinterpret_cast<int32_t*>(w + L.sel);
  int32_t* mark = reinterpret_cast<int32_t*>(w + L.mark);
  int32_t* slist = reinterpret_cast<int32_t*>(w + L.slist);
  int32_t* tshort = reinterpret_cast<int32_t*>(w + L.tshort);
  int32_t* tlong = reinterpret_cast<int32_t*>(w + L.tlong);
  int32_t* bc = reinterpret_cast<int32_t*>(w + L.bcount);
  long long* counts = reinterpret_cast<long long*>(w + L.counts);
  long long* bvol = reinterpret_cast<long long*>(w + L.bvol);
  uint32_t* bits = reinterpret_cast<uint32_t*>(w + L.bits);
  const dim3 rb(kRangeBlocks), eb(kEdgeBlocks), tb(kThreads);
#define CP_LAUNCH(...)                       \
  do {                                       \
    hipLaunchKernelGGL(__VA_ARGS__);         \
    const hipError_t e_ = hipGetLastError(); \
    if (e_ != hipSuccess) return e_;         \
  } while (0)
  CP_LAUNCH(push_degree_kernel, rb, tb, 0, st, DegreeArgs{g->row_ptr, g->n, deg});
  CP_LAUNCH(push_seed_kernel, dim3(1), tb, 0, st,
            SeedArgs{g->row_ptr, g->col_idx, qp.s_int, c[0], rbuf[0], rbuf[1], yv});
  int cur = 0;  // rbuf[cur] is r_cur
  for (int32_t k = 1; k < K; ++k) {
    const int nxt = cur ^ 1;
    CP_LAUNCH(push_select_kernel, rb, tb, 0, st,
              SelectArgs{g->n, deg, rbuf[cur], yv, pv, sel, k, eps[k], c[k], bc, bvol});
    CP_LAUNCH(push_decide_kernel, dim3(1), tb, 0, st, DecideArgs{g->n, g->nnz, bc, bvol, counts});
    const ListArgs ls{g->n, sel, deg, k, 0, bc, bc + kRangeBlocks, slist, slist, counts + 0, counts + 0,
                      counts + 5};
    CP_LAUNCH(push_list_kernel, rb, tb, 0, st, ls);
    CP_LAUNCH(push_mark_kernel, eb, tb, 0, st,
              MarkArgs{g->row_ptr, g->col_idx, slist, counts + 0, mark, k, counts + 5});
    const ListArgs lt{g->n, mark, deg, k, 1, bc + kRangeBlocks, bc + 2 * kRangeBlocks, tshort, tlong,
                      counts + 1, counts + 2, counts + 5};
    CP_LAUNCH(push_count_kernel, rb, tb, 0, st, lt);
    CP_LAUNCH(push_list_kernel, rb, tb, 0, st, lt);
    CP_LAUNCH(push_bits_kernel, rb, tb, 0, st, BitsArgs{g->n, sel, k, bits, counts + 5});
    CP_LAUNCH(push_pull_short_kernel, eb, tb, 0, st,
              PullArgs{g->row_ptr, g->col_idx, pv, bits, rbuf[nxt], tshort, counts + 1, counts + 5});
    CP_LAUNCH(push_pull_long_kernel, eb, tb, 0, st,
              PullArgs{g->row_ptr, g->col_idx, pv, bits, rbuf[nxt], tlong, counts + 2, counts + 5});
    e = dense_pull(g, pv, rbuf[nxt], w, L, counts + 5, st);
    if (e != hipSuccess) return e;
    cur = nxt;
  }
  return hipSuccess;
}

// Alg. 5's second phase on top of push_phase's y: the residual (one pull
// over every row), the walk list, the walks.
hipError_t rw_phase(const cp_graph* g, const QueryPlan& qp, double alpha, double W, uint64_t seed, char* w,
                    const RwLayout& L, hipStream_t st) {
  const PushLayout& P = L.push;
  double* yv = reinterpret_cast<double*>(w + P.y);
  double* pv = reinterpret_cast<double*>(w + P.pv);
  double* acc = reinterpret_cast<double*>(w + P.r[0]);
  int32_t* deg = reinterpret_cast<int32_t*>(w + P.deg);
  long long* rc = reinterpret_cast<long long*>(w + L.counts);
  const dim3 rb(kRangeBlocks), tb(kThreads);
  CP_LAUNCH(rw_zero_counts_kernel, dim3(1), dim3(64), 0, st, rc);
  CP_LAUNCH(rw_scale_kernel, rb, tb, 0, st, ScaleArgs{g->n, deg, yv, pv, acc});
  {
    const hipError_t e = dense_pull(g, pv, acc, w, P, nullptr, st);
    if (e != hipSuccess) return e;
  }
  double* res = reinterpret_cast<double*>(w + L.res);
  long long* wv = reinterpret_cast<long long*>(w + L.wv);
  int32_t* bnodes = reinterpret_cast<int32_t*>(w + L.bnodes);
  long long* bwalks = reinterpret_cast<long long*>(w + L.bwalks);
  CP_LAUNCH(rw_residual_kernel, rb, tb, 0, st,
            ResidualArgs{g->n, qp.s_int, alpha, W, yv, acc, res, wv, bnodes, bwalks});
  int32_t* starts = reinterpret_cast<int32_t*>(w + L.starts);
  long long* first = reinterpret_cast<long long*>(w + L.first);
  CP_LAUNCH(rw_list_kernel, rb, tb, 0, st, WalkListArgs{g->n, wv, bnodes, bwalks, starts, first, rc + 0, rc + 1});
  CP_LAUNCH(rw_walk_kernel, dim3(4096), tb, 0, st,
            WalkArgs{g->row_ptr, g->col_idx, g->perm, starts, first, rc + 0, rc + 1, wv, res, alpha, seed, yv,
                     rc + 2});
  return hipSuccess;
}
#undef CP_LAUNCH

}  // namespace
}  // namespace cp

using namespace cp;

extern "C" {

size_t cp_push_workspace_bytes(const cp_graph* g) { return g ? push_layout(g).total : 0; }

size_t cp_push_rw_workspace_bytes(const cp_graph* g) { return g ? rw_layout(g).total : 0; }

}  // extern "C"

namespace {

// Shared tail of cp_push and cp_push_rw: output in caller ids (and the
// Def. 8 space), optional mass, counters, timing.
cp_status push_finish(const cp_graph* g, const cp_query* q, const QueryPlan& qp, char* w, const PushLayout& L,
                      const long long* rw_counts, double* y, hipStream_t st, hipEvent_t* ev, cp_info* info) {
  const bool stats = q->flags & CP_Q_STATS;
  const bool timing = q->flags & CP_Q_TIMING;
  double* sums = reinterpret_cast<double*>(w + L.sums);
  const double* yv = reinterpret_cast<const double*>(w + L.y);
  PushFinalArgs fa{g->row_ptr, g->perm, g->n, yv, y, -q->a, qp.oscale, stats ? sums : nullptr};
  hipLaunchKernelGGL(push_final_kernel, dim3(kRangeBlocks), dim3(kThreads), 0, st, fa);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && stats) {
    hipLaunchKernelGGL(push_sum_kernel, dim3(1), dim3(64), 0, st, sums, kRangeBlocks);
    e = hipGetLastError();
  }
  if (e == hipSuccess && timing) e = hipEventRecord(ev[3], st);
  if (e != hipSuccess) { set_hip_error(e); return CP_EHIP; }
  if (info) {
    info->K = qp.K;
    info->steps = qp.K - 1;
    info->tail = qp.tail;
    info->tail_bound_l1 = NAN;  // ChebyPush's guarantee is the degree-normalised eps_a (Thm. 4)
    info->mass = NAN;
    info->elapsed_ms = NAN;
    info->step_ms = NAN;
    info->latency_ms = NAN;
    info->wait_ms = NAN;
    info->pushes = -1;
    info->arcs = -1;
    info->walks = rw_counts ? -1 : 0;
    info->walk_steps = rw_counts ? -1 : 0;
  }
  if (!(stats || timing)) return CP_OK;
  e = hipStreamSynchronize(st);
  long long host[kCounts] = {0}, rwh[8] = {0};
  if (e == hipSuccess) e = hipMemcpy(host, w + L.counts, sizeof(host), hipMemcpyDeviceToHost);
  if (e == hipSuccess && rw_counts) e = hipMemcpy(rwh, rw_counts, sizeof(rwh), hipMemcpyDeviceToHost);
  double m = NAN;
  if (e == hipSuccess && stats) e = hipMemcpy(&m, sums, sizeof(double), hipMemcpyDeviceToHost);
  float ms_all = NAN, ms_loop = NAN;
  if (e == hipSuccess && timing) e = hipEventElapsedTime(&ms_all, ev[0], ev[3]);
  if (e == hipSuccess && timing) e = hipEventElapsedTime(&ms_loop, ev[1], ev[2]);
  if (e != hipSuccess) { set_hip_error(e); return CP_EHIP; }
  if (info) {
    info->pushes = host[3];
    info->arcs = host[4];
    if (rw_counts) {
      info->walks = rwh[1];
      info->walk_steps = rwh[2];
    }
    if (stats) info->mass = m;
    if (timing) {
      info->elapsed_ms = ms_all;
      info->step_ms = ms_loop;
    }
  }
  return CP_OK;
}

struct Events {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  ~Events() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t create() {
    for (auto& e : ev) {
      const hipError_t x = hipEventCreate(&e);
      if (x != hipSuccess) return x;
    }
    return hipSuccess;
  }
};

}  // namespace

extern "C" {

cp_status cp_push(const cp_graph* g, const cp_query* q, double eps_a, double* y, void* ws, size_t ws_bytes,
                  void* stream, cp_info* info) {
  if (!g || !q || !y || !(eps_a >= 0.0 && std::isfinite(eps_a))) return CP_EINVAL;
  if (q->flags & CP_Q_PWMETHOD) return CP_EINVAL;
  QueryPlan qp;
  cp_status rc = plan_query(g, q, kDefaultKMax, &qp);
  if (rc != CP_OK) return rc;
  const PushLayout L = push_layout(g);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return CP_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const bool timing = q->flags & CP_Q_TIMING;
  Events E;
  hipError_t e = timing ? E.create() : hipSuccess;
  if (e == hipSuccess && timing) e = hipEventRecord(E.ev[0], st);
  if (e == hipSuccess && timing) e = hipEventRecord(E.ev[1], st);
  if (e == hipSuccess) e = push_phase(g, qp, eps_a, w, L, st);
  if (e == hipSuccess && timing) e = hipEventRecord(E.ev[2], st);
  if (e != hipSuccess) { set_hip_error(e); return CP_EHIP; }
  return push_finish(g, q, qp, w, L, nullptr, y, st, E.ev, info);
}

cp_status cp_push_rw(const cp_graph* g, const cp_query* q, double eps_r, double delta, double r_max,
                     uint64_t seed, double* y, void* ws, size_t ws_bytes, void* stream, cp_info* info) {
  if (!g || !q || !y || q->kind != CP_PPR || (q->flags & CP_Q_PWMETHOD)) return CP_EINVAL;
  if (!(eps_r > 0.0 && std::isfinite(eps_r)) || !(delta > 0.0 && delta < 1.0) || !(r_max >= 0.0)) return CP_EINVAL;
  const double alpha = q->param;
  if (!(alpha > 0.0 && alpha < 1.0)) return CP_EINVAL;
  // W and r_max of Alg. 5 (log read as natural); r_max > 0 overrides
  const double W = 2.0 * (2.0 * eps_r / 3.0 + 2.0) * std::log((double)g->n) / (eps_r * eps_r * delta);
  if (!(W >= 1.0 && W < 9.0e18)) return CP_EINVAL;
  const double rmax = r_max > 0.0 ? r_max : std::sqrt(alpha) / W;
  cp_query qk = *q;
  qk.tol = std::min(rmax, 0.5);  // the truncation rules read the threshold as their tolerance
  QueryPlan qp;
  cp_status rc = plan_query(g, &qk, kDefaultKMax, &qp);
  if (rc != CP_OK) return rc;
  const RwLayout L = rw_layout(g);
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return CP_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const bool timing = q->flags & CP_Q_TIMING;
  Events E;
  hipError_t e = timing ? E.create() : hipSuccess;
  if (e == hipSuccess && timing) e = hipEventRecord(E.ev[0], st);
  if (e == hipSuccess && timing) e = hipEventRecord(E.ev[1], st);
  if (e == hipSuccess) e = push_phase(g, qp, rmax, w, L.push, st);
  if (e == hipSuccess && timing) e = hipEventRecord(E.ev[2], st);
  if (e == hipSuccess) e = rw_phase(g, qp, alpha, W, seed, w, L, st);
  if (e != hipSuccess) { set_hip_error(e); return CP_EHIP; }
  return push_finish(g, q, qp, w, L.push, reinterpret_cast<const long long*>(w + L.counts), y, st, E.ev, info);
}

}  // extern "C"
