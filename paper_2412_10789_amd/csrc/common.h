// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "chebyprop.h"

namespace cp {

// ---------------------------------------------------------------- work plan
//
// The step kernel walks the CSR in "blocks", one workgroup each:
//   kind 0 (stream): a run of consecutive rows whose arcs fit in one LDS
//          tile (at most kTileNnz arcs and kTileRows rows);
//   kind 1 (long):   one row with more than kTileNnz arcs, streamed from
//          global memory by the whole workgroup;
//   kind 2 (hub):    one segment of kHubSeg arcs of a row with more than
//          kHubThreshold arcs; the segments' partial sums are combined in
//          segment order by whichever workgroup finishes its row last.
// Blocks are ordered hubs, long rows (longest first), then stream blocks in
// row order.

constexpr int kThreads = 256;      // workgroup size (4 wave64)
constexpr int kTileNnz = 2048;     // arcs per stream tile (8 per thread)
constexpr int kTileRows = 256;     // rows per stream tile (1 per thread)
constexpr int kPerThread = kTileNnz / kThreads;
constexpr int64_t kHubThreshold = 16384;
constexpr int64_t kHubSeg = 8192;
constexpr int64_t kBatchLong = 256;  // batched kernel: rows above this use the whole workgroup
constexpr int kMaxUploadWords = 960; // 32-bit words per kernel-argument upload launch

enum BlockKind : int32_t { kStream = 0, kLong = 1, kHub = 2 };

struct BlockDesc {
  int32_t r0;    // first row
  int32_t r1;    // one past the last row (stream, long); hub id (hub)
  int32_t kind;  // BlockKind
  int32_t aux;   // stream: arc count; hub: segment index within the row
  int64_t p0;    // stream: CSR offset of the tile's first arc (so the column
                 // stream starts without waiting for the row offsets)
  int64_t pad;
};

struct HubDesc {
  int32_t row;
  int32_t nseg;
  int32_t base;  // index of segment 0 in the partial-sum array
  int32_t seg;   // arcs per segment (the last one may hold fewer)
};

// Row-split parameters of a work plan: rows above long_cut arcs leave the
// stream tiles (at most kTileNnz: a stream tile's arcs sit in LDS), rows
// above hub_cut arcs are split into segments of hub_seg arcs.
struct PlanShape {
  int64_t long_cut;
  int64_t hub_cut = kHubThreshold;
  int64_t hub_seg = kHubSeg;
};

struct Plan {
  std::vector<BlockDesc> blocks;
  std::vector<HubDesc> hubs;
  int64_t nspecial = 0;  // hub + long blocks at the front
  int64_t nlong = 0;
  int64_t hub_segments = 0;
  PlanShape shape{kTileNnz};
};

// The default long_cut is kTileNnz for the single-source kernel and
// kBatchLong for the batched one; the autotuner tries others.
Plan build_plan(const int64_t* row_ptr, int64_t n, const PlanShape& shape);

// Plan as uploaded to the device.
struct DevPlan {
  BlockDesc* blocks = nullptr;
  HubDesc* hubs = nullptr;
  int64_t nblocks = 0, nspecial = 0, nlong = 0, nhubs = 0, hub_segments = 0;
  PlanShape shape{kTileNnz};
};

// ------------------------------------------------------------ XCD stripes
//
// With CP_GRAPH_XCD_STRIPES the nodes are relabelled so that degree rank r
// goes to stripe r % S, position r / S: S contiguous id ranges of equal
// size and (statistically) equal arc mass, each degree-ordered, S in
// {2, 4, 8} (stripe_count).  Each stripe's arcs are also stored as a CSR of
// their own (all rows, columns in that stripe only).  A Chebyshev step then
// runs as
//   1. stripe kernel: workgroup w = S t + j handles row tile t restricted
//      to stripe j; workgroups are dispatched round-robin over the 8 XCDs,
//      so stripe j is only ever gathered on XCDs j, j + S, ... and its slice
//      of x stays in their L2; each writes the partial row sums of its
//      stripe;
//   2. combine kernel: the S partials of every row are added in stripe
//      order and the recurrence / estimate update is applied.
// Fewer stripes mean fewer partials to write and read; more stripes mean a
// smaller slice per L2.  stripe_count picks the fewest whose FP32 slice
// fits one XCD's 4 MiB L2 (at least 2, at most 8).

constexpr int kMaxStripes = 8;
constexpr int64_t kStripeSliceBytes = int64_t(4) << 20;
inline int32_t stripe_count(int64_t n) {
  int32_t s = 2;
  while (s < kMaxStripes && n * 4 > kStripeSliceBytes * s) s *= 2;
  return s;
}
constexpr int kStripeTileNnz = 2048;   // arcs per (tile, stripe)
constexpr int kPackPosBits = 11;       // position of an arc within its tile block
constexpr int kPackLocalBits = 32 - kPackPosBits;
static_assert(kStripeTileNnz <= (1 << kPackPosBits), "tile positions must fit the packed form");
constexpr int kStripeTileRows = 1000;  // rows per tile (keeps 8 workgroups per CU in LDS)

// One workgroup of the striped step: rows [r0, r0 + nr) of the tile,
// restricted to stripe (block index % S), whose arcs are cols[p0, p0 + cnt)
// of that stripe's CSR.  cnt > kStripeTileNnz marks a single long row
// streamed by the whole workgroup.
//
// Packed form (used when every stripe holds at most 2^kPackLocalBits
// nodes): the arcs of a tile block (cnt <= kStripeTileNnz) are stored sorted by
// column, each as (column - stripe start) << kPackPosBits | its position in
// the block's CSR order, so that arcs of different rows that share a column
// sit in the same wave's load and the hardware merges them into one cache
// request; the gathered value is put back at its CSR position in LDS, so the
// row sums are the same, bit for bit, as in CSR order.  Long-row blocks keep
// plain column ids.
struct StripeBlock {
  int32_t r0, nr;
  int32_t p0, cnt;
};

// Row update of a step (all step kernels): the Chebyshev step of Eq. 6,
// z = 2 acc / d - z; the power step of Alg. 1, z = acc / d; or the pull of
// ChebyPush's push form (Alg. 4, Sec. 4.2), z += acc with x the push values
// 2 r(u) / d_u (FP64 only, no estimate update).
enum StepMode : int32_t { kStepCheb = 0, kStepPower = 1, kStepAdd = 2 };

struct StripeArgs {
  const int32_t* rp;                // [S][n+1] per-stripe row offsets
  const int32_t* cols;              // stripe CSRs, concatenated
  int64_t col_off[kMaxStripes];     // start of stripe j's columns in cols
  int64_t base[kMaxStripes];        // first node of stripe j (packed form)
  int32_t packed;                   // tile blocks hold the packed form
  int32_t nstripes;                 // S
  const StripeBlock* blocks;        // [ntiles * S], block index = S * tile + stripe
  int64_t ntiles;
  int64_t n;
  const void* x;
  void* partial;                    // Acc[S][n]
  const long long* gate;            // non-null: the launch does nothing while *gate == 0
};
hipError_t launch_stripe_gather(int32_t prec, const StripeArgs& a, hipStream_t st);

struct CombineArgs {
  const int64_t* row_ptr;
  int64_t n;
  const void* partial;              // Acc[S][n]
  int32_t nstripes;                 // S
  void* z;
  void* yacc;
  double c;
  const long long* gate;            // as StripeArgs
};
hipError_t launch_stripe_combine(int32_t prec, const CombineArgs& a, StepMode mode, hipStream_t st);

// ------------------------------------------------------------------ kernels

// Chebyshev step over all blocks: for every row v
//   acc = sum_{u in N(v)} x[u]            (x = D^{-1} r_k)
//   z[v] = 2 acc / d_v - z[v]             (z: D^{-1} r_{k-1} -> D^{-1} r_{k+1})
//   yacc[v] += c * z[v]                   (yacc = D^{-1} y)
// The mode selects the row update (see StepMode).
struct StepArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const BlockDesc* blocks;
  const HubDesc* hubs;
  int64_t nblocks;
  int64_t nspecial;
  const void* x;
  void* z;
  void* yacc;
  double c;
  void* hub_partial;  // Acc[hub_segments]
  int32_t* hub_count; // int32[nhubs], zero between steps
  const long long* gate;  // non-null: the launch does nothing while *gate == 0
};

hipError_t launch_step(int32_t prec, const StepArgs& a, StepMode mode, hipStream_t st);

// Zero-fill `bytes` bytes (multiple of 4) at `p`.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// r~_0 = e_s / d_s, r~_1 = D^{-1} P e_s, yacc = c0 r~_0 + c1 r~_1, for one
// source (s, internal id); buffers already zero.
struct InitArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  int64_t s;
  void* r0;
  void* r1;
  void* yacc;
  double c0, c1;
};
hipError_t launch_init(int32_t prec, const InitArgs& a, hipStream_t st);

// y_out[perm(v)] = oscale * d_v^oexp * yacc[v] (d_v yacc[v] is y = f(P) e_s;
// oexp = 1 - a, oscale = d_s^a give the generalized output of Def. 8);
// optional double sum of the output into *mass.
struct FinalArgs {
  const int64_t* row_ptr;
  const int32_t* perm;  // internal -> caller id, or null
  int64_t n;
  const void* yacc;
  void* y_out;
  double* mass;         // device, or null
  double oexp, oscale;
};
hipError_t launch_finalize(int32_t prec, const FinalArgs& a, hipStream_t st);

// ----------------------------------------------------------- batched kernels
//
// Queries sorted by K (descending) occupy "slots"; slots are grouped into
// source tiles of width bw.  Tile t owns three tile-major matrices
// [n][bw]: two recurrence buffers (storage type) and the estimate
// (accumulator type).  coef is a [(Kmax+1)][nq_pad] table of c_k per slot
// (zero once k exceeds the slot's own K).

// One pass of the batched step over a CSR: its row offsets, columns and
// work plan.
struct BatchPass {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const BlockDesc* blocks;
  const HubDesc* hubs;
  int64_t nblocks;
  int64_t nspecial;
};

// Hot/cold split of the batched step (CP_GRAPH_HOT_SPLIT, degree-ordered
// graphs): `hot` holds the arcs whose column is one of the hot_nodes
// highest-degree nodes (ids below hot_nodes), `cold` the others, each row's
// arcs in the same (column) order as in the graph.  A step runs the hot
// pass, which gathers only from the first hot_nodes rows of x, a slice the
// caches can keep, and stores each row's sum in a partial; then the cold
// pass, which adds its gathers to that partial and applies the row update.
struct BatchSplit {
  BatchPass hot, cold;
  int64_t hot_nodes;
};

struct BatchStepArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const BlockDesc* blocks;
  const HubDesc* hubs;
  int64_t nblocks;
  int64_t nspecial;
  const BatchSplit* split;  // host pointer: non-null runs the hot and cold passes (launch_batch_step)
  const int64_t* deg_rp;    // row offsets the degree d_v comes from (null: row_ptr)
  void* part;               // A[ntiles][n][bw] partial sums of the hot pass (split only)
  int64_t n;
  int32_t bw;
  int32_t ntiles;        // active tiles in this launch (grid.y)
  int32_t nq_pad;
  const void* x;         // tile 0 base of x; tile t at + t*n*bw elements
  void* z;
  void* yacc;
  const double* coef_row;  // coef + (k+1)*nq_pad
  const double* rec;     // [nq_pad] per slot: 2 (Chebyshev step, Eq. 6) or 1 (power step, Alg. 1)
                         // (row 0 of the slot parameters, see kSlotParams)
  void* hub_partial;     // A[hub_segments][nq_pad]
  int32_t* hub_count;    // int32[nhubs][ntiles_total]
  int32_t ntiles_total;
  int32_t mode;          // kBatchForward, kClenshawStep or kClenshawLast
  int32_t lanes;         // 0: every slot of the launched tiles; one of kNarrowLanes below bw:
                         // only the first `lanes` slots of tile 0 (the others hold no query)
};
// Slot counts a narrow launch of a wider tile can update: rows are still bw
// apart, but the lane groups are `lanes` wide and gather lanes * s bytes of
// each row.
constexpr int32_t kNarrowLanes[2] = {8, 16};
// Row update of a batched step.  Forward (Alg. 3 / Alg. 1): z = u acc / d -
// (u - 1) z and yacc += c z.  Clenshaw's backward form of the same series,
// with yacc holding the start vector x~: a step writes b_k = c x~ + u acc / d
// - b_{k+2} over z (u = 2); the last one writes c_0 x~ + acc / d - b_2 over
// yacc (u = 1).
// kBatchHot: the hot pass of a split step, writing each row's sum to part.
enum BatchMode : int32_t { kBatchForward = 0, kClenshawStep = 1, kClenshawLast = 2, kBatchHot = 3 };
hipError_t launch_batch_step(int32_t prec, const BatchStepArgs& a, hipStream_t st);

// Hub scratch a step needs on graph g (single-source or batched, every
// pass, every plan shape the autotuners may install): rows split into
// segments and their segments.
int64_t batch_hub_rows(const cp_graph* g);
int64_t batch_hub_segments(const cp_graph* g);
extern const PlanShape kHubShapes[3];
// The graph's CSR and work plan for the batched step (and its hot/cold
// split, if any) into a; `part` is the split's partial buffer (workspace).
void set_batch_plan(const cp_graph* g, BatchStepArgs& a, void* part);

struct BatchInitArgs {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const int64_t* src;    // [nq_pad] internal source id per slot (-1: unused slot)
  int64_t n;
  int32_t bw;
  int32_t nq_pad;
  void* r0;
  void* r1;
  void* yacc;
  const double* coef;    // rows 0 and 1 used
};
hipError_t launch_batch_init(int32_t prec, const BatchInitArgs& a, int32_t nslots, hipStream_t st);

struct BatchFinalArgs {
  const int64_t* row_ptr;
  const int32_t* perm;   // internal -> caller id, or null
  const int32_t* slot_of_query;  // [nq]
  int64_t n;
  int32_t bw;
  int32_t nq;
  const void* yacc;
  void* Y;               // [n][nq] caller ids
  const double* oexp;    // [slots] output exponent 1 - a
  const double* oscale;  // [slots] output scale (d_s^a, or 1)
};

// Per-slot parameters of batched and served queries, [kSlotParams][slots]
// doubles: step factor (2 or 1), output exponent 1 - a, output scale, and a
// row of ones (the step factor of the first step of a dense start).
constexpr int kSlotParams = 4;
std::vector<double> slot_params(int32_t nslots);  // host image with the defaults

// Dense start vectors (Thm. 5): column j of the caller's X [n][k] (caller
// ids) becomes slot j with r~_0(v) = d_v^{a-1} X[perm(v)][j] (0 where d_v = 0)
// and yacc = c0 r~_0.
struct DenseInitArgs {
  const int64_t* row_ptr;
  const int32_t* perm;   // internal -> caller id, or null
  int64_t n;
  int32_t bw;
  int32_t k;
  const void* X;         // double for CP_F64, float otherwise
  double a;
  double cr, cy;         // r0 = cr x~ and yacc = cy x~, x~ = D^{a-1} x (D^{-1} basis)
  void* r0;
  void* yacc;
};
hipError_t launch_dense_init(int32_t prec, const DenseInitArgs& a, hipStream_t st);
hipError_t launch_batch_finalize(int32_t prec, const BatchFinalArgs& a, hipStream_t st);

// Server: for finished (or cancelled) slots, write y = D yacc of the slot
// (caller ids) to its output (if non-null) and zero the slot's columns of
// all three tile-major buffers, leaving the slot ready for a new query.
struct SlotFinishArgs {
  const int64_t* row_ptr;
  const int32_t* perm;
  int64_t n;
  int32_t bw;
  const int32_t* slots;  // [count]
  void* const* outs;     // [count] device pointers (null: clear only)
  void* rA;
  void* rB;
  void* yacc;
  const double* oexp;    // [slots]
  const double* oscale;  // [slots]
};
hipError_t launch_slot_finish(int32_t prec, const SlotFinishArgs& a, int32_t count, hipStream_t st);

// Copy `bytes` (multiple of 4) of host data to device memory through kernel
// arguments (no host buffer has to outlive the call; capturable in graphs).
hipError_t launch_upload(void* dst, const void* host, size_t bytes, hipStream_t st);

// ------------------------------------------------------------- host helpers

cp_status coeffs_impl(int32_t kind, double param, int32_t K, double* c);
cp_status choose_K_impl(int32_t kind, double param, double tol, int32_t kmode, int32_t K_fixed,
                        double vol, double d_s, int32_t K_max, int32_t* K_out, double* tail_out);

void set_hip_error(hipError_t e);

// Validate a query against a graph (source range and degree, parameter
// domain, flags, truncation step) and plan it: everything a query needs
// before launch.  s_int is the source in internal node order, L the l1
// multiplier of the tail bound (sqrt(vol / d_s) for Alg. 3).  Alg. 3: c = c_0..c_K, top = K.
// Alg. 1 (CP_Q_PWMETHOD): c = zeta_0..zeta_{N-1} (zero-padded to two
// entries), top = max(N - 1, 1), L = 1.  Both run the same launch sequence:
// init gives r_0, r_1 and c_0 r_0 + c_1 r_1, then top - 1 steps add
// c_{k+1} r_{k+1}.
struct QueryPlan {
  int64_t s_int = 0;
  int32_t K = 0;      // reported truncation step: K (Alg. 3) or N (Alg. 1)
  int32_t top = 0;    // highest coefficient index
  double tail = 0, L = 1;
  double rec = 2.0;   // step factor: 2 (Eq. 6) or 1 (Alg. 1)
  double oexp = 1.0;  // output d_v^oexp yacc(v) scaled by oscale (Def. 8: 1 - a, d_s^a)
  double oscale = 1.0;
  std::vector<double> c;
};
cp_status plan_query(const cp_graph* g, const cp_query* q, int32_t K_max, QueryPlan* p);
// Workspace of one cp_power query on g at precision prec.
size_t single_ws_bytes(const cp_graph* g, int32_t prec);
cp_status taylor_impl(int32_t kind, double param, int32_t N, double* zeta);
cp_status choose_N_impl(int32_t kind, double param, double tol, int32_t kmode, int32_t N_fixed,
                        int32_t N_max, int32_t* N_out, double* tail_out);

constexpr int32_t kDefaultKMax = 4096;
constexpr int32_t kBatchKCap = 1024;  // largest K a batched query may need

}  // namespace cp

struct cp_graph {
  int64_t n = 0, nnz = 0, d_max = 0;
  int device = 0;
  const int64_t* row_ptr = nullptr;  // internal node order
  const int32_t* col_idx = nullptr;
  void* owned_csr = nullptr;         // allocation holding row_ptr/col_idx when owned
  int32_t* perm = nullptr;           // internal -> caller id (reordered graphs)
  std::vector<int32_t> ext2int;      // caller id -> internal id (reordered graphs)
  std::vector<int32_t> degree;       // by caller id
  // XCD-striped layout (CP_GRAPH_XCD_STRIPES)
  bool striped = false;
  int32_t s_count = 0;              // stripes S
  int32_t* s_rp = nullptr;          // [S][n+1]
  int32_t* s_cols = nullptr;        // nnz
  int64_t s_col_off[cp::kMaxStripes] = {};
  int64_t s_base[cp::kMaxStripes] = {};  // first node of each stripe
  bool s_packed = false;              // tile blocks in the packed form
  cp::StripeBlock* s_blocks = nullptr;
  int64_t s_ntiles = 0, s_nlong = 0;
  cp::DevPlan single;  // plan of the single-source step kernel
  cp::DevPlan batch;   // plan of the batched step kernel
  // hot/cold split of the batched step (CP_GRAPH_HOT_SPLIT)
  bool hot_split = false;
  cp::BatchSplit split{};
  cp::DevPlan hot_plan, cold_plan;
  void* split_mem = nullptr;          // allocation holding both split CSRs and their plans
  int64_t hot_arcs = 0;
  void* plan_mem = nullptr;
  int64_t device_bytes = 0;
  bool reordered = false, borrowed = false;
  // batched source-tile width chosen by cp_autotune_batch, keyed by (nq, prec)
  std::map<int64_t, int32_t> tuned_bw;
  std::mutex tune_mu;
  // row offsets in internal order (host), from which the autotuners rebuild
  // plans, and the device memory of plans they installed
  std::vector<int64_t> host_rp;
  void* tuned_plan_mem[2] = {nullptr, nullptr};  // single, batch
  // hub rows and segments of the plan shape with the most of them, over
  // every shape the autotuners may install: workspaces are sized by these,
  // so a plan installed later never outgrows a workspace sized earlier
  int64_t hub_rows_cap = 1, hub_segs_cap = 1;
};
