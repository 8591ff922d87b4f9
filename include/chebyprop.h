/* chebyprop.h - C ABI of the MI355X (gfx950) ChebyPower library.
 *
 * Computes graph-propagation vectors y = f(P) e_s on an undirected graph,
 * P = A D^{-1} (Sec. 2.1, Eq. 1), for
 *   CP_PPR  : f(x) = alpha / (1 - (1-alpha) x), alpha in (0,1)   (Def. 3)
 *   CP_HKPR : f(x) = exp(-t (1 - x)),           t > 0            (Def. 4)
 * by ChebyPower (Alg. 3): the truncated Chebyshev expansion
 *   y_K = sum_{k=0..K} c_k T_k(P) e_s                            (Lemma 1)
 * with the closed-form coefficients of Lemma 2 (PPR) and Lemma 3 (HKPR),
 * evaluated with the three-term recurrence r_{k+1} = 2 P r_k - r_{k-1}
 * (Eq. 6).
 *
 * Conventions for every call
 *  - Return value: cp_status (CP_OK = 0, errors < 0).  No C++ exception
 *    crosses the ABI.  After CP_EHIP, cp_last_hip_error() gives the raw
 *    hipError_t of the failing HIP call (thread-local).
 *  - Pointers marked "device" are HIP device pointers (e.g. the data_ptr()
 *    of a torch tensor on the GPU); "host" pointers are ordinary memory.
 *    The caller owns every buffer it passes; the library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it and is complete when the stream is.
 *    Calls return without waiting for the GPU unless a query sets
 *    CP_Q_STATS or CP_Q_TIMING.
 *  - A cp_graph is immutable after creation; concurrent queries on one
 *    graph from different streams are allowed as long as each uses its own
 *    output and workspace buffers.
 */
#ifndef CHEBYPROP_H
#define CHEBYPROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CP_OK = 0,
  CP_EINVAL = -1,     /* bad argument (NULL pointer, size, parameter domain, K < 1) */
  CP_ESOURCE = -2,    /* source id outside [0, n) */
  CP_EISOLATED = -3,  /* source has degree 0: P = A D^{-1} is undefined there */
  CP_ENOMEM = -4,     /* device or host allocation failed */
  CP_EHIP = -5,       /* a HIP runtime call failed, see cp_last_hip_error() */
  CP_EKMAX = -6,      /* the tolerance needs more than the allowed number of terms */
  CP_EBUSY = -7,      /* server: admission refused (HBM budget or queue full) */
  CP_ECANCELLED = -8, /* server: query was cancelled */
  CP_ENOTFOUND = -9,  /* server: unknown ticket */
  CP_EGRAPH = -10,    /* graph validation failed (see cp_graph_create) */
  CP_EPENDING = -11,  /* server: query not finished yet */
  CP_EWORKSPACE = -12 /* workspace missing or smaller than cp_workspace_bytes() */
} cp_status;

typedef enum { CP_PPR = 0, CP_HKPR = 1 } cp_kind;

/* Precision of the recurrence vectors (the bytes every step gathers) and of
 * the arithmetic.  CP_F64: double storage and arithmetic.  CP_F32: float
 * storage of the recurrence vectors, double arithmetic (gather sums, update)
 * and a double estimate; l1 rounding error is a few 1e-8 on million-node
 * power-law graphs.  CP_F32F: float storage and float arithmetic, with the
 * estimate and the partial sums in float too (fewer bytes per step than
 * CP_F32); l1 rounding error about 1e-7 to 3e-7 on million-node graphs, so
 * it suits tolerances from about 3e-7 up.  CP_BF16: bfloat16 storage,
 * float arithmetic and estimate (l1 error around 1e-3).  Output y is double
 * for CP_F64 and float otherwise.  Coefficients, K and the estimate's
 * final scaling are computed in double in every precision. */
typedef enum { CP_F64 = 0, CP_F32 = 1, CP_BF16 = 2, CP_F32F = 3 } cp_prec;

/* How K is chosen for a tolerance `tol` (Thm. 2 and its l1 reading):
 *  CP_K_CERTIFIED: smallest K >= 1 with sqrt(vol(G)/d_s) * tail(K) <= tol,
 *                  tail(K) = sum_{k>K} |c_k|.  Because
 *                  ||T_k(P) e_s||_1 <= sqrt(vol/d_s), this bounds the l1
 *                  truncation error by tol.
 *  CP_K_TAIL:      Thm. 2 as printed: tail(K) <= tol.
 *  CP_K_PAPER:     the experiments' K = ceil(ln(1/tol)/sqrt(alpha)) for PPR
 *                  and ceil(sqrt(t) ln(1/tol)) for HKPR (Sec. 6.1, 6.2).
 *  CP_K_FIXED:     K = K_fixed (must be >= 1). */
typedef enum { CP_K_CERTIFIED = 0, CP_K_TAIL = 1, CP_K_PAPER = 2, CP_K_FIXED = 3 } cp_kmode;

/* cp_graph_create flags */
#define CP_GRAPH_BORROW 0x1   /* keep using the caller's CSR buffers (caller keeps
                                 them alive until cp_graph_destroy); ignored when
                                 CP_GRAPH_REORDER is set */
#define CP_GRAPH_VALIDATE 0x2 /* O(nnz) checks: monotone offsets, ids in range, no
                                 self-loops, no duplicate arcs, symmetry */
#define CP_GRAPH_REORDER 0x4  /* relabel nodes internally by decreasing degree
                                 (results are still returned in caller ids) */
#define CP_GRAPH_HOST 0x8     /* row_ptr / col_idx are host pointers */
#define CP_GRAPH_XCD_STRIPES 0x10 /* relabel nodes into S degree-interleaved column
                                     stripes (S = 2, 4 or 8, see
                                     cp_graph_stats.stripe_count) and keep one CSR
                                     per stripe, so that single-source steps
                                     gather each stripe on its own XCDs (from
                                     their L2); costs a second copy of the column
                                     ids plus S (n+1) int32 offsets, so each
                                     stripe must hold fewer than 2^31 arcs
                                     (CP_EINVAL otherwise) */
#define CP_GRAPH_HOT_SPLIT 0x20   /* relabel by degree (as CP_GRAPH_REORDER, or the
                                     stripes of CP_GRAPH_XCD_STRIPES) and keep the
                                     batched step's arcs in two CSRs: arcs into the
                                     cp_graph_stats.hot_nodes highest-degree nodes,
                                     and the rest.  A batched step (cp_power_batch,
                                     cp_propagate, the server) then sums each row's
                                     hot arcs first, gathering from a slice of the
                                     vectors small enough for the caches to keep,
                                     and the rest second, starting from that sum.
                                     hot_nodes is sized so that the slice of an
                                     8-wide FP32 tile (32 bytes a node) is 16 MiB
                                     (524,288 nodes), or set by the environment variable
                                     CHEBYPROP_HOT_NODES at create.  Costs a second
                                     copy of the column ids, two (n+1) int64 offset
                                     arrays, and an estimate-sized partial buffer in
                                     every batched workspace.  Results equal the
                                     unsplit step's up to the order of the sums. */

/* cp_query.flags */
#define CP_Q_STATS 0x1  /* after the run, synchronize and fill cp_info.mass */
#define CP_Q_TIMING 0x2 /* time the run and each Chebyshev step with HIP events
                           (synchronizes; fills elapsed_ms, step_ms) */
#define CP_Q_PWMETHOD 0x4 /* evaluate with PwMethod (Alg. 1) instead of
                             ChebyPower: y = sum_{k<N} zeta_k P^k e_s with the
                             Taylor weights of Def. 3 / Def. 4.  N (reported
                             in cp_info.K) is the smallest N whose exact l1
                             tail sum_{k>=N} zeta_k is <= tol for every kmode
                             but CP_K_FIXED (N = K_fixed); that tail is also
                             the exact l1 truncation error (tail_bound_l1).
                             Runs max(N - 2, 0) full power steps after the
                             init, on the same kernels as Alg. 3. */
#define CP_Q_CLENSHAW 0x8 /* cp_propagate only: evaluate the same K-term
                             Chebyshev series by Clenshaw's backward recurrence
                             (Clenshaw 1955), b_k = c_k x + 2 P b_{k+1} -
                             b_{k+2}, sum = c_0 x + P b_1 - b_2: K full steps
                             as in the forward form, but no estimate vector is
                             read or written (the start vector is read
                             instead).  Not with CP_Q_PWMETHOD (CP_EINVAL). */

typedef struct cp_graph cp_graph;

typedef struct {
  int32_t kind;    /* cp_kind */
  int32_t kmode;   /* cp_kmode */
  double param;    /* alpha (PPR) or t (HKPR) */
  double tol;      /* l1 tolerance in (0,1); unused for CP_K_FIXED */
  int64_t source;  /* s, in the caller's node ids */
  int32_t K_fixed; /* K for CP_K_FIXED */
  int32_t flags;   /* CP_Q_* (any other bit: CP_EINVAL) */
  double a;        /* output space, 0 <= a <= 1 (Def. 8 with b = 1 - a): the
                      result is z = f(D^{-a} A D^{-b}) e_s = d_s^a D^{-a} f(P) e_s
                      (the single-source form of Thm. 5).  0 gives y = f(P) e_s,
                      1/2 gives f(A~) e_s for A~ = D^{-1/2} A D^{-1/2}. */
} cp_query;

typedef struct {
  int32_t K;            /* truncation step used: K of Alg. 3, or N of Alg. 1 */
  int32_t steps;        /* full step launches for this query: K - 1 (Alg. 3), max(N - 2, 0) (Alg. 1) */
  double tail;          /* sum_{k>K} |c_k|, or sum_{k>=N} zeta_k */
  double tail_bound_l1; /* bound on the l1 truncation error: sqrt(vol/d_s) * tail
                           (Alg. 3, CP_K_CERTIFIED reading), tail (Alg. 1, exact) */
  double mass;          /* sum_u y(u) (CP_Q_STATS; 1 up to truncation and rounding) */
  double elapsed_ms;    /* whole query on the device (CP_Q_TIMING) */
  double step_ms;       /* sum of the Chebyshev step kernels' durations (CP_Q_TIMING) */
  double latency_ms;    /* server: submit -> result written (host clock) */
  double wait_ms;       /* server: submit -> admitted into a resident slot */
  int64_t pushes;       /* cp_push: push operations (sum of |S_k|); 0 for the other paths */
  int64_t arcs;         /* arcs the full steps processed: steps * nnz, or for cp_push the
                           sum of vol(S_k) (with CP_Q_STATS / CP_Q_TIMING, else -1) */
  int64_t walks;        /* cp_push_rw: random walks run (CP_Q_STATS / CP_Q_TIMING, else -1); 0 otherwise */
  int64_t walk_steps;   /* cp_push_rw: moves made by those walks */
} cp_info;

typedef struct {
  int64_t n, nnz, d_max;
  int64_t blocks;       /* work blocks of the step kernel */
  int64_t long_rows;    /* rows streamed by a whole workgroup */
  int64_t hub_rows;     /* rows split over several workgroups */
  int64_t device_bytes; /* graph bytes held in HBM by the library */
  int32_t reordered;
  int32_t borrowed;
  int64_t stripe_tiles; /* row tiles of the XCD-striped step (0 if not striped) */
  int64_t stripe_packed; /* 1: striped tile arcs stored sorted by column with their
                            CSR positions (every stripe holds at most 2^21 nodes,
                            i.e. n <= 2^24); 0: plain column ids or not striped */
  int64_t stripe_count;  /* column stripes S of the XCD-striped layout (0 if not
                            striped): the fewest of 2, 4, 8 whose FP32 slice of
                            the vector, 4 n / S bytes, fits 4 MiB */
  int64_t hot_nodes;     /* hot nodes of the CP_GRAPH_HOT_SPLIT layout (0 without) */
  int64_t hot_arcs;      /* arcs into them (the hot pass's share of nnz) */
  /* row splits of the work plans (set at create, changed by the autotuners):
   * rows above long_cut arcs are streamed by a whole workgroup instead of
   * sharing a tile, rows above hub_cut arcs are split into hub_seg-arc
   * segments over several workgroups */
  int64_t single_long_cut, single_hub_cut, single_hub_seg;  /* cp_power, single CSR */
  int64_t batch_long_cut, batch_hub_cut, batch_hub_seg;     /* batched steps */
} cp_graph_stats;

/* Build a graph from symmetric CSR (Sec. 2.1: undirected, A in {0,1}):
 * row v lists N(v); d_v = row_ptr[v+1] - row_ptr[v].
 *   n        nodes (1 <= n < 2^31)
 *   nnz      arcs = 2 m (row_ptr[n]); int32 column ids
 *   row_ptr  int64[n+1], device (host with CP_GRAPH_HOST)
 *   col_idx  int32[nnz], device (host with CP_GRAPH_HOST)
 *   flags    CP_GRAPH_*
 * Errors: CP_EINVAL (sizes, NULL, row_ptr[0] != 0, row_ptr[n] != nnz, a
 * decreasing offset or a degree of 2^31 or more; these offset checks run
 * on every create), CP_EGRAPH (CP_GRAPH_VALIDATE failed),
 * CP_ENOMEM, CP_EHIP.  Synchronizes `stream`.  Nodes with degree 0 are
 * allowed (they are never reached and get y = 0) but cannot be sources. */
cp_status cp_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          int32_t flags, void* stream, cp_graph** out);
/* Free the graph's device memory.  Queries still running on it and servers
 * created on it must be finished and destroyed first (a server keeps using
 * the graph until cp_server_destroy returns). */
cp_status cp_graph_destroy(cp_graph* g);
/* Sizes and layout of the graph into host *out.  Errors: CP_EINVAL. */
cp_status cp_graph_get_stats(const cp_graph* g, cp_graph_stats* out);

/* Chebyshev coefficients c_0..c_K into host c_out[K+1], FP64
 * (Lemma 2: c_0 = gamma, c_k = 2 gamma beta^k;
 *  Lemma 3: c_0 = e^{-t} I_0(t), c_k = 2 e^{-t} I_k(t)).
 * Pure host code.  Errors: CP_EINVAL. */
cp_status cp_coeffs(int32_t kind, double param, int32_t K, double* c_out);

/* Truncation step for a tolerance (see cp_kmode); vol = sum of degrees,
 * d_s = degree of the source (only used by CP_K_CERTIFIED).  Writes K and
 * tail(K).  Pure host code.  Errors: CP_EINVAL, CP_EKMAX (K > K_max). */
cp_status cp_choose_K(int32_t kind, double param, double tol, int32_t kmode, int32_t K_fixed,
                      double vol, double d_s, int32_t K_max, int32_t* K_out, double* tail_out);

/* Taylor weights zeta_0..zeta_{N-1} of PwMethod into host zeta_out[N], FP64
 * (Def. 3: zeta_k = alpha (1 - alpha)^k; Def. 4: zeta_k = e^{-t} t^k / k!).
 * Pure host code.  Errors: CP_EINVAL. */
cp_status cp_taylor(int32_t kind, double param, int32_t N, double* zeta_out);

/* PwMethod's number of terms N for a tolerance: the smallest N >= 1 with
 * sum_{k>=N} zeta_k <= tol (every P^k e_s is a probability vector, so this
 * tail is the exact l1 error), or N_fixed for CP_K_FIXED.  Writes N and the
 * tail.  Pure host code.  Errors: CP_EINVAL, CP_EKMAX (N > N_max). */
cp_status cp_choose_N(int32_t kind, double param, double tol, int32_t kmode, int32_t N_fixed, int32_t N_max,
                      int32_t* N_out, double* tail_out);

/* Device workspace needed by cp_power (nq = 1) or cp_power_batch (nq
 * queries) at precision `prec`.  Returns 0 for invalid arguments. */
size_t cp_workspace_bytes(const cp_graph* g, int32_t nq, int32_t prec);

/* One query (Alg. 3): y = sum_{k<=K} c_k T_k(P) e_s (Alg. 1 with CP_Q_PWMETHOD).
 *   y     device, n elements (double for CP_F64, float otherwise), caller ids
 *   ws    device workspace of at least cp_workspace_bytes(g, 1, prec) bytes,
 *         256-byte aligned; contents are scratch
 *   info  host, may be NULL; K/steps/tail fields are valid on return, the
 *         rest after the stream completes (or on return with CP_Q_STATS /
 *         CP_Q_TIMING, which synchronize)
 * Errors: CP_EINVAL, CP_ESOURCE, CP_EISOLATED, CP_EKMAX, CP_EWORKSPACE, CP_EHIP. */
cp_status cp_power(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws,
                   size_t ws_bytes, void* stream, cp_info* info);

/* Bytes of the device array cp_power_noalloc works in. */
#define CP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* cp_power for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument, and no hipMalloc, hipFree, event or other allocating
 * call.  The workspace is one static device array of CP_NOALLOC_SCRATCH_BYTES
 * (64 MiB), which each GPU the library runs on holds until the process
 * ends; its address is looked up once per device, on the first call with
 * that device current.
 *   y, info  as cp_power; the current device must be the graph's
 * Every call on a GPU works in that GPU's one array and leaves its contents
 * there (each call clears what it needs zero first), so calls that overlap
 * on one GPU (other streams, other host threads) race: serialize them.
 * Results are bitwise those of cp_power.
 * Errors: those of cp_power; CP_EWORKSPACE when the query's workspace
 * exceeds CP_NOALLOC_SCRATCH_BYTES: two recurrence vectors of n storage
 * elements, an n-element estimate (double; float for CP_F32F and CP_BF16), S n more
 * estimate-width partials on a graph with S XCD stripes, and a few KiB of
 * counters (FP32: 16 n bytes, about 4M nodes, or 16 n + 8 S n with
 * stripes); CP_EINVAL for CP_Q_TIMING (its events would be created per
 * call) or when the current device is not the graph's. */
cp_status cp_power_noalloc(const cp_graph* g, const cp_query* q, int32_t prec, void* y, void* stream,
                           cp_info* info);

/* nq queries at once (each with its own kind, parameter, tolerance and K):
 * the batched form of Alg. 3.  Y is device [n][nq] row-major in caller ids
 * (double for CP_F64, float otherwise); infos is host [nq] or NULL.
 * Errors as cp_power; no output is written if any query is invalid. */
cp_status cp_power_batch(const cp_graph* g, int32_t nq, const cp_query* q, int32_t prec, void* Y,
                         void* ws, size_t ws_bytes, void* stream, cp_info* infos);

/* Generalized graph propagation of a feature matrix (Def. 8, Thm. 5):
 * Z = f(D^{-a} A D^{-b}) X with b = 1 - a, computed as Z = D^{-a} y^ where y^
 * is the K-term series of Alg. 3 (or N terms of Alg. 1 with CP_Q_PWMETHOD;
 * or Alg. 3's series by Clenshaw's recurrence with CP_Q_CLENSHAW) started
 * from D^{a} x_j, for the k columns of X together (batched steps, k columns
 * in source tiles).
 *   q     kind, param, a, K_fixed, flags (CP_Q_PWMETHOD or CP_Q_CLENSHAW,
 *         CP_Q_TIMING) and
 *         the truncation rule: CP_K_FIXED, CP_K_TAIL (tail(K) <= tol) or
 *         CP_K_PAPER; CP_K_CERTIFIED needs norms of X and gives CP_EINVAL;
 *         source is ignored
 *   X, Z  device [n][k] row-major in caller ids, double for CP_F64 and float
 *         otherwise; Z may be X (X is read once, before Z is written)
 *   ws    device workspace of cp_workspace_bytes(g, k, prec) bytes (256-byte
 *         aligned); the source-tile width follows cp_set_batch_width /
 *         cp_autotune_batch for nq = k
 *   info  host, may be NULL: K (or N), steps (full step launches, K), tail;
 *         tail_bound_l1 is NaN (it depends on X)
 * Reading: a node of degree 0 is outside the propagation; its row of X is
 * ignored and its row of Z is 0.  Errors: CP_EINVAL, CP_EKMAX (K > 1024),
 * CP_EWORKSPACE, CP_EHIP. */
cp_status cp_propagate(const cp_graph* g, const cp_query* q, int32_t k, int32_t prec, const void* X, void* Z,
                       void* ws, size_t ws_bytes, void* stream, cp_info* info);

/* ChebyPush (Alg. 4, Sec. 4.2): the subset Chebyshev recurrence of Def. 7
 * in push form, touching only the nodes whose residual passes the step
 * threshold eps_k = eps_a / (4 K sum_{l=k}^{K} |c_l|), tested as
 * |r(u)| > eps_k d_u (Alg. 4's test; the paper's prose squares r).  Output
 * y^ = c_0 e_s + sum_{k<K} c_k r^_k|S_k, in FP64, in the space chosen by
 * q->a (y^ scaled by d_s^a D^{-a}).  Thm. 4 bounds the degree-normalised
 * error max_u |y(u) - y^(u)| / d_u by eps_a when K meets Thm. 2's tail at
 * eps_a / 2 (under the paper's stability assumption).
 *   q      as cp_power (kind, param, source, K rule, a; CP_Q_STATS,
 *          CP_Q_TIMING); CP_Q_PWMETHOD gives CP_EINVAL
 *   eps_a  >= 0 (0 pushes every non-zero residual: the first K terms of
 *          Alg. 3)
 *   y      device, n doubles, caller ids
 *   ws     device workspace of cp_push_workspace_bytes(g) bytes, 256-byte
 *          aligned
 *   info   pushes and arcs need CP_Q_STATS or CP_Q_TIMING (synchronizes)
 * An iteration makes a few coalesced passes over per-node flags (select,
 * listing) and otherwise touches the arcs of S_k and of the rows they reach;
 * an iteration that pushes more than n/8 nodes or nodes with more than
 * nnz/128 arcs pulls every row with the single-source step kernels instead.
 * No floating-point atomics: results are bitwise reproducible run to run.
 * Errors as cp_power. */
size_t cp_push_workspace_bytes(const cp_graph* g);
cp_status cp_push(const cp_graph* g, const cp_query* q, double eps_a, double* y, void* ws, size_t ws_bytes,
                  void* stream, cp_info* info);

/* ChebyPush + random walks for SSPPR (Alg. 5, Sec. 5.2).  With
 * W = 2 (2 eps_r / 3 + 2) ln(n) / (eps_r^2 delta) and r_max = sqrt(alpha) / W
 * (or the caller's r_max > 0), ChebyPush runs with threshold r_max, then
 * every node with a non-zero residual r = e_s - alpha^{-1} [I - (1 - alpha)
 * P] pi^ starts ceil(|r(v)| W) alpha-random walks, each adding r(v) / W_v at
 * its end node.  The guarantee is Alg. 5's: |pi^(u) - pi_s(u)| < eps_r
 * pi_s(u) wherever pi_s(u) > delta, with high probability.
 *   q      CP_PPR only (param = alpha), source, a (output space),
 *          CP_Q_STATS / CP_Q_TIMING; K by q->kmode with r_max as the
 *          tolerance (CP_K_PAPER gives the analysis' K = ln(1/r_max) /
 *          sqrt(alpha)) or K_fixed
 *   seed   walk j from node v draws SplitMix64 (Steele, Lea & Flood, 2014)
 *          outputs j * 2^32 + 2 t and j * 2^32 + 2 t + 1 of the stream
 *          whose seed is output v (caller id) of the stream of `seed`:
 *          step t stops when (x >> 11) 2^-53 < alpha, else moves to neighbour
 *          (x' d) >> 64 of the current row in the graph's internal CSR
 *          order (the caller's order unless the graph was reordered)
 *   y      device, n doubles, caller ids
 *   ws     device workspace of cp_push_rw_workspace_bytes(g) bytes
 *   info   walks and walk_steps as for pushes; step_ms times the push phase
 * End-node contributions use FP64 atomic adds: results agree run to run up
 * to rounding.  Errors: CP_EINVAL (not PPR, eps_r, delta or r_max out of
 * range), otherwise as cp_push. */
size_t cp_push_rw_workspace_bytes(const cp_graph* g);
cp_status cp_push_rw(const cp_graph* g, const cp_query* q, double eps_r, double delta, double r_max,
                     uint64_t seed, double* y, void* ws, size_t ws_bytes, void* stream, cp_info* info);

/* Pick the source-tile width (8, 16, 32 or 64 sources per tile) that runs
 * these nq queries fastest on this graph and remember it for later
 * cp_power_batch calls with the same nq and precision.  Runs the queries
 * once per candidate width (Y, ws as for cp_power_batch; Y holds the last
 * run's result).  Then, at that width and on a graph without
 * CP_GRAPH_HOT_SPLIT, tunes the batched plan's row splits as
 * cp_autotune_single does (long-row cuts 64, 128, 256, 512, 1024 arcs and
 * the same hub shapes) and keeps the fastest for every batched call on the
 * graph (servers and cp_propagate included).  Workspaces are sized for any
 * of these plans, so one sized before the call stays valid.  Must not run
 * while other calls use the graph.  Synchronizes `stream`.  bw_out may be
 * NULL. */
cp_status cp_autotune_batch(cp_graph* g, int32_t nq, const cp_query* q, int32_t prec, void* Y, void* ws,
                            size_t ws_bytes, void* stream, int32_t* bw_out);

/* Row-split autotuner of the single-source step on a graph without XCD
 * stripes (striped graphs run fixed stripe tiles; the call returns CP_OK and
 * changes nothing): runs the query (y, ws as for cp_power; y holds the last
 * run's result) with each candidate long-row cut (256, 512, 1024, 2048 arcs)
 * and hub shape (rows above 16384 / 4096 / 65536 arcs in segments of 8192 /
 * 2048 / 16384), each against the best so far, and keeps the fastest plan
 * for every later single-source query on the graph (cp_graph_stats reports
 * it).  Results change only in the order of the sums of split rows.  Must
 * not run while other calls use the graph.  Synchronizes `stream`.  Errors
 * as cp_power, CP_ENOMEM. */
cp_status cp_autotune_single(cp_graph* g, const cp_query* q, int32_t prec, void* y, void* ws, size_t ws_bytes,
                             void* stream);

/* Fix the source-tile width used by cp_power_batch for (nq, prec) on this
 * graph (bw in {8, 16, 32, 64}; 0 forgets the choice and returns to the
 * built-in default).  Errors: CP_EINVAL. */
cp_status cp_set_batch_width(cp_graph* g, int32_t nq, int32_t prec, int32_t bw);

/* ------------------------------------------------------------ query server
 *
 * A server keeps the graph and the recurrence state of up to `slots`
 * queries resident in HBM and advances every admitted query by one
 * Chebyshev step per batched launch (iteration-level batching: queries join
 * and leave at step boundaries, each with its own K and coefficients).
 * Slots are sized by the HBM budget: one slot costs n * (2 * storage + 1 *
 * accumulator) bytes; queries beyond the resident slots wait in a host
 * queue of `max_queue` entries.  The server drives the GPU from its own
 * host thread on its own stream; all calls are thread-safe. */
typedef struct cp_server cp_server;

typedef struct {
  int64_t slots;        /* resident query slots */
  int64_t active;       /* slots holding a running query */
  int64_t queued;       /* queries waiting for a slot */
  int64_t completed;    /* queries finished since creation */
  int64_t cancelled;
  int64_t ticks;        /* batched step launches */
  int64_t device_bytes; /* HBM held by the server (state + scratch) */
  int32_t tile_width;   /* sources per tile in the step kernel */
  int32_t prec;
  int32_t waiters;      /* threads blocked in cp_server_wait */
  int32_t direct_limit; /* longest queue an idle server runs one by one (see below) */
  int64_t direct;       /* queries run on the single-source path (see below) */
  int64_t narrow_ticks; /* batched launches that updated only the first 8 or 16 slots (see below) */
} cp_server_stats;

/* While no query is resident and at most direct_limit wait, the server runs
 * the oldest waiting query on the single-source path (cp_power's kernels on
 * the server's stream) instead of a batched launch, where a few queries
 * would pay a whole tile's gathers; longer queues are batched.
 * direct_limit starts at 3 and then follows t_b / t_s (at least 1, at most
 * 16), from running means of the host-clock time of a one-tile batched step
 * (t_b) and of a single-source query per Chebyshev step (t_s): q queries
 * one by one take about q K t_s, one batched tile about K t_b.  Results of
 * the two paths differ only in the order of sums.  Queries take the lowest
 * free slots, and while only the first 8 (or 16) slots hold stepping
 * queries a batched launch updates just those (8 or 16 values of each tile
 * row gathered instead of a whole row: 1.3 instead of 1.75 ms a step with 8
 * on a 4M-node graph in FP32).
 * g: the graph every query runs on; it must outlive the server.
 * hbm_budget_bytes: HBM the server may use for query state (>= one slot).
 * max_slots: upper bound on resident queries (0: as many as the budget
 * allows, at most 1024).  max_queue: waiting-queue capacity.  prec: CP_F32 / CP_F32F /
 * CP_F64 / CP_BF16 for all slots.  Errors: CP_EINVAL, CP_ENOMEM (budget below
 * one slot or allocation failure), CP_EHIP.  Besides the slots, the server
 * holds one cp_power workspace in HBM. */
cp_status cp_server_create(const cp_graph* g, size_t hbm_budget_bytes, int32_t max_slots, int32_t max_queue,
                           int32_t prec, cp_server** out);
/* Queue a query whose result y (device, n elements: float, or double for
 * CP_F64) will be written to y_out, in caller ids.  y_out must stay valid
 * until the query is done or cancelled.  Errors: CP_EINVAL, CP_ESOURCE,
 * CP_EISOLATED, CP_EKMAX (as cp_power), CP_EBUSY (queue full). */
cp_status cp_server_submit(cp_server* s, const cp_query* q, void* y_out, uint64_t* ticket);
/* CP_OK and info (may be NULL) when the result is in y_out; CP_EPENDING while
 * queued or running; CP_ECANCELLED; CP_ENOTFOUND for unknown tickets.  A
 * ticket is forgotten once poll has returned CP_OK or CP_ECANCELLED. */
cp_status cp_server_poll(cp_server* s, uint64_t ticket, cp_info* info);
/* As poll, but blocks until the query is done or cancelled (timeout_ms < 0:
 * no limit; on timeout returns CP_EPENDING). */
cp_status cp_server_wait(cp_server* s, uint64_t ticket, int64_t timeout_ms, cp_info* info);
/* Cancel a queued or running query (its y_out is left partially written or
 * untouched).  Errors: CP_ENOTFOUND (unknown or already finished). */
cp_status cp_server_cancel(cp_server* s, uint64_t ticket);
cp_status cp_server_get_stats(cp_server* s, cp_server_stats* out);
/* Stop the server thread (queued and running queries are cancelled) and
 * free its memory.  Threads blocked in cp_server_wait on this server return
 * CP_ECANCELLED before it is freed; no other call on it may start once
 * destroy has been called. */
cp_status cp_server_destroy(cp_server* s);

/* Static text naming a status code ("unknown status" for other values). */
const char* cp_status_str(int32_t st);
/* The raw hipError_t behind the calling thread's last CP_EHIP (0 if none). */
int32_t cp_last_hip_error(void);
/* Static version string of the library. */
const char* cp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHEBYPROP_H */
