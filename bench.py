#!/usr/bin/env python3
"""ChebyPower benchmark on one MI355X.

Headline (the JSON's "value"): a batch of 8 personalized-PageRank sources
(alpha = 0.2, l1 tolerance 1e-6 with the certified truncation step) on a
seeded Chung-Lu graph shaped like Friendster (n = 65,000,000 target nodes,
1,800,000,000 undirected edges, degree exponent 2.1, int64 offsets / int32
columns, 3.6 billion CSR arcs), FP32 vector storage.  One "step" of this
benchmark is one pass of the whole path (coefficients, K, init, the
Chebyshev steps, finalize) for the 8 sources.

Beside it:
  "single":  heat-kernel PageRank (t = 5), 16 sources one at a time, on a
             Chung-Lu graph shaped like LiveJournal (n = 4M, 35M edges,
             exponent 2.3), FP32 storage, XCD-striped layout;
  "batched": 64 PPR sources with tolerances from {1e-4, 1e-6, 1e-7} in one
             batch on a graph shaped like Orkut (n = 3M, 117M edges,
             exponent 2.2), autotuned source-tile width;
  "served":  a Poisson query stream on the LiveJournal-shaped graph (60 s at
             200 queries/s after a 5-s warm-up, and 50 queries/s), the
             batched server against plain one-query-at-a-time runs;
  and the PwMethod, feature-matrix, ChebyPush and small-graph latency
  measurements.  The headline and "single" also time their workload with
  BF16 storage ("storage_bf16") and with FP32 arithmetic ("arith_f32",
  CP_F32F: float sums, partials and estimate); the FP32 runs themselves
  store float vectors and compute in double.

Prints one JSON line: GTEPS (CSR arcs traversed per second, summed over
sources), the roofline of the dominant kernel against MI355X's 8 TB/s HBM
(algorithmic bytes per launch: column ids, row offsets and five vector
terms per node and source at the storage width), the error of every result
against the FP64 oracle, and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "GTEPS of Chebyshev steps, % HBM peak; served queries/s + p50/p99 vs plain"

HEADLINES = {
    # name: (n, m, gamma, seed, alpha, sources, tol, prec)
    "ppr-batch-friendster": (65_000_000, 1_800_000_000, 2.1, 5, 0.2, 8, 1e-6, "f32"),
    "ppr-batch-friendster-small": (2_000_000, 55_000_000, 2.1, 5, 0.2, 8, 1e-6, "f32"),
}

WORKLOADS = {
    # name: (n, m, gamma, seed, kind, param, tol, sources, prec)
    "hkpr-livejournal": (4_000_000, 35_000_000, 2.3, 2, "hkpr", 5.0, 1e-6, 16, "f32"),
    "hkpr-small": (200_000, 1_750_000, 2.3, 2, "hkpr", 5.0, 1e-6, 16, "f32"),
    # the Friendster-sized graph of the headline, one source at a time
    "ppr-friendster": (65_000_000, 1_800_000_000, 2.1, 5, "ppr", 0.2, 1e-6, 4, "f32"),
}

BATCH_WORKLOADS = {
    # name: (n, m, gamma, seed, alpha, sources, tolerance choices, prec)
    "ppr-batch-orkut": (3_000_000, 117_000_000, 2.2, 3, 0.2, 64, (1e-4, 1e-6, 1e-7), "f32"),
    "ppr-batch-small": (200_000, 4_000_000, 2.2, 3, 0.2, 64, (1e-4, 1e-6, 1e-7), "f32"),
}

STORAGE_BYTES = {"f64": 8, "f32": 4, "f32f": 4, "bf16": 2}
ACC_BYTES = {"f64": 8, "f32": 8, "f32f": 4, "bf16": 4}  # estimate as the kernels keep it (f32: double estimate)
ARITH_DTYPE = {"f64": "f64", "f32": "f64", "f32f": "f32", "bf16": "f32"}  # what the kernels add and multiply in


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SINGLE_SOURCES = ("kernels.hip", "common.h")         # the single-source step kernels
BATCH_SOURCES = ("kernels_batch.hip", "common.h")    # the batched step kernel


def kernel_hash(files=SINGLE_SOURCES) -> str:
    """First 16 hex digits of the sha256 of the given kernel sources."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2412_10789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_bytes(n: int, nnz: int, prec: str, sources: int = 1) -> int:
    """Algorithmic bytes of one Chebyshev step launch: column ids and row
    offsets once, and per node and source five vector terms at the storage
    width s: one compulsory gather of x, read + write of z, read + write of
    the estimate."""
    s = STORAGE_BYTES[prec]
    return 4 * nnz + 8 * (n + 1) + 5 * n * sources * s


def impl_step_bytes(n: int, nnz: int, prec: str, sources: int = 1) -> int:
    """The same step with the estimate at the width the kernels keep it
    (double for FP32 storage): the implementation's compulsory bytes, not the
    roofline's."""
    s, a = STORAGE_BYTES[prec], ACC_BYTES[prec]
    return 4 * nnz + 8 * (n + 1) + n * sources * (3 * s + 2 * a)


def clenshaw_step_bytes(n: int, nnz: int, prec: str, sources: int) -> int:
    """Algorithmic bytes of one step of Clenshaw's backward form: column ids
    and row offsets once, and per node and column four vector terms at the
    storage width: gather of b_{k+1}, read of b_{k+2}, write of b_k, read of
    the start vector (no estimate stream)."""
    s = STORAGE_BYTES[prec]
    return 4 * nnz + 8 * (n + 1) + 4 * n * sources * s


def measured_traffic(key: str, files=SINGLE_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken with the current sources of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "step_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    e = rec.get(key)
    if not e or e.get("kernel_hash") != kernel_hash(files):
        return None
    return e.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_ceiling(torch, nbytes: int = 1 << 30) -> float:
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def roofline(bytes_per_launch: float, avg_launch_ms: float, kernel: str, traffic=None, **extra) -> dict:
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
           "bytes_per_launch": int(bytes_per_launch), "avg_launch_us": round(avg_launch_ms * 1e3, 2)}
    out.update(extra)
    return out


def batch_launch_bytes(n: int, nnz: int, prec: str, Ks, fn=step_bytes) -> int:
    """Algorithmic bytes of one batch's step launches: launch k (k = 1 ..
    max K - 1) carries the sources whose K exceeds k."""
    return sum(fn(n, nnz, prec, sum(1 for K in Ks if K > k)) for k in range(1, max(Ks)))


def worst(rows, keys):
    """Largest value of each key over a list of per-result dicts."""
    return {k: max(r[k] for r in rows) for k in keys if rows and all(k in r for r in rows)}


# ------------------------------------------------------------------ oracle checks


def exact_vectors(g, kinds, params, srcs, chebyshev_for_ppr=False):
    """The converged vectors f(P) e_s as columns of an [n][B] array: the
    plain-C PwMethod with its exact l1 tail below 1e-15, except, with
    chebyshev_for_ppr, PPR columns (for small alpha PwMethod needs hundreds
    of steps): the plain-C Alg. 3 with the certified K for l1 1e-12."""
    from oracle import coefficients as C
    from oracle import native as NO
    from oracle import truncation as T

    ex = np.empty((g.n, len(srcs)), dtype=np.float64)
    cheb = [j for j, k in enumerate(kinds) if chebyshev_for_ppr and k == "ppr"]
    pw = [j for j in range(len(srcs)) if j not in cheb]
    if pw:
        Ns = [T.pwmethod_steps(kinds[j], params[j], 1e-15) for j in pw]
        ex[:, pw] = NO.power_method_multi(g.row_ptr, g.col_idx, [srcs[j] for j in pw],
                                          [C.taylor_coeffs(kinds[j], params[j], N) for j, N in zip(pw, Ns)], Ns)
    if cheb:
        Kx = [T.choose_K("ppr", params[j], 1e-12, vol=g.nnz, d_s=int(g.degrees[srcs[j]])) for j in cheb]
        ex[:, cheb] = NO.cheby_power_multi(g.row_ptr, g.col_idx, [srcs[j] for j in cheb],
                                           [C.ppr_chebyshev_coeffs(params[j], K) for j, K in zip(cheb, Kx)], Kx)
    return ex


def check_same_k_and_exact(g, Yg, kinds, params, srcs, Ks, chebyshev_for_ppr=False, refs=None):
    """Every column of Yg ([n][B], caller ids) against the FP64 oracle: Alg. 3
    at the GPU's K (the plain-C several-source form; rounding error of the
    GPU variant) and the converged vector (exact_vectors): l1, max-abs, the
    degree-normalized error of Def. 5 (Normalized RelErr) and mass.  refs, a
    dict, keeps the oracle's two sets of vectors for later calls on the same
    queries.  Returns the per-column rows and the oracle's wall time."""
    from oracle import coefficients as C
    from oracle import errors as E
    from oracle import native as NO

    t0 = time.perf_counter()
    refs = {} if refs is None else refs
    if "ref_K" not in refs:
        cs = [C.chebyshev_coeffs(k, p, K) for k, p, K in zip(kinds, params, Ks)]
        refs["ref_K"] = NO.cheby_power_multi(g.row_ptr, g.col_idx, srcs, cs, Ks)
        refs["exact"] = exact_vectors(g, kinds, params, srcs, chebyshev_for_ppr)
    ref_K, exact = refs["ref_K"], refs["exact"]
    oracle_s = time.perf_counter() - t0
    deg = g.degrees
    rows = []
    for j in range(len(srcs)):
        y = np.asarray(Yg[:, j], dtype=np.float64)
        rows.append({"source": int(srcs[j]), "kind": kinds[j], "param": params[j], "K": int(Ks[j]),
                     "l1_vs_same_K": E.l1(y, ref_K[:, j]), "max_abs_vs_same_K": E.max_abs(y, ref_K[:, j]),
                     "l1_vs_exact": E.l1(y, exact[:, j]), "max_abs_vs_exact": E.max_abs(y, exact[:, j]),
                     "norm_rel_err_vs_exact": E.degree_normalized(y, exact[:, j], deg),
                     "mass": float(y.sum())})
    return rows, oracle_s


def check_ppr_certificate(g, Yg, srcs, alphas):
    """Every column of Yg ([n][B], caller ids, PPR results) against the
    fixed-point equation of Def. 3: the l1 residual divided by alpha bounds
    the l1 distance to the exact PPR vector (no reference vector needed; one
    plain-C FP64 pass over the CSR for all columns), plus mass."""
    from oracle import native as NO

    t0 = time.perf_counter()
    res = NO.ppr_residual_multi(g.row_ptr, g.col_idx, srcs, alphas, Yg)
    oracle_s = time.perf_counter() - t0
    mass = np.asarray(Yg, dtype=np.float64).sum(axis=0)
    rows = [{"source": int(s), "alpha": float(a), "l1_bound_vs_exact": float(r / a), "mass": float(m)}
            for s, a, r, m in zip(srcs, alphas, res, mass)]
    return rows, oracle_s


def _host(t):
    """A device result as a host float64 array."""
    return t.double().cpu().numpy()


GRAPH_CACHE = None  # directory for generated graphs (--graph-cache), shared by profiling passes


def chung_lu(synth, n, m, gamma, seed, tune_passes=3):
    """synth.chung_lu, optionally kept as .npy files in GRAPH_CACHE so that
    repeated runs (profiler passes) read the graph instead of generating it."""
    if not GRAPH_CACHE:
        return synth.chung_lu(n, m, gamma, seed=seed, tune_passes=tune_passes)
    base = os.path.join(GRAPH_CACHE, f"chunglu_{n}_{m}_{gamma}_{seed}_{tune_passes}")
    if os.path.exists(base + "_ci.npy"):
        rp = np.load(base + "_rp.npy", mmap_mode="r")
        ci = np.load(base + "_ci.npy", mmap_mode="r")
        meta = {"d_max": int(np.diff(rp).max())}
        return synth.CSRGraph(np.ascontiguousarray(rp), np.ascontiguousarray(ci), meta=meta)
    g = synth.chung_lu(n, m, gamma, seed=seed, tune_passes=tune_passes)
    os.makedirs(GRAPH_CACHE, exist_ok=True)
    np.save(base + "_rp.npy", g.row_ptr)
    np.save(base + "_ci.npy", g.col_idx)
    return g


def run_headline(args, torch, cp, synth):
    """The headline: a batch of PPR sources on the Friendster-shaped graph,
    timed over args.steps batches after args.warmup, with FP32 storage; the
    same batch with BF16 storage; every result's certified l1 distance to the
    exact vector; the plain-C oracle timed on one step of the same batch."""
    n_t, m_t, gamma, seed, alpha, nq, tol, prec = HEADLINES[args.headline]
    t0 = time.time()
    g = chung_lu(synth, n_t, m_t, gamma, seed, tune_passes=0 if n_t > 10_000_000 else 3)
    gen_s = time.time() - t0
    log(f"[headline] graph: n={g.n} nnz={g.nnz} d_max={g.meta['d_max']} ({gen_s:.1f}s)")
    t0 = time.time()
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=True, hot_split=not args.no_hot_split)
    create_s = time.time() - t0
    log(f"[headline] graph create (degree order, hot split {G.stats['hot_nodes']} nodes / "
        f"{G.stats['hot_arcs'] / g.nnz:.3f} of arcs) {create_s:.1f}s, device bytes {G.stats['device_bytes']}")
    srcs = [int(s) for s in synth.sources(g, nq, seed=seed)]
    qs = [cp.make_query("ppr", alpha, s, tol) for s in srcs]
    qt = [cp.make_query("ppr", alpha, s, tol, flags=cp.CP_Q_TIMING) for s in srcs]
    bw = G.autotune_batch(qs, prec=prec) if nq > 8 else 8
    G.set_batch_width(nq, prec, bw)
    deg = g.degrees

    def timed(p: str, Yp, warmup: int, steps: int):
        for _ in range(warmup):
            G.power_batch(qs, prec=p, Y=Yp)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        ev0.record()
        step_ms, launches, infos = 0.0, 0, None
        for _ in range(steps):
            _, infos = G.power_batch(qt, prec=p, Y=Yp)
            step_ms += infos[0]["step_ms"]
            launches += max(i["steps"] for i in infos)  # the batch runs until its longest query is done
        ev1.record()
        torch.cuda.synchronize()
        total_s = max(time.perf_counter() - w0, ev0.elapsed_time(ev1) * 1e-3)
        Ks = [i["K"] for i in infos]
        arcs = steps * sum((K - 1) * g.nnz + int(deg[s]) for K, s in zip(Ks, srcs))
        avg_launch_ms = step_ms / max(launches, 1)
        per_batch = batch_launch_bytes(g.n, g.nnz, p, Ks)
        per_batch_impl = batch_launch_bytes(g.n, g.nnz, p, Ks, impl_step_bytes)
        nl = max(Ks) - 1
        log(f"[headline] {p}: K {Ks}; {total_s / steps * 1e3:.1f} ms per batch; avg launch {avg_launch_ms:.3f} ms")
        return dict(total_s=total_s, Ks=Ks, arcs=arcs, avg_launch_ms=avg_launch_ms,
                    bytes_per_launch=per_batch / nl, impl_bytes_per_launch=per_batch_impl / nl, launches=launches)

    Y = torch.empty((g.n, nq), dtype=G.out_dtype(cp.PRECS[prec]), device="cuda")
    R = timed(prec, Y, args.warmup, args.steps)
    out = {
        "workload": f"{args.headline}: {nq} PPR alpha={alpha} sources in one batch, tol {tol} l1 (certified K), "
                    f"Chung-Lu n={n_t} m={m_t} gamma={gamma} seed={seed}, degree-ordered layout"
                    + ("" if args.no_hot_split else " with the hot/cold split of the batched step"),
        "value": R["arcs"] / R["total_s"] / 1e9,
        "total_s": R["total_s"], "n": g.n, "nnz": g.nnz, "d_max": int(deg.max()), "sources": nq, "Ks": R["Ks"],
        "prec": prec, "source_tile_width": bw, "generate_s": round(gen_s, 1), "create_s": round(create_s, 1),
        "hot_nodes": G.stats["hot_nodes"], "hot_arc_share": round(G.stats["hot_arcs"] / g.nnz, 4),
        "roofline": roofline(R["bytes_per_launch"], R["avg_launch_ms"], f"batch_step_kernel (width {bw})",
                             traffic=measured_traffic(f"{args.headline}:batch", BATCH_SOURCES),
                             implementation_bytes_per_launch=int(R["impl_bytes_per_launch"]),
                             launches_timed=R["launches"]),
        "launch_bytes_rule": "4 nnz + 8 (n+1) + 5 n B_k s per launch, B_k the sources still active in launch k",
    }
    results = {"f32": _host(Y)}
    if not args.no_bf16:
        Yb = torch.empty((g.n, nq), dtype=torch.float32, device="cuda")
        Rb = timed("bf16", Yb, 0, args.bf16_steps)
        if Rb["Ks"] != R["Ks"]:
            raise RuntimeError("BF16 batch took other K than the FP32 one")
        out["storage_bf16"] = {
            "workload": "the same batch with BF16 vector storage (float arithmetic and estimate)",
            "value": round(Rb["arcs"] / Rb["total_s"] / 1e9, 3), "unit": "GTEPS",
            "ms_per_batch": round(Rb["total_s"] * 1e3 / args.bf16_steps, 2), "steps": args.bf16_steps,
            "roofline": roofline(Rb["bytes_per_launch"], Rb["avg_launch_ms"], f"batch_step_kernel (width {bw})")}
        results["bf16"] = _host(Yb)
        del Yb
    if not args.no_f32f:
        Yf = torch.empty((g.n, nq), dtype=torch.float32, device="cuda")
        Rf = timed("f32f", Yf, 0, args.bf16_steps)
        if Rf["Ks"] != R["Ks"]:
            raise RuntimeError("FP32-arithmetic batch took other K than the FP32 one")
        out["arith_f32"] = {
            "workload": "the same batch with FP32 storage and FP32 arithmetic (float sums, float estimate and "
                        "float hot-pass partials; CP_F32F)",
            "value": round(Rf["arcs"] / Rf["total_s"] / 1e9, 3), "unit": "GTEPS",
            "ms_per_batch": round(Rf["total_s"] * 1e3 / args.bf16_steps, 2), "steps": args.bf16_steps,
            "roofline": roofline(Rf["bytes_per_launch"], Rf["avg_launch_ms"], f"batch_step_kernel (width {bw})",
                                 implementation_bytes_per_launch=int(Rf["impl_bytes_per_launch"]))}
        results["f32f"] = _host(Yf)
        del Yf
    del Y
    G.close()
    torch.cuda.empty_cache()
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import native as NO

        # every result: certified l1 distance to the exact PPR vector (FP32 and BF16 columns in one pass)
        names = list(results)
        Yall = np.concatenate([results[k] for k in names], axis=1)
        rows, cert_s = check_ppr_certificate(g, Yall, srcs * len(names), [alpha] * (nq * len(names)))
        acc = {}
        for i, k in enumerate(names):
            rk = rows[i * nq:(i + 1) * nq]
            acc[k] = {"worst": worst(rk, ["l1_bound_vs_exact"]),
                      "mass_range": [min(r["mass"] for r in rk), max(r["mass"] for r in rk)],
                      "per_source": rk}
        acc["method"] = (f"plain-C FP64 residual of Def. 3's fixed point, ||alpha e_s + (1-alpha) P y - y||_1 / "
                         f"alpha, for every result ({cert_s:.1f} s for {Yall.shape[1]} columns)")
        out["accuracy_vs_fp64_oracle"] = acc
        log("[headline] accuracy: " + ", ".join(f"{k} worst {acc[k]['worst']}" for k in names))
        del Yall, results
        # CPU baseline: the oracle's several-source Alg. 3 on the same batch, init and one full step
        c2 = [C.ppr_chebyshev_coeffs(alpha, 2)] * nq
        t0 = time.perf_counter()
        NO.cheby_power_multi(g.row_ptr, g.col_idx, srcs, c2, [2] * nq)
        cpu_s = time.perf_counter() - t0
        arcs_cpu = sum(g.nnz + int(deg[s]) for s in srcs)
        out["cpu_baseline"] = {
            "value": round(arcs_cpu / cpu_s / 1e9, 4), "unit": "GTEPS", "cores": NO.threads(), "kind": "oracle",
            "sample": f"the same {nq} sources, init plus one of their {max(R['Ks']) - 1} Chebyshev steps: plain-C "
                      f"FP64 Alg. 3 (several-source form, OpenMP node loop), {cpu_s:.1f} s",
            "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}
        log(f"[headline] cpu baseline {out['cpu_baseline']}")
    return out


def run_single(args, torch, cp, synth):
    """Single-source queries one at a time (the LiveJournal-shaped HKPR
    workload) on the XCD-striped layout, FP32 and BF16 storage; every result
    against the FP64 oracle; the oracle timed on the same queries on all
    host threads and on one."""
    n_t, m_t, gamma, seed, kind, param, tol, nsrc, prec = WORKLOADS[args.workload]
    t0 = time.time()
    g = chung_lu(synth, n_t, m_t, gamma, seed, tune_passes=0 if n_t > 10_000_000 else 3)
    log(f"[single] graph: n={g.n} nnz={g.nnz} d_max={g.meta['d_max']} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout == "degree", stripes=args.layout == "stripes")
    create_s = time.time() - t0
    log(f"[single] graph create (layout={args.layout}): {create_s:.2f}s, stats={G.stats}")
    srcs = [int(s) for s in synth.sources(g, nsrc, seed=seed)]
    Y = torch.empty((nsrc, g.n), dtype=G.out_dtype(cp.PRECS[prec]), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    steps = args.single_steps

    def one_step(timing: bool, p: str, Yp):
        # HIP events time every step of the last query of the step; that
        # query's CP_Q_TIMING synchronises, so the other queries are queued
        # behind it without a host round trip each
        infos = []
        for i, s in enumerate(srcs):
            timed = timing and i == nsrc - 1
            r = G.power(kind, param, s, tol=tol, prec=p, flags=cp.CP_Q_TIMING if timed else 0,
                        y=Yp[i], stream=stream)
            infos.append(r.info)
        return infos

    def timed_run(p: str, Yp, warmup: int):
        for _ in range(warmup):
            one_step(False, p, Yp)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        infos = []
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record()
        for _ in range(steps):
            infos += one_step(True, p, Yp)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        total_s = max(wall, ev0.elapsed_time(ev1) * 1e-3)
        arcs = sum((inf["K"] - 1) * g.nnz + int(g.degrees[s]) for inf, s in zip(infos, srcs * steps))
        timed = [inf for inf in infos if inf["step_ms"] == inf["step_ms"]]  # not NaN: the timed queries
        launches = sum(inf["steps"] for inf in timed)
        avg_step_ms = sum(inf["step_ms"] for inf in timed) / max(launches, 1)
        Ks = [inf["K"] for inf in infos[:nsrc]]
        log(f"[single] {p}: K per source: {Ks}; avg step kernel {avg_step_ms * 1e3:.1f} us; "
            f"wall {wall * 1e3:.1f} ms")
        return dict(value=arcs / total_s / 1e9, total_s=total_s, launches=launches, avg_step_ms=avg_step_ms,
                    Ks=Ks)

    R = timed_run(prec, Y, args.warmup)
    kern = "stripe_gather_kernel + stripe_combine_kernel" if args.layout == "stripes" else "step_kernel"
    out = {
        "workload": f"{args.workload}: {'HKPR t' if kind == 'hkpr' else 'PPR alpha'}={param}, {nsrc} sources one "
                    f"at a time, tol {tol} l1 (certified K), "
                    f"Chung-Lu n={n_t} m={m_t} gamma={gamma} seed={seed}",
        "value": round(R["value"], 3), "unit": "GTEPS", "steps": steps,
        "ms_per_step": round(R["total_s"] * 1e3 / steps, 3),
        "n": g.n, "nnz": g.nnz, "d_max": int(g.degrees.max()), "K_per_source": R["Ks"], "layout": args.layout,
        "prec": prec, "dtype": ARITH_DTYPE[prec], "graph_create_s": round(create_s, 3),
        "roofline": roofline(step_bytes(g.n, g.nnz, prec), R["avg_step_ms"], kern,
                             traffic=measured_traffic(f"{args.workload}:{args.layout}"),
                             implementation_bytes_per_launch=impl_step_bytes(g.n, g.nnz, prec),
                             launches_timed=R["launches"]),
    }
    results = {prec: Y.double().cpu().numpy().T}
    if not args.no_bf16:
        # the same queries with BF16 vector storage (float arithmetic and estimate)
        Yb = torch.empty((nsrc, g.n), dtype=torch.float32, device="cuda")
        B = timed_run("bf16", Yb, 1)
        if B["Ks"] != R["Ks"]:
            raise RuntimeError("BF16 query took another K than the FP32 one")
        out["storage_bf16"] = {
            "workload": "the same queries (graph, sources, steps, layout) with BF16 vector storage: float "
                        "arithmetic and a float estimate",
            "value": round(B["value"], 3), "unit": "GTEPS", "ms_per_step": round(B["total_s"] * 1e3 / steps, 3),
            "roofline": roofline(step_bytes(g.n, g.nnz, "bf16"), B["avg_step_ms"], kern)}
        results["bf16"] = Yb.double().cpu().numpy().T
        del Yb
    if not args.no_f32f:
        # the same queries with FP32 arithmetic (float sums, float partials and estimate)
        Yf = torch.empty((nsrc, g.n), dtype=torch.float32, device="cuda")
        F = timed_run("f32f", Yf, 1)
        if F["Ks"] != R["Ks"]:
            raise RuntimeError("FP32-arithmetic query took another K than the FP32 one")
        out["arith_f32"] = {
            "workload": "the same queries (graph, sources, steps, layout) with FP32 storage and FP32 arithmetic: "
                        "float sums, float stripe partials and a float estimate (CP_F32F)",
            "value": round(F["value"], 3), "unit": "GTEPS", "ms_per_step": round(F["total_s"] * 1e3 / steps, 3),
            "roofline": roofline(step_bytes(g.n, g.nnz, "f32f"), F["avg_step_ms"], kern,
                                 implementation_bytes_per_launch=impl_step_bytes(g.n, g.nnz, "f32f"))}
        results["f32f"] = Yf.double().cpu().numpy().T
        del Yf
    G.close()
    del Y
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import native as NO

        acc, refs = {}, {}
        for p, Yh in results.items():
            rows, oracle_s = check_same_k_and_exact(g, Yh, [kind] * nsrc, [param] * nsrc, srcs, R["Ks"],
                                                    refs=refs)
            acc[p] = {"results": len(rows),
                      "worst": worst(rows, ["l1_vs_same_K", "max_abs_vs_same_K", "l1_vs_exact", "max_abs_vs_exact",
                                            "norm_rel_err_vs_exact"]),
                      "mass_range": [min(r["mass"] for r in rows), max(r["mass"] for r in rows)]}
            log(f"[single] accuracy {p}: {acc[p]}")
        acc["method"] = ("every result against plain-C FP64 Alg. 3 at the same K (several-source form) and the "
                         "converged vector (plain-C FP64 PwMethod, exact tail 1e-15); Normalized RelErr is Def. 5's "
                         "degree-normalized error")
        out["accuracy_vs_fp64_oracle"] = acc
        # the oracle on the timed workload: the 16 queries one at a time on all host threads, and the
        # first query on one thread
        cs = [C.chebyshev_coeffs(kind, param, K) for K in R["Ks"]]
        arcs = sum((K - 1) * g.nnz + int(g.degrees[s]) for K, s in zip(R["Ks"], srcs))
        t0 = time.perf_counter()
        for s, c, K in zip(srcs, cs, R["Ks"]):
            NO.cheby_power(g.row_ptr, g.col_idx, s, c, K)
        all_s = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(arcs / all_s / 1e9, 4), "unit": "GTEPS", "cores": NO.threads(), "kind": "oracle",
            "sample": f"all {nsrc} queries of one step, one at a time, same K: plain-C FP64 Alg. 3 (OpenMP node "
                      f"loop), {all_s:.2f} s"}
        NO.set_threads(1)
        try:
            t0 = time.perf_counter()
            NO.cheby_power(g.row_ptr, g.col_idx, srcs[0], cs[0], R["Ks"][0])
            one_s = time.perf_counter() - t0
        finally:
            NO.set_threads(0)
        out["cpu_baseline_1thread"] = {
            "value": round(((R["Ks"][0] - 1) * g.nnz + int(g.degrees[srcs[0]])) / one_s / 1e9, 4), "unit": "GTEPS",
            "cores": 1, "kind": "oracle",
            "sample": f"the first of the {nsrc} queries, same K: plain-C FP64 Alg. 3 on one thread, {one_s:.2f} s"}
        log(f"[single] cpu baselines {out['cpu_baseline']} {out['cpu_baseline_1thread']}")
    return out, g


def run_batch(args, torch, cp, synth):
    """64 PPR sources with mixed tolerances in one batch (the Orkut-shaped
    workload), FP32 and BF16 storage, autotuned source-tile width; every
    column's certified distance to the exact vector, and the rounding error
    of the tightest column of each tolerance class against Alg. 3 at the
    same K."""
    n_t, m_t, gamma, seed, alpha, nq, tol_choices, prec = BATCH_WORKLOADS[args.batch_workload]
    t0 = time.time()
    g = chung_lu(synth, n_t, m_t, gamma, seed)
    log(f"[batch] graph: n={g.n} nnz={g.nnz} d_max={g.meta['d_max']} ({time.time() - t0:.1f}s)")
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout != "native" or args.batch_hot_split,
                 hot_split=args.batch_hot_split)
    srcs = [int(s) for s in synth.sources(g, nq, seed=seed)]
    tols = [float(t) for t in synth.tolerance_choice(seed, nq, tol_choices)]
    qs = [cp.make_query("ppr", alpha, s, t) for s, t in zip(srcs, tols)]
    bw = G.autotune_batch(qs, prec=prec)
    log(f"[batch] autotuned source-tile width {bw}")
    qt = [cp.make_query("ppr", alpha, s, t, flags=cp.CP_Q_TIMING) for s, t in zip(srcs, tols)]
    nb = max(1, args.steps // 2)
    deg = g.degrees

    def timed_batches(p: str, Yp):
        for _ in range(max(1, args.warmup)):
            G.power_batch(qs, prec=p, Y=Yp)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        step_ms = 0.0
        launches = 0
        infos = None
        for _ in range(nb):
            _, infos = G.power_batch(qt, prec=p, Y=Yp)
            step_ms += infos[0]["step_ms"]
            launches += max(i["steps"] for i in infos)  # the batch runs until its longest query is done
        torch.cuda.synchronize()
        total_s = time.perf_counter() - w0
        Ks = [i["K"] for i in infos]
        arcs = nb * sum((k - 1) * g.nnz + int(deg[s]) for k, s in zip(Ks, srcs))
        nl = max(Ks) - 1
        return dict(total_s=total_s, Ks=Ks, arcs=arcs, avg_launch_ms=step_ms / max(launches, 1),
                    bytes_per_launch=batch_launch_bytes(g.n, g.nnz, p, Ks) / nl,
                    impl_bytes_per_launch=batch_launch_bytes(g.n, g.nnz, p, Ks, impl_step_bytes) / nl,
                    launches=launches)

    Yb = torch.empty((g.n, nq), dtype=G.out_dtype(cp.PRECS[prec]), device="cuda")
    R = timed_batches(prec, Yb)
    out = {
        "workload": f"{args.batch_workload}: {nq} PPR alpha={alpha} sources in one batch, tol per source from "
                    f"{list(tol_choices)} (certified K), Chung-Lu n={n_t} m={m_t} gamma={gamma} seed={seed}"
                    + (f", hot/cold split ({G.stats['hot_nodes']} hot nodes, "
                       f"{G.stats['hot_arcs'] / g.nnz:.3f} of the arcs)" if args.batch_hot_split else ""),
        "value": round(R["arcs"] / R["total_s"] / 1e9, 3), "unit": "GTEPS",
        "ms_per_batch": round(R["total_s"] * 1e3 / nb, 3), "batches": nb,
        "n": g.n, "nnz": g.nnz, "source_tile_width": bw, "K_min": min(R["Ks"]), "K_max": max(R["Ks"]),
        "roofline": roofline(R["bytes_per_launch"], R["avg_launch_ms"], f"batch_step_kernel (width {bw})",
                             traffic=None if args.batch_hot_split else
                             measured_traffic(f"{args.batch_workload}:batch", BATCH_SOURCES),
                             implementation_bytes_per_launch=int(R["impl_bytes_per_launch"]),
                             launches_timed=R["launches"]),
    }
    results = {prec: _host(Yb)}
    Ks = R["Ks"]
    if not args.no_bf16:
        # the same batch with BF16 storage (float arithmetic and estimate), its own autotuned width
        del Yb
        bwb = G.autotune_batch(qs, prec="bf16")
        Ybb = torch.empty((g.n, nq), dtype=torch.float32, device="cuda")
        Rb = timed_batches("bf16", Ybb)
        if Rb["Ks"] != Ks:
            raise RuntimeError("BF16 batch took other K than the FP32 one")
        out["storage_bf16"] = {
            "workload": "the same batch with BF16 vector storage (float arithmetic and estimate)",
            "value": round(Rb["arcs"] / Rb["total_s"] / 1e9, 3), "unit": "GTEPS",
            "ms_per_batch": round(Rb["total_s"] * 1e3 / nb, 3), "source_tile_width": bwb,
            "roofline": roofline(Rb["bytes_per_launch"], Rb["avg_launch_ms"], f"batch_step_kernel (width {bwb})")}
        results["bf16"] = _host(Ybb)
        del Ybb
        log(f"[batch] bf16 storage: {out['storage_bf16']}")
    G.close()
    torch.cuda.empty_cache()
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import errors as E
        from oracle import native as NO

        acc = {}
        # the tightest-tolerance column of each class: rounding error against Alg. 3 at the same K
        pick = sorted({min((j for j in range(nq) if tols[j] == t), key=lambda j: -Ks[j]) for t in set(tols)})
        t0 = time.perf_counter()
        ref = NO.cheby_power_multi(g.row_ptr, g.col_idx, [srcs[j] for j in pick],
                                   [C.ppr_chebyshev_coeffs(alpha, Ks[j]) for j in pick], [Ks[j] for j in pick])
        same_k_s = time.perf_counter() - t0
        for p, Yh in results.items():
            rows, cert_s = check_ppr_certificate(g, Yh, srcs, [alpha] * nq)
            for r, t in zip(rows, tols):
                r["tol"] = t
                r["meets_tol"] = r["l1_bound_vs_exact"] <= t
            same_k = [{"column": j, "tol": tols[j], "K": Ks[j], "l1": E.l1(Yh[:, j], ref[:, i]),
                       "max_abs": E.max_abs(Yh[:, j], ref[:, i])} for i, j in enumerate(pick)]
            acc[p] = {"results": len(rows),
                      "worst_l1_bound_by_tol": {str(t): max(r["l1_bound_vs_exact"] for r in rows if r["tol"] == t)
                                                for t in sorted(set(tols))},
                      "all_meet_tol": all(r["meets_tol"] for r in rows),
                      "mass_range": [min(r["mass"] for r in rows), max(r["mass"] for r in rows)],
                      "same_K_rounding": same_k}
            log(f"[batch] accuracy {p}: {acc[p]}")
        acc["method"] = (f"every column: plain-C FP64 residual of Def. 3's fixed point / alpha, a certified bound on "
                         f"the l1 distance to the exact vector ({cert_s:.1f} s per precision); the tightest column of "
                         f"each tolerance class also against plain-C FP64 Alg. 3 at the same K ({same_k_s:.1f} s)")
        out["accuracy_vs_fp64_oracle"] = acc
    return out


SERVE_KINDS = [("ppr", 0.1), ("ppr", 0.2), ("hkpr", 3.0), ("hkpr", 5.0), ("hkpr", 10.0)]


def serve_trace(g, synth, seconds: float, rate: float, seed: int = 4):
    """Seeded Poisson arrivals: exponential gaps, kind uniform over the five
    GP functions, tolerance log-uniform in [1e-7, 1e-4], uniform sources."""
    nmax = int(seconds * rate * 2 + 50)
    u = synth.uniform01(seed ^ 0xA11, nmax)
    gaps = -np.log1p(-u) / rate
    t = np.cumsum(gaps)
    n = int(np.searchsorted(t, seconds))
    kinds = synth.uniform_ints(seed ^ 0xB22, n, len(SERVE_KINDS))
    tols = synth.tolerance_loguniform(seed ^ 0xC33, n, 1e-7, 1e-4)
    srcs = synth.sources(g, n, seed=seed ^ 0xD44)
    return [(float(t[i]), *SERVE_KINDS[int(kinds[i])], int(srcs[i]), float(tols[i])) for i in range(n)]


def _pct(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if len(xs) else None


def _lat_summary(lat, span_s, extra=None, done=None):
    """Latency percentiles of lat (ms) and the throughput: done completions
    (default len(lat)) over span_s seconds."""
    done = len(lat) if done is None else done
    out = {"completed": len(lat), "qps": round(done / span_s, 1) if span_s > 0 else None,
           "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "mean_ms": float(np.mean(lat)) if lat else None,
           "span_s": round(span_s, 3)}
    if extra:
        out.update(extra)
    return out


def run_serve(args, torch, cp, synth, g):
    """Served query stream on the LiveJournal-shaped graph: the batched
    server against plain one-at-a-time queries (same graph, FP32) on the
    same seeded Poisson traces, at the configured rate for the configured
    time after a warm-up, and at a lower rate that plain sustains.  The
    latency of a query is its completion time minus its arrival time; the
    first warm-up seconds of a trace are not counted."""
    warm = args.serve_warmup
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout != "native", stripes=args.layout == "stripes")
    nbuf = 512  # one result buffer per server slot
    bufs = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in range(nbuf)]
    S = cp.Server(G, hbm_budget_bytes=16 << 30, max_slots=512, max_queue=100000, prec="f32")
    stream = torch.cuda.current_stream().cuda_stream
    first = serve_trace(g, synth, 1.0, 50.0, seed=3)
    for (_, kind, param, s, tol) in first[:8]:  # code objects and caches, both paths
        G.power(kind, param, s, tol=tol, prec="f32", y=bufs[0])
        S.wait(S.submit(cp.make_query(kind, param, s, tol), bufs[1]))
    torch.cuda.synchronize()

    def replay_server(tr):
        """Submit at the trace's arrival times; results land in a ring of
        buffers (a buffer is reused once its previous query is done)."""
        tickets = [None] * len(tr)
        t0 = time.perf_counter()
        for i, (ta, kind, param, s, tol) in enumerate(tr):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            if i >= nbuf:
                tickets[i - nbuf] = S.wait(tickets[i - nbuf])
            tickets[i] = S.submit(cp.make_query(kind, param, s, tol), bufs[i % nbuf])
            if i and i % 4000 == 0:
                log(f"[serve] server: {i} of {len(tr)} queries submitted")
        for i in range(max(0, len(tr) - nbuf), len(tr)):
            if not isinstance(tickets[i], tuple):
                tickets[i] = S.wait(tickets[i])
        return tickets, time.perf_counter() - t0

    def server_leg(tr, rate):
        st0 = S.stats()
        tickets, t_end = replay_server(tr)
        counted = [(info["latency_ms"], info["K"]) for (ta, *_), (st, info) in zip(tr, tickets)
                   if st == cp.CP_OK and ta >= warm]
        lat = [x for x, _ in counted]
        span = t_end - warm
        done = sum(1 for (ta, *_), (st, info) in zip(tr, tickets)
                   if st == cp.CP_OK and ta + info["latency_ms"] * 1e-3 >= warm)
        st = S.stats()
        return _lat_summary(lat, span, {"offered_qps": rate, "arrivals_counted": sum(1 for x in tr if x[0] >= warm),
                                        "batched_launches": st["ticks"] - st0["ticks"],
                                        "narrow_launches": st["narrow_ticks"] - st0["narrow_ticks"],
                                        "single_source_path": st["direct"] - st0["direct"],
                                        "single_source_queue_limit": st["direct_limit"], "slots": st["slots"],
                                        "tile_width": st["tile_width"],
                                        "mean_K": float(np.mean([k for _, k in counted])) if counted else None},
                            done=done)

    def plain_leg(tr, rate, limit_s):
        """FIFO, one cp_power at a time; stops once limit_s of wall time has
        passed (the queue of an overloaded plain path only grows).  Latency
        counts the queries that arrive after the warm-up; throughput counts
        every query completed after it, also those that arrived during it
        (an overloaded queue still holds them)."""
        lat, t0, stopped, done = [], time.perf_counter(), False, 0
        for (ta, kind, param, s, tol) in tr:
            now = time.perf_counter() - t0
            if now > limit_s:
                stopped = True
                break
            if ta > now:
                time.sleep(ta - now)
            G.power(kind, param, s, tol=tol, prec="f32", y=bufs[0], stream=stream)
            torch.cuda.synchronize()
            t_done = time.perf_counter() - t0
            done += t_done >= warm
            if ta >= warm:
                lat.append((t_done - ta) * 1e3)
        span = time.perf_counter() - t0 - warm
        extra = {"offered_qps": rate}
        if stopped:
            extra["stopped_after_s"] = limit_s
            extra["note"] = (f"plain falls behind the offered rate, so its queue grows for as long as the trace "
                             f"runs; it was stopped after {limit_s:g} s of wall time, and its latencies are those of "
                             f"the queries completed by then")
        return _lat_summary(lat, span, extra, done=done)

    out = {"workload": f"Poisson arrivals, PPR alpha in {{0.1, 0.2}}, HKPR t in {{3, 5, 10}} uniformly, tol "
                       f"log-uniform [1e-7, 1e-4] (certified K), FP32 resident state, on the single-source "
                       f"workload's graph; latency = completion - arrival, the first {warm:g} s of each trace are "
                       f"warm-up and not counted",
           "rates": []}
    for rate, seconds, plain_limit in ((args.serve_rate, args.serve_seconds, args.plain_limit_s),
                                       (args.serve_rate_low, args.serve_seconds_low, None)):
        if seconds <= 0 or rate <= 0:
            continue
        tr = serve_trace(g, synth, seconds + warm, rate, seed=4 if rate == args.serve_rate else 6)
        srv = server_leg(tr, rate)
        log(f"[serve] {rate}/s server: {srv}")
        pl = plain_leg(tr, rate, plain_limit if plain_limit else float("inf"))
        log(f"[serve] {rate}/s plain: {pl}")
        out["rates"].append({"offered_qps": rate, "trace_s": seconds + warm, "queries": len(tr), "server": srv,
                             "plain": pl, "p99_ratio_plain_over_server":
                             round(pl["p99_ms"] / srv["p99_ms"], 2) if pl["p99_ms"] and srv["p99_ms"] else None})
    if args.saturation_rate > 0:
        burst = serve_trace(g, synth, 1.0, args.saturation_rate, seed=7)
        bt, b_end = replay_server(burst)
        blat = [info["latency_ms"] for st, info in bt if st == cp.CP_OK]
        out["server_saturation"] = _lat_summary(blat, b_end, {
            "offered_qps": args.saturation_rate, "queries": len(burst),
            "latency_from": "submission (a submit waits for a free result buffer)"})
        log(f"[serve] saturation burst: {out['server_saturation']}")
    if not args.no_cpu and args.serve_check > 0:
        # served results against the FP64 oracle: queries spread over the first trace, rerun
        # through the server into buffers of their own
        tr = serve_trace(g, synth, args.serve_seconds + warm, args.serve_rate, seed=4)
        idx = np.linspace(0, len(tr) - 1, min(args.serve_check, len(tr))).astype(int)
        pend = [(S.submit(cp.make_query(tr[i][1], tr[i][2], tr[i][3], tr[i][4]), bufs[k]), i)
                for k, i in enumerate(idx)]
        got = [(S.wait(t), i) for t, i in pend]
        if any(st != cp.CP_OK for (st, _), _ in got):
            raise RuntimeError("served check query failed")
        Yh = torch.stack([bufs[k] for k in range(len(idx))], dim=1).double().cpu().numpy()
        rows, oracle_s = check_same_k_and_exact(g, Yh, [tr[i][1] for i in idx], [tr[i][2] for i in idx],
                                                [tr[i][3] for i in idx], [info["K"] for (_, info), _ in got],
                                                chebyshev_for_ppr=True)
        for r, i in zip(rows, idx):
            r["tol"] = tr[i][4]
            r["meets_tol"] = r["l1_vs_exact"] <= tr[i][4]
        out["accuracy_vs_fp64_oracle"] = {
            "results": len(rows), "all_meet_tol": all(r["meets_tol"] for r in rows),
            "worst": worst(rows, ["l1_vs_same_K", "max_abs_vs_same_K", "l1_vs_exact", "norm_rel_err_vs_exact"]),
            "worst_l1_over_tol": max(r["l1_vs_exact"] / r["tol"] for r in rows),
            "mass_range": [min(r["mass"] for r in rows), max(r["mass"] for r in rows)],
            "method": f"{len(rows)} queries spread over the trace, rerun through the server: plain-C FP64 Alg. 3 at "
                      f"the same K and the converged vector (plain-C PwMethod with tail 1e-15 for HKPR, plain-C "
                      f"Alg. 3 with the certified K for l1 1e-12 for PPR), {oracle_s:.1f} s"}
        log(f"[serve] accuracy {out['accuracy_vs_fp64_oracle']}")
    S.close()
    G.close()
    return out


KVN_CASES = [("ppr", 0.2), ("ppr", 0.05), ("ppr", 0.01), ("hkpr", 5.0), ("hkpr", 20.0)]


def run_kvn(args, torch, cp, synth, g):
    """ChebyPower (Alg. 3) against PwMethod (Alg. 1) on the main line's graph
    at the same l1 guarantee: K from the certified Chebyshev tail, N from the
    exact Taylor tail, both in FP64 so neither is limited by storage
    rounding.  Reports K, N and the device time of each query."""
    tol, nsrc = args.kvn_tol, 2
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout == "degree", stripes=args.layout == "stripes")
    srcs = [int(s) for s in synth.sources(g, nsrc, seed=11)]
    y = torch.empty(g.n, dtype=torch.float64, device="cuda")
    G.power("ppr", 0.2, srcs[0], tol=tol, prec="f64", y=y)  # warm-up
    G.power("ppr", 0.2, srcs[0], tol=tol, prec="f64", y=y, method="power")
    rows = []
    for kind, param in KVN_CASES:
        row = {"kind": kind, "param": param, "tol": tol}
        for method in ("cheby", "power"):
            ms, steps, K, bound = [], 0, [], []
            for s in srcs:
                r = G.power(kind, param, s, tol=tol, prec="f64", y=y, method=method, flags=cp.CP_Q_TIMING)
                ms.append(r.info["elapsed_ms"])
                K.append(r.info["K"])
                bound.append(r.info["tail_bound_l1"])
            key = "K" if method == "cheby" else "N"
            row[key] = K
            row[f"ms_{method}"] = round(float(np.mean(ms)), 3)
            row[f"l1_bound_{method}"] = max(bound)
        row["N_over_K"] = round(float(np.mean(row["N"]) / np.mean(row["K"])), 2)
        row["speedup"] = round(row["ms_power"] / row["ms_cheby"], 2)
        rows.append(row)
        log(f"[kvn] {row}")
    out = {"workload": f"{nsrc} sources, tol {tol} l1, FP64, on the main line's graph ({args.layout} layout): "
                       f"ChebyPower with the certified K vs PwMethod with the exact-tail N",
           "rows": rows}
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import errors as E
        from oracle import native as NO
        from oracle import truncation as T

        kind, param, s = "ppr", 0.2, srcs[0]
        Nref = T.pwmethod_steps(kind, param, 1e-15)
        t0 = time.perf_counter()
        ref = NO.power_method(g.row_ptr, g.col_idx, s, C.taylor_coeffs(kind, param, Nref), Nref)
        ref_s = time.perf_counter() - t0
        acc = {"source": s, "kind": kind, "param": param,
               "reference": f"plain-C FP64 PwMethod with tail 1e-15 (N={Nref}, {ref_s:.1f} s)"}
        for method in ("cheby", "power"):
            r = G.power(kind, param, s, tol=tol, prec="f64", y=y, method=method)
            v = y.cpu().numpy()
            acc[method] = {"K": r.info["K"], "l1": E.l1(v, ref), "l1_bound": r.info["tail_bound_l1"]}
        out["accuracy_vs_fp64_oracle"] = acc
        log(f"[kvn] accuracy {acc}")
    G.close()
    return out


def run_propagate(args, torch, cp, synth, g):
    """Feature-matrix propagation (Def. 8 through Thm. 5) on the main line's
    graph: Z = f(D^{-1/2} A D^{-1/2}) X for X [n x k] FP32, PPR alpha = 0.1,
    K from the Thm. 2 tail at 1e-6 (the certified rule needs norms of X)."""
    k, alpha, tol, a = args.propagate_cols, 0.1, 1e-6, 0.5
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=True)
    X = (torch.rand((g.n, k), generator=torch.Generator().manual_seed(5), dtype=torch.float32) - 0.5).cuda()
    Z = torch.empty_like(X)
    G.propagate(X, "ppr", alpha, a=a, tol=tol, prec="f32", Z=Z)  # warm-up (default width)
    best = None
    for w in (16, 32, 64):  # same tile widths as the batched kernel; keep the fastest
        if w > max(8, k):  # widths above the column count are not allowed
            continue
        G.set_batch_width(k, "f32", w)
        _, info = G.propagate(X, "ppr", alpha, a=a, tol=tol, prec="f32", Z=Z, flags=cp.CP_Q_TIMING)
        if best is None or info["elapsed_ms"] < best[1]:
            best = (w, info["elapsed_ms"])
    bw = best[0]
    G.set_batch_width(k, "f32", bw)
    reps, ms, steps = 3, 0.0, 0
    for _ in range(reps):
        _, info = G.propagate(X, "ppr", alpha, a=a, tol=tol, prec="f32", Z=Z, flags=cp.CP_Q_TIMING)
        ms += info["elapsed_ms"]
        step_ms = info["step_ms"]
        steps = info["steps"]
    ms /= reps
    K = info["K"]
    bpl = step_bytes(g.n, g.nnz, "f32", k)
    # the same series by Clenshaw's backward recurrence (no estimate vector)
    Zc = torch.empty_like(X)
    G.propagate(X, "ppr", alpha, a=a, tol=tol, prec="f32", Z=Zc, method="clenshaw")
    msc = 0.0
    for _ in range(reps):
        _, ic = G.propagate(X, "ppr", alpha, a=a, tol=tol, prec="f32", Z=Zc, flags=cp.CP_Q_TIMING,
                            method="clenshaw")
        msc += ic["elapsed_ms"]
    msc /= reps
    bplc = clenshaw_step_bytes(g.n, g.nnz, "f32", k)
    stepc = ic["step_ms"] / ic["steps"]
    diff = float(((Zc - Z).abs().sum(0) / Z.abs().sum(0)).max())
    out = {"workload": f"Z = f(D^-1/2 A D^-1/2) X, X [n x {k}] FP32, PPR alpha={alpha}, K={K} (Thm. 2 tail "
                       f"{tol}), degree-ordered layout, on the main line's graph",
           "GTEPS": round(g.nnz * steps * k / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 2), "K": K,
           "source_tile_width": bw,
           "roofline": {"bound": "hbm", "kernel": "batch_step_kernel", "achieved":
                        round(bpl / (step_ms / steps * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": round(bpl / (step_ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                        "avg_launch_ms": round(step_ms / steps, 3)},
           "clenshaw": {"ms": round(msc, 2), "K": ic["K"], "steps": ic["steps"],
                        "GTEPS": round(g.nnz * ic["steps"] * k / (msc * 1e-3) / 1e9, 2),
                        "speedup_vs_forward": round(ms / msc, 3),
                        "roofline": {"bound": "hbm", "kernel": "batch_step_kernel (Clenshaw mode)",
                                     "achieved": round(bplc / (stepc * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                                     "unit": "GB/s", "frac": round(bplc / (stepc * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                     "avg_launch_ms": round(stepc, 3)},
                        "max_column_rel_l1_vs_forward": diff}}
    if not args.no_cpu:
        from oracle import errors as E
        from oracle import generalized as GG

        j = 0
        Xc = X[:, j:j + 1].double().cpu().numpy()
        ref = GG.generalized_gp(g.row_ptr, g.col_idx, Xc, a, "ppr", alpha, K)[:, 0]
        zj = Z[:, j].double().cpu().numpy()
        out["accuracy_vs_fp64_oracle"] = {"column": j, "rel_l1": E.l1(zj, ref) / float(np.abs(ref).sum())}
        refc = GG.generalized_gp(g.row_ptr, g.col_idx, Xc, a, "ppr", alpha, K, method="clenshaw")[:, 0]
        zc = Zc[:, j].double().cpu().numpy()
        out["clenshaw"]["accuracy_vs_fp64_oracle"] = {"column": j, "rel_l1": E.l1(zc, refc) / float(np.abs(refc).sum())}
    log(f"[propagate] {out}")
    G.close()
    return out


def run_push(args, torch, cp, synth, g):
    """ChebyPush (Alg. 4) against ChebyPower (Alg. 3) on the main line's graph:
    K from Thm. 2's tail at eps_a / 2 (Thm. 4's setting), both FP64; the
    push's work (sum of vol(S_k)) against the global iteration's (K - 1) nnz,
    device time of each, and the degree-normalised distance between them."""
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout == "degree", stripes=args.layout == "stripes")
    srcs = [int(s) for s in synth.sources(g, 2, seed=13)]
    deg = torch.tensor(g.degrees, dtype=torch.float64, device="cuda")
    G.push("hkpr", 5.0, srcs[0], 1e-6, tol=5e-7, kmode="tail")  # warm-up
    rows = []
    for kind, param in (("hkpr", 5.0), ("ppr", 0.2)):
        for eps_a in args.push_eps:
            row = {"kind": kind, "param": param, "eps_a": eps_a}
            ms_p, ms_c, arcs, pushes, dn = [], [], [], [], []
            for s in srcs:
                rp = G.push(kind, param, s, eps_a, tol=eps_a / 2, kmode="tail", flags=cp.CP_Q_TIMING)
                rc = G.power(kind, param, s, tol=eps_a / 2, kmode="tail", prec="f64", flags=cp.CP_Q_TIMING)
                K = rp.info["K"]
                ms_p.append(rp.info["elapsed_ms"])
                ms_c.append(rc.info["elapsed_ms"])
                arcs.append(rp.info["arcs"])
                pushes.append(rp.info["pushes"])
                live = deg > 0
                dn.append(float(((rp.y - rc.y).abs()[live] / deg[live]).max()))
            row.update(K=K, ms_push=round(float(np.mean(ms_p)), 3), ms_power_f64=round(float(np.mean(ms_c)), 3),
                       speedup=round(float(np.mean(ms_c)) / float(np.mean(ms_p)), 2),
                       push_arcs=int(np.mean(arcs)), power_arcs=(K - 1) * g.nnz, pushes=int(np.mean(pushes)),
                       work_fraction=round(float(np.mean(arcs)) / ((K - 1) * g.nnz), 4),
                       deg_norm_vs_power=max(dn))
            rows.append(row)
            log(f"[push] {row}")
    G.close()
    return {"workload": "ChebyPush vs ChebyPower, 2 sources, FP64, K from the Thm. 2 tail at eps_a / 2, "
                        f"on the main line's graph ({args.layout} layout); deg_norm_vs_power = max_u |y_push - "
                        "y_power| / d_u (Thm. 4 bounds the push's own error by eps_a)", "rows": rows}


def run_push_rw(args, torch, cp, synth, g):
    """ChebyPush + random walks (Alg. 5) for SSPPR on the main line's graph with
    the paper's parameters: eps_r = 0.5, delta = 1/n, r_max = sqrt(alpha)/W,
    K = ln(1/r_max)/sqrt(alpha); accuracy against a plain-C FP64 reference."""
    alpha, eps_r = 0.2, 0.5
    delta = 1.0 / g.n
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout == "degree", stripes=args.layout == "stripes")
    srcs = [int(s) for s in synth.sources(g, 2, seed=17)]
    G.push_rw(alpha, srcs[0], eps_r, delta, seed=1)  # warm-up
    rows = []
    for i, s in enumerate(srcs):
        r = G.push_rw(alpha, s, eps_r, delta, seed=100 + i, flags=cp.CP_Q_TIMING | cp.CP_Q_STATS)
        rc = G.power("ppr", alpha, s, tol=1e-7, prec="f64", flags=cp.CP_Q_TIMING)
        row = {"source": s, "K": r.info["K"], "ms": round(r.info["elapsed_ms"], 2),
               "ms_push_phase": round(r.info["step_ms"], 2), "pushes": r.info["pushes"], "arcs": r.info["arcs"],
               "walks": r.info["walks"], "walk_moves": r.info["walk_steps"], "mass": r.info["mass"],
               "chebypower_f64_ms_at_l1_1e-7": round(rc.info["elapsed_ms"], 2)}
        if not args.no_cpu and i == 0:
            from oracle import coefficients as C
            from oracle import native as NO
            from oracle import truncation as T

            N = T.pwmethod_steps("ppr", alpha, 1e-15)
            exact = NO.power_method(g.row_ptr, g.col_idx, s, C.taylor_coeffs("ppr", alpha, N), N)
            y = r.y.cpu().numpy()
            big = exact > delta
            row["max_rel_err_where_pi_gt_delta"] = float(np.max(np.abs(y[big] - exact[big]) / exact[big]))
            row["nodes_with_pi_gt_delta"] = int(np.count_nonzero(big))
        rows.append(row)
        log(f"[push_rw] {row}")
    G.close()
    return {"workload": f"Alg. 5 for SSPPR alpha={alpha}, eps_r={eps_r}, delta=1/n, r_max and K as the paper sets "
                        f"them, on the main line's graph ({args.layout} layout); the relative error is checked "
                        "against a plain-C FP64 PwMethod with tail 1e-15", "rows": rows}


def run_latency(args, torch, cp, synth):
    """Query latency where launches dominate: PPR alpha = 0.2, FP64, l1
    tolerance 1e-8 (certified K) on the small Chung-Lu graph (n = 20,000,
    average degree 10, exponent 2.5).  The same query is issued eagerly and
    as a replay of a HIP graph that captured it (the library issues kernels
    only, with coefficients and ids as kernel arguments); every replay must
    equal the eager result bit for bit."""
    g = synth.chung_lu(20_000, 100_000, 2.5, seed=1)
    s = int(synth.sources(g, 1, seed=5)[0])
    G = cp.Graph(g.row_ptr, g.col_idx)
    Gc = cp.Graph(g.row_ptr, g.col_idx)  # its workspace stays bound to the captured graph
    y = torch.empty(g.n, dtype=torch.float64, device="cuda")
    yc = torch.empty(g.n, dtype=torch.float64, device="cuda")
    q = dict(kind="ppr", param=0.2, source=s, tol=1e-8, prec="f64")
    st = torch.cuda.current_stream()
    K = G.power(**q, y=y).info["K"]
    ref = y.clone()

    def one(fn, reps):
        lat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            st.synchronize()
            lat.append((time.perf_counter() - t0) * 1e6)
        lat.sort()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        st.synchronize()
        return lat[len(lat) // 2], (time.perf_counter() - t0) * 1e6 / reps

    eager = lambda: G.power(**q, y=y, stream=st.cuda_stream)
    one(eager, 20)
    e_p50, e_pipe = one(eager, 200)
    Gc.power(**q, y=yc)  # sizes the workspace outside the capture
    st.synchronize()
    hg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(hg):
        Gc.power(**q, y=yc, stream=torch.cuda.current_stream().cuda_stream)
    replay = hg.replay
    one(replay, 20)
    yc.fill_(-1.0)
    g_p50, g_pipe = one(replay, 200)
    same = bool(torch.equal(yc, ref))
    G.close()
    out = {"workload": "PPR alpha=0.2, 1 source, FP64, l1 tol 1e-8 (certified K) on a Chung-Lu graph "
                       f"n={g.n}, nnz={g.nnz}, exponent 2.5 (caller order)",
           "K": K, "eager_us_p50": round(e_p50, 1), "eager_us_back_to_back": round(e_pipe, 1),
           "hipgraph_us_p50": round(g_p50, 1), "hipgraph_us_back_to_back": round(g_pipe, 1),
           "hipgraph_equals_eager": same}
    if not args.no_cpu:
        from oracle import propagation as PR

        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        exact = PR.ground_truth(P, s, "ppr", 0.2)
        out["l1_vs_fp64_fixed_point"] = float(np.abs(ref.cpu().numpy() - exact).sum())
    log(f"[latency] {out}")
    if not same:
        raise RuntimeError("HIP graph replay differs from the eager query")
    return out


def run_gather_footprint(args, torch, cp):
    """Gather rate of the batched step kernel against the size of the set of
    rows it gathers from.  Synthetic CSR: n rows of d arcs whose columns are
    uniform over the first F rows, so one launch gathers n d rows of bw
    values from a slice of F bw s bytes; F from L2-sized (4 MiB per XCD)
    through Infinity-Cache-sized (256 MiB) to HBM-sized.  Timing only: the
    graph is not symmetric and the values are not a propagation."""
    n, d = args.footprint_rows, 8
    rows = []
    stream = torch.cuda.current_stream().cuda_stream
    rp = np.arange(n + 1, dtype=np.int64) * d
    gen = torch.Generator(device="cuda").manual_seed(11)
    for bw in (8, 32):
        for F in (16_384, 65_536, 131_072, 524_288, 2_097_152, 8_388_608, n):
            if F > n:
                continue
            ci = torch.randint(0, F, (n * d,), generator=gen, device="cuda", dtype=torch.int32)
            G = cp.Graph(torch.from_numpy(rp).cuda(), ci, host_input=False)
            del ci
            qs = [cp.make_query("ppr", 0.2, s, kmode="fixed", K=8, flags=cp.CP_Q_TIMING) for s in range(bw)]
            G.set_batch_width(bw, "f32", bw)
            Y = torch.empty((n, bw), dtype=torch.float32, device="cuda")
            G.power_batch(qs, prec="f32", Y=Y, stream=stream)
            ms, launches = 0.0, 0
            for _ in range(3):
                _, infos = G.power_batch(qs, prec="f32", Y=Y, stream=stream)
                ms += infos[0]["step_ms"]
                launches += infos[0]["steps"]
            per = ms / launches
            row = {"width": bw, "slice_rows": F, "slice_MiB": round(F * bw * 4 / 2**20, 2),
                   "launch_ms": round(per, 4), "G_gathers_per_s": round(n * d / (per * 1e-3) / 1e9, 1),
                   "G_lines_per_s": round(n * d * max(1, bw * 4 // 128) / (per * 1e-3) / 1e9, 1)}
            log(f"[footprint] {row}")
            rows.append(row)
            G.close()
            del Y
            torch.cuda.empty_cache()
    return {"workload": f"batched step kernel, FP32, {n} rows x {d} arcs, columns uniform over the first "
                        f"slice_rows rows (one gather = width x 4 bytes), K = 8", "rows": rows}


def run_legs(args, torch, cp, synth, result) -> None:
    """The workloads beside the headline, each into its key of result."""
    g_main = None
    if args.workload != "none":
        result["single"], g_main = run_single(args, torch, cp, synth)
    if not args.no_latency:
        result["latency"] = run_latency(args, torch, cp, synth)
    if g_main is not None:
        if args.kvn_tol > 0:
            result["cheby_vs_power"] = run_kvn(args, torch, cp, synth, g_main)
        if args.propagate_cols > 0:
            result["propagate"] = run_propagate(args, torch, cp, synth, g_main)
        if args.push_eps:
            result["push"] = run_push(args, torch, cp, synth, g_main)
        if not args.no_push_rw:
            result["push_rw"] = run_push_rw(args, torch, cp, synth, g_main)
        if args.serve_seconds > 0:
            result["served"] = run_serve(args, torch, cp, synth, g_main)
    del g_main
    if args.batch_workload != "none":
        result["batched"] = run_batch(args, torch, cp, synth)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed headline batches (the JSON's steps)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed headline batches before them")
    ap.add_argument("--headline", default="ppr-batch-friendster", choices=sorted(HEADLINES) + ["none"],
                    help="the headline workload (none: only the other legs, e.g. for profiler runs)")
    ap.add_argument("--bf16-steps", type=int, default=3,
                    help="timed batches of each of the headline's variants (BF16 storage, FP32 arithmetic)")
    ap.add_argument("--batch-hot-split", action="store_true",
                    help="run the batched workload on the hot/cold split too (hot nodes: CHEBYPROP_HOT_NODES)")
    ap.add_argument("--no-hot-split", action="store_true",
                    help="run the headline's batched steps without the hot/cold split (CP_GRAPH_HOT_SPLIT)")
    ap.add_argument("--workload", default="hkpr-livejournal", choices=sorted(WORKLOADS) + ["none"],
                    help="single-source measurement reported beside the headline")
    ap.add_argument("--single-steps", type=int, default=10,
                    help="timed passes over the single-source workload's queries")
    ap.add_argument("--batch-workload", default="ppr-batch-orkut", choices=sorted(BATCH_WORKLOADS) + ["none"],
                    help="batched measurement reported beside the headline")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="counted length of the Poisson trace at --serve-rate (0: skip the served measurement)")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="warm-up seconds at the start of each trace")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="offered queries per second")
    ap.add_argument("--plain-limit-s", type=float, default=12.0,
                    help="wall time after which the plain leg of the --serve-rate trace stops")
    ap.add_argument("--serve-rate-low", type=float, default=50.0,
                    help="second offered rate, one the plain path sustains (0: skip)")
    ap.add_argument("--serve-seconds-low", type=float, default=20.0, help="counted length of that trace")
    ap.add_argument("--serve-check", type=int, default=16, help="served queries checked against the oracle")
    ap.add_argument("--saturation-rate", type=float, default=2000.0,
                    help="offered rate of a 1-second burst that measures the server's capacity (0: skip)")
    ap.add_argument("--layout", default="stripes", choices=["stripes", "degree", "native"],
                    help="graph layout inside the library for single-source queries: XCD column stripes "
                         "(CP_GRAPH_XCD_STRIPES), degree order (CP_GRAPH_REORDER) or the caller's ids; "
                         "results are always in caller ids")
    ap.add_argument("--kvn-tol", type=float, default=1e-6,
                    help="l1 tolerance of the ChebyPower-vs-PwMethod comparison (0: skip it)")
    ap.add_argument("--propagate-cols", type=int, default=64,
                    help="columns of the feature-matrix propagation measurement (0: skip it)")
    ap.add_argument("--push-eps", type=float, nargs="*", default=[1e-5, 1e-6, 1e-7, 1e-8],
                    help="eps_a values of the ChebyPush measurement (none: skip it)")
    ap.add_argument("--no-push-rw", action="store_true", help="skip the ChebyPush + random walk measurement")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-storage variants")
    ap.add_argument("--no-f32f", action="store_true",
                    help="skip the FP32-arithmetic variants (CP_F32F) of the headline and single-source legs")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the small-graph latency measurement (eager vs HIP graph replay)")
    ap.add_argument("--gather-footprint", action="store_true",
                    help="only measure the batched kernel's gather rate against the gathered slice's size")
    ap.add_argument("--footprint-rows", type=int, default=16_777_216, help="rows of that measurement's graph")
    ap.add_argument("--graph-cache", default="",
                    help="directory where generated graphs are kept as .npy files and read back by later runs")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(queries would shard by source across GPUs, with the graph replicated on each)",
              file=sys.stderr)
        return 2

    global np
    import numpy as np
    import torch

    import synth
    from paper_2412_10789_amd import chebyprop as cp

    cp.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    global GRAPH_CACHE
    GRAPH_CACHE = args.graph_cache or None
    if args.gather_footprint:
        print(json.dumps({"metric": "gather rate against gathered slice size", "n_gpus": 1,
                          "gather_footprint": run_gather_footprint(args, torch, cp)}), flush=True)
        return 0
    copy_gbps = copy_ceiling(torch)
    log(f"device copy ceiling: {copy_gbps:.0f} GB/s")

    if args.headline == "none":
        result = {"metric": METRIC, "n_gpus": 1, "note": "headline skipped (--headline none)"}
        run_legs(args, torch, cp, synth, result)
        print(json.dumps(result), flush=True)
        return 0
    H = run_headline(args, torch, cp, synth)
    result = {
        "metric": METRIC,
        "value": round(H["value"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(H["total_s"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ARITH_DTYPE[H["prec"]],  # arithmetic; vectors are stored as config.prec
        "storage_dtype": H["prec"],
        "data": "synthetic (seeded Chung-Lu graphs shaped like Friendster / LiveJournal / Orkut; random sources)",
        "config": {
            "workload": H["workload"], "n": H["n"], "nnz": H["nnz"], "d_max": H["d_max"], "sources": H["sources"],
            "K_per_source": H["Ks"], "prec": H["prec"], "layout": "degree", "source_tile_width": H["source_tile_width"],
            "hot_nodes": H["hot_nodes"], "hot_arc_share": H["hot_arc_share"],
            "graph_generate_s": H["generate_s"], "graph_create_s": H["create_s"], "parallelism": "single-gpu",
        },
        "roofline": H["roofline"],
        "launch_bytes_rule": H["launch_bytes_rule"],
        "copy_ceiling_gbps": round(copy_gbps, 1),
    }
    for k in ("cpu_baseline", "accuracy_vs_fp64_oracle", "storage_bf16", "arith_f32"):
        if k in H:
            result[k] = H[k]
    del H
    run_legs(args, torch, cp, synth, result)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
