#!/usr/bin/env python3
"""ChebyPower benchmark on one MI355X.

Main line (the JSON's "value"): heat-kernel PageRank (t = 5) on a seeded
Chung-Lu graph shaped like LiveJournal (n = 4,000,000 target nodes,
35,000,000 undirected edges, degree exponent 2.3, int64 offsets / int32
columns), 16 random sources run one at a time, FP32 vectors, l1 tolerance
1e-6 with the certified truncation step.  One "step" of this benchmark is
one pass of the whole path (coefficients, K, init, K-1 Chebyshev steps,
finalize) for all 16 sources.

Beside it ("batched"): 64 PPR (alpha = 0.2) sources with per-source
tolerances drawn from {1e-4, 1e-6, 1e-7} in one batch on a Chung-Lu graph
shaped like Orkut (n = 3,000,000, 117,000,000 edges, exponent 2.2), FP32,
autotuned source-tile width.

Prints one JSON line: GTEPS (CSR arcs traversed per second, summed over
sources), the roofline of the dominant kernel (the Chebyshev step) against
MI355X's 8 TB/s HBM, accuracy against the FP64 oracle, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
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

WORKLOADS = {
    # name: (n, m, gamma, seed, kind, param, tol, sources, prec)
    "hkpr-livejournal": (4_000_000, 35_000_000, 2.3, 2, "hkpr", 5.0, 1e-6, 16, "f32"),
    "hkpr-small": (200_000, 1_750_000, 2.3, 2, "hkpr", 5.0, 1e-6, 16, "f32"),
}

BATCH_WORKLOADS = {
    # name: (n, m, gamma, seed, alpha, sources, tolerance choices, prec)
    "ppr-batch-orkut": (3_000_000, 117_000_000, 2.2, 3, 0.2, 64, (1e-4, 1e-6, 1e-7), "f32"),
    "ppr-batch-small": (200_000, 4_000_000, 2.2, 3, 0.2, 64, (1e-4, 1e-6, 1e-7), "f32"),
}

STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16": 2}
ACC_BYTES = {"f64": 8, "f32": 8, "bf16": 4}  # estimate precision (FP32 storage keeps a double estimate)
ARITH_DTYPE = {"f64": "f64", "f32": "f64", "bf16": "f32"}  # what the kernels add and multiply in


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(files=("kernels.hip", "kernels_batch.hip", "common.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2412_10789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_bytes(n: int, nnz: int, prec: str, sources: int = 1) -> int:
    """Algorithmic bytes of one Chebyshev step launch: column ids and row
    offsets once, and per node and source one compulsory gather of x,
    read + write of z, read + write of the estimate."""
    s, a = STORAGE_BYTES[prec], ACC_BYTES[prec]
    return 4 * nnz + 8 * (n + 1) + n * sources * (3 * s + 2 * a)


def clenshaw_step_bytes(n: int, nnz: int, prec: str, sources: int) -> int:
    """Algorithmic bytes of one step of Clenshaw's backward form: column ids
    and row offsets once, and per node and column one gather of b_{k+1},
    read of b_{k+2}, write of b_k and read of the start vector (kept at the
    estimate's precision); no estimate stream."""
    s, a = STORAGE_BYTES[prec], ACC_BYTES[prec]
    return 4 * nnz + 8 * (n + 1) + n * sources * (3 * s + a)


def measured_traffic(key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken with the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "step_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    e = rec.get(key)
    if not e or e.get("kernel_hash") != kernel_hash():
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


def run_single(args, torch, cp, synth):
    n_t, m_t, gamma, seed, kind, param, tol, nsrc, prec = WORKLOADS[args.workload]
    t0 = time.time()
    g = synth.chung_lu(n_t, m_t, gamma, seed=seed)
    log(f"[single] graph: n={g.n} nnz={g.nnz} d_max={g.meta['d_max']} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout == "degree", stripes=args.layout == "stripes")
    create_s = time.time() - t0
    log(f"[single] graph create (layout={args.layout}): {create_s:.2f}s, stats={G.stats}")
    srcs = [int(s) for s in synth.sources(g, nsrc, seed=seed)]
    Y = torch.empty((nsrc, g.n), dtype=G.out_dtype(cp.PRECS[prec]), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

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
        for _ in range(args.steps):
            infos += one_step(True, p, Yp)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        total_s = max(wall, ev0.elapsed_time(ev1) * 1e-3)
        arcs = sum((inf["K"] - 1) * g.nnz + int(g.degrees[s]) for inf, s in zip(infos, srcs * args.steps))
        timed = [inf for inf in infos if inf["step_ms"] == inf["step_ms"]]  # not NaN: the timed queries
        launches = sum(inf["steps"] for inf in timed)
        avg_step_ms = sum(inf["step_ms"] for inf in timed) / max(launches, 1)
        bpl = step_bytes(g.n, g.nnz, p)
        Ks = [inf["K"] for inf in infos[:nsrc]]
        log(f"[single] {p}: K per source: {Ks}; avg step kernel {avg_step_ms * 1e3:.1f} us; "
            f"wall {wall * 1e3:.1f} ms")
        return dict(value=arcs / total_s / 1e9, total_s=total_s, launches=launches, bpl=bpl,
                    achieved=bpl / (avg_step_ms * 1e-3) / 1e9, avg_step_ms=avg_step_ms, Ks=Ks)

    out = timed_run(prec, Y, args.warmup)
    out.update(
        g=g, srcs=srcs, Y=Y, layout=args.layout, create_s=create_s, kind=kind, param=param, tol=tol, nsrc=nsrc,
        prec=prec,
        workload=f"{args.workload}: HKPR t={param}, {nsrc} sources one at a time, tol {tol} l1 (certified K), "
                 f"Chung-Lu n={n_t} m={m_t} gamma={gamma} seed={seed}",
    )
    if not args.no_bf16:
        # the same queries with BF16 vector storage (float arithmetic and estimate)
        Yb = torch.empty((nsrc, g.n), dtype=torch.float32, device="cuda")
        out["bf16"] = timed_run("bf16", Yb, 1)
        out["bf16"]["Y"] = Yb
    G.close()
    return out


def run_batch(args, torch, cp, synth):
    n_t, m_t, gamma, seed, alpha, nq, tol_choices, prec = BATCH_WORKLOADS[args.batch_workload]
    t0 = time.time()
    g = synth.chung_lu(n_t, m_t, gamma, seed=seed)
    log(f"[batch] graph: n={g.n} nnz={g.nnz} d_max={g.meta['d_max']} ({time.time() - t0:.1f}s)")
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout != "native")
    srcs = [int(s) for s in synth.sources(g, nq, seed=seed)]
    tols = [float(t) for t in synth.tolerance_choice(seed, nq, tol_choices)]
    qs = [cp.make_query("ppr", alpha, s, t) for s, t in zip(srcs, tols)]
    bw = G.autotune_batch(qs, prec=prec)
    log(f"[batch] autotuned source-tile width {bw}")
    qt = [cp.make_query("ppr", alpha, s, t, flags=cp.CP_Q_TIMING) for s, t in zip(srcs, tols)]
    nb = max(1, args.steps // 2)

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
        arcs = nb * sum((k - 1) * g.nnz for k in Ks)
        # algorithmic bytes of each launch: sources still active in it
        per_batch_bytes = 0
        for k in range(1, max(Ks)):
            active = sum(1 for K in Ks if K > k)
            per_batch_bytes += step_bytes(g.n, g.nnz, p, active)
        avg_launch_ms = step_ms / max(launches, 1)
        achieved = per_batch_bytes * nb / (step_ms * 1e-3) / 1e9
        return total_s, Ks, arcs, avg_launch_ms, achieved

    Yb = torch.empty((g.n, nq), dtype=G.out_dtype(cp.PRECS[prec]), device="cuda")
    total_s, Ks, arcs, avg_launch_ms, achieved = timed_batches(prec, Yb)
    out = {
        "workload": f"{args.batch_workload}: {nq} PPR alpha={alpha} sources in one batch, tol per source from "
                    f"{list(tol_choices)} (certified K), Chung-Lu n={n_t} m={m_t} gamma={gamma} seed={seed}",
        "value": round(arcs / total_s / 1e9, 3),
        "unit": "GTEPS",
        "ms_per_batch": round(total_s * 1e3 / nb, 3),
        "n": g.n, "nnz": g.nnz, "source_tile_width": bw, "K_min": min(Ks), "K_max": max(Ks),
        "roofline": {
            "bound": "hbm", "kernel": "batch_step_kernel",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(f"{args.batch_workload}:batch"),
            "avg_launch_ms": round(avg_launch_ms, 4),
        },
    }
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import errors as E
        from oracle import propagation as PR

        j = min(range(nq), key=lambda i: tols[i])  # the tightest tolerance
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        ref = PR.cheby_power(P, srcs[j], C.ppr_chebyshev_coeffs(alpha, Ks[j]), Ks[j])
        col = Yb[:, j].double().cpu().numpy()
        out["accuracy_vs_fp64_oracle"] = {"column": j, "tol": tols[j], "K": Ks[j],
                                          "l1": E.l1(col, ref), "max_abs": E.max_abs(col, ref)}
    if not args.no_bf16:
        # the same batch with BF16 storage (float arithmetic and estimate), its own autotuned width
        del Yb
        bwb = G.autotune_batch(qs, prec="bf16")
        Ybb = torch.empty((g.n, nq), dtype=torch.float32, device="cuda")
        total_b, Ks_b, arcs_b, launch_b, achieved_b = timed_batches("bf16", Ybb)
        ent = {"workload": "the same batch with BF16 vector storage (float arithmetic and estimate)",
               "value": round(arcs_b / total_b / 1e9, 3), "unit": "GTEPS", "ms_per_batch": round(total_b * 1e3 / nb, 3),
               "source_tile_width": bwb,
               "roofline": {"bound": "hbm", "kernel": "batch_step_kernel", "achieved": round(achieved_b, 1),
                            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved_b / HBM_PEAK_GBPS, 4),
                            "avg_launch_ms": round(launch_b, 4)}}
        if Ks_b != Ks:
            raise RuntimeError("BF16 batch took other K than the FP32 one")
        if not args.no_cpu:
            col = Ybb[:, j].double().cpu().numpy()
            ent["accuracy_vs_fp64_oracle"] = {"column": j, "l1": E.l1(col, ref), "max_abs": E.max_abs(col, ref)}
        log(f"[batch] bf16 storage: {ent}")
        out["storage_bf16"] = ent
    G.close()
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


def run_serve(args, torch, cp, synth, g):
    """Served query stream: the batched server vs plain one-at-a-time
    queries on the same arrival trace (same graph, same FP32 precision)."""
    trace = serve_trace(g, synth, args.serve_seconds, args.serve_rate)
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=args.layout != "native", stripes=args.layout == "stripes")
    nbuf = 512  # one result buffer per server slot
    bufs = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in range(nbuf)]
    # warm both paths (code objects, caches)
    for (_, kind, param, s, tol) in trace[:4]:
        G.power(kind, param, s, tol=tol, prec="f32", y=bufs[0])
    torch.cuda.synchronize()

    # ---- batched server
    S = cp.Server(G, hbm_budget_bytes=16 << 30, max_slots=512, max_queue=100000, prec="f32")
    for (_, kind, param, s, tol) in trace[:8]:
        S.wait(S.submit(cp.make_query(kind, param, s, tol), bufs[1]))

    def replay(tr):
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

    ticks0 = S.stats()["ticks"]
    tickets, t_end = replay(trace)
    lat = [info["latency_ms"] for st, info in tickets if st == cp.CP_OK]
    Ks = [info["K"] for st, info in tickets if st == cp.CP_OK]
    sstats = S.stats()
    sat = None
    if args.saturation_rate > 0:
        burst = serve_trace(g, synth, 1.0, args.saturation_rate, seed=7)
        bt, b_end = replay(burst)
        blat = [info["latency_ms"] for st, info in bt if st == cp.CP_OK]
        sat = {"offered_qps": args.saturation_rate, "queries": len(burst), "completed": len(blat),
               "qps": round(len(blat) / b_end, 1), "p50_ms": _pct(blat, 50), "p99_ms": _pct(blat, 99),
               "span_s": round(b_end, 3), "latency_from": "submission (a submit waits for a free result buffer)"}
        log(f"[serve] saturation burst: {sat}")
    # accuracy of two served results (rerun into a fresh buffer through the server)
    acc = None
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import errors as E
        from oracle import propagation as PR

        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        acc = []
        for i in (0, len(trace) // 2):
            _, kind, param, s, tol = trace[i]
            st, info = S.wait(S.submit(cp.make_query(kind, param, s, tol), bufs[2]))
            ref = PR.cheby_power(P, s, C.chebyshev_coeffs(kind, param, info["K"]), info["K"])
            y = bufs[2].double().cpu().numpy()
            acc.append({"kind": kind, "param": param, "tol": tol, "K": info["K"],
                        "l1": E.l1(y, ref), "max_abs": E.max_abs(y, ref)})
    S.close()
    server = {"completed": len(lat), "qps": round(len(lat) / t_end, 1), "p50_ms": _pct(lat, 50),
              "p99_ms": _pct(lat, 99), "mean_ms": float(np.mean(lat)) if lat else None,
              "span_s": round(t_end, 3), "slots": sstats["slots"], "tile_width": sstats["tile_width"],
              "batched_launches": sstats["ticks"] - ticks0, "mean_K": float(np.mean(Ks)) if Ks else None}
    log(f"[serve] server: {server}")

    # ---- plain: one query at a time, FIFO, single-source path
    lat_p = []
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    for (ta, kind, param, s, tol) in trace:
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        G.power(kind, param, s, tol=tol, prec="f32", y=bufs[0], stream=stream)
        torch.cuda.synchronize()
        lat_p.append((time.perf_counter() - t0 - ta) * 1e3)
        if len(lat_p) % 4000 == 0:
            log(f"[serve] plain: {len(lat_p)} of {len(trace)} queries done")
    t_end_p = time.perf_counter() - t0
    plain = {"completed": len(lat_p), "qps": round(len(lat_p) / t_end_p, 1), "p50_ms": _pct(lat_p, 50),
             "p99_ms": _pct(lat_p, 99), "mean_ms": float(np.mean(lat_p)), "span_s": round(t_end_p, 3)}
    log(f"[serve] plain: {plain}")
    G.close()
    out = {
        "workload": f"Poisson arrivals at {args.serve_rate}/s for {args.serve_seconds} s ({len(trace)} queries): "
                    f"PPR alpha in {{0.1, 0.2}}, HKPR t in {{3, 5, 10}} uniformly, tol log-uniform [1e-7, 1e-4] "
                    f"(certified K), FP32 resident state, on the main line's graph",
        "offered_qps": args.serve_rate,
        "server": server,
        "plain": plain,
        "speedup_qps": round(server["qps"] / plain["qps"], 2) if plain["qps"] else None,
    }
    if sat is not None:
        out["server_saturation"] = sat
        out["capacity_vs_plain"] = round(sat["qps"] / plain["qps"], 2) if plain["qps"] else None
    if acc is not None:
        out["accuracy_vs_fp64_oracle"] = acc
    return out


LARGE = (65_000_000, 1_800_000_000, 2.1, 5, 0.2, 8, 1e-6)


def run_large(args, torch, cp, synth):
    """Friendster-sized graph (n = 65M target nodes, 1.8B undirected edges,
    exponent 2.1): a batch of 8 PPR sources with FP32 and with BF16 storage,
    one single-source query, and the l1 / max error of each against the
    plain-C FP64 oracle on one source (full vector)."""
    n_t, m_t, gamma, seed, alpha, nq, tol = LARGE
    t0 = time.time()
    g = synth.chung_lu(n_t, m_t, gamma, seed=seed, tune_passes=0, verbose=True)
    gen_s = time.time() - t0
    log(f"[large] graph: n={g.n} nnz={g.nnz} d_max={g.meta['d_max']} ({gen_s:.0f}s)")
    t0 = time.time()
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=True)
    create_s = time.time() - t0
    log(f"[large] graph create {create_s:.0f}s, device bytes {G.stats['device_bytes']}")
    srcs = [int(s) for s in synth.sources(g, nq, seed=seed)]
    qs = [cp.make_query("ppr", alpha, s, tol, flags=cp.CP_Q_TIMING) for s in srcs]
    out = {"workload": f"large: {nq} PPR alpha={alpha} sources, tol {tol} l1 (certified K), Chung-Lu n={n_t} "
                       f"m={m_t} gamma={gamma} seed={seed} (one generation pass)",
           "n": g.n, "nnz": g.nnz, "d_max": int(g.degrees.max()), "generate_s": round(gen_s, 1),
           "graph_create_s": round(create_s, 1)}
    cols = {}
    for prec in ("f32", "bf16"):
        G.set_batch_width(nq, prec, 8)
        Yb, infos = G.power_batch(qs, prec=prec)  # warm-up
        Yb, infos = G.power_batch(qs, prec=prec, Y=Yb)
        Ks = [i["K"] for i in infos]
        ms = infos[0]["elapsed_ms"]
        arcs = sum((k - 1) * g.nnz for k in Ks)
        out[f"batch_{prec}"] = {"GTEPS": round(arcs / ms / 1e6, 2), "ms_per_batch": round(ms, 1),
                                "avg_launch_ms": round(infos[0]["step_ms"] / max(i["steps"] for i in infos), 3),
                                "K": Ks, "source_tile_width": 8}
        cols[prec] = Yb[:, 0].double().cpu().numpy()
        log(f"[large] batch {prec}: {out[f'batch_{prec}']}")
        del Yb
    r = G.power("ppr", alpha, srcs[0], tol=tol, prec="f32", flags=cp.CP_Q_TIMING)
    out["single_f32"] = {"GTEPS": round((r.info["K"] - 1) * g.nnz / r.info["elapsed_ms"] / 1e6, 2),
                         "ms": round(r.info["elapsed_ms"], 1), "K": r.info["K"],
                         "avg_step_ms": round(r.info["step_ms"] / r.info["steps"], 3)}
    cols["single_f32"] = r.y.double().cpu().numpy()
    log(f"[large] single: {out['single_f32']}")
    G.close()
    # the main line's layout (XCD stripes; plain column ids at this n)
    t0 = time.time()
    Gs = cp.Graph(g.row_ptr, g.col_idx, stripes=True)
    log(f"[large] striped graph create {time.time() - t0:.0f}s, stats {Gs.stats}")
    Gs.power("ppr", alpha, srcs[0], tol=tol, prec="f32")  # warm-up
    r = Gs.power("ppr", alpha, srcs[0], tol=tol, prec="f32", flags=cp.CP_Q_TIMING)
    out["single_f32_stripes"] = {"GTEPS": round((r.info["K"] - 1) * g.nnz / r.info["elapsed_ms"] / 1e6, 2),
                                 "ms": round(r.info["elapsed_ms"], 1), "K": r.info["K"],
                                 "avg_step_ms": round(r.info["step_ms"] / r.info["steps"], 3),
                                 "stripe_packed": Gs.stats["stripe_packed"]}
    cols["single_f32_stripes"] = r.y.double().cpu().numpy()
    log(f"[large] single (stripes): {out['single_f32_stripes']}")
    Gs.close()
    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import errors as E
        from oracle import native as NO

        NO.set_verbose(True)
        K = out["batch_f32"]["K"][0]
        t0 = time.perf_counter()
        ref = NO.cheby_power(g.row_ptr, g.col_idx, srcs[0], C.ppr_chebyshev_coeffs(alpha, K), K)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round((K - 1) * g.nnz / cpu_s / 1e9, 4), "unit": "GTEPS",
                               "cores": NO.threads(), "kind": "oracle",
                               "sample": f"1 of the {nq} sources, same K={K}: plain-C FP64 Alg. 3 with an OpenMP "
                                         f"node loop, {cpu_s:.0f} s"}
        out["accuracy_vs_fp64_oracle"] = {k: {"l1": E.l1(v, ref), "max_abs": E.max_abs(v, ref)}
                                          for k, v in cols.items()}
        log(f"[large] accuracy {out['accuracy_vs_fp64_oracle']}")
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hkpr-livejournal", choices=sorted(WORKLOADS))
    ap.add_argument("--batch-workload", default="ppr-batch-orkut", choices=sorted(BATCH_WORKLOADS) + ["none"],
                    help="batched measurement reported beside the main line")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="length of the Poisson arrival trace for the served measurement (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="offered queries per second")
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
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the main line's BF16-storage variant")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the small-graph latency measurement (eager vs HIP graph replay)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (counter scaling for rocprofv3 --pmc)")
    ap.add_argument("--large", action="store_true",
                    help="run only the Friendster-sized measurement (n=65M, 1.8B edges; minutes, ~60 GB host RAM)")
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
    if args.large:
        res = {"metric": METRIC, "n_gpus": 1, "large": run_large(args, torch, cp, synth)}
        print(json.dumps(res), flush=True)
        return 0
    copy_gbps = copy_ceiling(torch)
    log(f"device copy ceiling: {copy_gbps:.0f} GB/s")

    S = run_single(args, torch, cp, synth)
    result = {
        "metric": METRIC,
        "value": round(S["value"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(S["total_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ARITH_DTYPE[S["prec"]],  # arithmetic; vectors are stored as config.prec
        "storage_dtype": S["prec"],
        "data": "synthetic (seeded Chung-Lu graphs shaped like LiveJournal / Orkut; random sources)",
        "config": {
            "workload": S["workload"],
            "n": S["g"].n, "nnz": S["g"].nnz, "d_max": int(S["g"].degrees.max()), "sources": S["nsrc"],
            "K_per_source": S["Ks"], "layout": S["layout"], "prec": S["prec"],
            "graph_create_s": round(S["create_s"], 3), "parallelism": "single-gpu",
        },
        "hbm_frac_whole_run": round(S["launches"] * S["bpl"] / S["total_s"] / 1e9 / HBM_PEAK_GBPS, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": "stripe_gather_kernel + stripe_combine_kernel" if S["layout"] == "stripes" else "step_kernel",
            "achieved": round(S["achieved"], 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(S["achieved"] / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(f"{args.workload}:{S['layout']}"),
            "bytes_per_launch": S["bpl"],
            "avg_launch_us": round(S["avg_step_ms"] * 1e3, 2),
            "launches_timed": S["launches"],
        },
        "copy_ceiling_gbps": round(copy_gbps, 1),
    }

    if not args.no_cpu:
        from oracle import coefficients as C
        from oracle import errors as E
        from oracle import propagation as PR

        # bounded sample: whole queries of the timed workload, in order, until
        # about 10 s of single-thread oracle time
        g = S["g"]
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        cpu_s, cpu_arcs, done, l1s, maxs, refs = 0.0, 0, 0, [], [], []
        for i, (s, K) in enumerate(zip(S["srcs"], S["Ks"])):
            c = C.chebyshev_coeffs(S["kind"], S["param"], K)
            c0 = time.perf_counter()
            y_ref = PR.cheby_power(P, s, c, K)
            cpu_s += time.perf_counter() - c0
            cpu_arcs += (K - 1) * g.nnz + int(g.degrees[s])
            y_gpu = S["Y"][i].double().cpu().numpy()
            l1s.append(E.l1(y_gpu, y_ref))
            maxs.append(E.max_abs(y_gpu, y_ref))
            refs.append((s, K, c, y_ref))
            done += 1
            if cpu_s >= 10.0:
                break
        result["cpu_baseline"] = {
            "value": round(cpu_arcs / cpu_s / 1e9, 4),
            "unit": "GTEPS",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the first {done} of the {S['nsrc']} sources (same graph, same K per source): FP64 Alg. 3 "
                      f"with scipy CSR products, {cpu_s:.1f} s",
        }
        result["accuracy_vs_fp64_oracle"] = {"sources": done, "max_l1": max(l1s), "max_abs": max(maxs),
                                             "K": [r[1] for r in refs]}
        # the same sample on every host thread: the plain-C oracle (OpenMP node loop)
        from oracle import native as NO

        c0 = time.perf_counter()
        agree = 0.0
        for (s, K, c, y_ref) in refs:
            y_c = NO.cheby_power(g.row_ptr, g.col_idx, s, c, K)
            agree = max(agree, E.l1(y_c, y_ref))
        cpu_t = time.perf_counter() - c0
        result["cpu_baseline_threads"] = {
            "value": round(cpu_arcs / cpu_t / 1e9, 4), "unit": "GTEPS", "cores": NO.threads(), "kind": "oracle",
            "sample": f"the same {done} sources and K: plain-C FP64 Alg. 3, {cpu_t:.2f} s",
            "agrees_with_scipy_oracle_l1": agree,
            "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()},
        }
    if "bf16" in S:
        B = S["bf16"]
        entry = {
            "workload": "the main line's queries (same graph, sources, steps and layout) with BF16 vector "
                        "storage: float arithmetic and a float estimate",
            "value": round(B["value"], 3), "unit": "GTEPS", "ms_per_step": round(B["total_s"] * 1e3 / args.steps, 4),
            "K_per_source": B["Ks"],
            "roofline": {"bound": "hbm", "achieved": round(B["achieved"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(B["achieved"] / HBM_PEAK_GBPS, 4), "bytes_per_launch": B["bpl"],
                         "avg_launch_us": round(B["avg_step_ms"] * 1e3, 2)},
        }
        if not args.no_cpu:
            l1b, maxb = [], []
            for i, (s, K, c, y_ref) in enumerate(refs):
                if B["Ks"][i] != K:
                    raise RuntimeError("BF16 query took another K than the FP32 one")
                y_b = B["Y"][i].double().cpu().numpy()
                l1b.append(E.l1(y_b, y_ref))
                maxb.append(E.max_abs(y_b, y_ref))
            entry["accuracy_vs_fp64_oracle"] = {"sources": len(refs), "max_l1": max(l1b), "max_abs": max(maxb)}
        log(f"[single] bf16 storage: {entry}")
        result["storage_bf16"] = entry
    g_main = S["g"]
    del S
    if not args.no_latency:
        result["latency"] = run_latency(args, torch, cp, synth)
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
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
