"""Query server (iteration-level batching) against single-query runs and the
oracle; admission, cancellation and error paths."""

import time

import numpy as np
import pytest

import synth
from gpu_util import F32_L1, compare, f32_bar, f32f_bar, gpu_graph, oracle_exact_multi, oracle_yK_multi, require_gpu  # noqa: F401
from oracle import errors as E

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def graph():
    return synth.chung_lu(120_000, 1_000_000, 2.3, seed=41)


def _mixed_queries(g, n, seed):
    from paper_2412_10789_amd import chebyprop as cp

    kinds = [("ppr", 0.1), ("ppr", 0.2), ("hkpr", 3.0), ("hkpr", 5.0), ("hkpr", 10.0)]
    srcs = synth.sources(g, n, seed=seed)
    tols = synth.tolerance_loguniform(seed, n, 1e-9, 1e-4)
    return [cp.make_query(*kinds[i % 5], int(srcs[i]), float(tols[i])) for i in range(n)]


@pytest.mark.parametrize("layout", ["degree", "stripes"])
def test_server_results_equal_single_queries_f64(torch, graph, layout):
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    G = gpu_graph(g, reorder=layout == "degree", stripes=layout == "stripes")
    per_tile = 3 * g.n * 16 * 8
    S = cp.Server(G, hbm_budget_bytes=2 * per_tile + 4096, prec="f64")
    assert S.stats()["slots"] == 32 and S.stats()["tile_width"] == 16
    qs = _mixed_queries(g, 70, seed=2)
    ys = [torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda") for _ in qs]
    print("CASE server-f64", layout, flush=True)
    tickets = [S.submit(q, y) for q, y in zip(qs, ys)]
    infos = []
    for t in tickets:
        st, info = S.wait(t, timeout_ms=60_000)
        assert st == cp.CP_OK, st
        infos.append(info)
    torch.cuda.synchronize()
    for q, y, info in zip(qs, ys, infos):
        kind = "hkpr" if q.kind == 1 else "ppr"
        r = G.power(kind, q.param, q.source, tol=q.tol, prec="f64")
        assert r.info["K"] == info["K"]
        np.testing.assert_allclose(y.cpu().numpy(), r.y.cpu().numpy(), atol=1e-14, rtol=1e-12)
        assert info["latency_ms"] >= info["wait_ms"] >= 0
    st = S.stats()
    assert st["completed"] == 70 and st["active"] == 0 and st["queued"] == 0
    S.close()


def _meta(q):
    return ("hkpr" if q.kind == 1 else "ppr", q.param, q.source)


def test_server_f32_against_oracle(torch, graph):
    """Every served FP32 result against Alg. 3 in FP64 at its K and against
    the converged vector (l1 within the query's tolerance plus FP32
    rounding)."""
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    G = gpu_graph(g)
    S = cp.Server(G, hbm_budget_bytes=1 << 30, max_slots=64, prec="f32")
    qs = _mixed_queries(g, 24, seed=3)
    ys = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in qs]
    print("CASE server-f32", flush=True)
    tickets = []
    for q, y in zip(qs, ys):  # staggered arrivals: queries join running batches
        tickets.append(S.submit(q, y))
        time.sleep(0.002)
    Ks = []
    for t in tickets:
        st, info = S.wait(t, timeout_ms=60_000)
        assert st == cp.CP_OK
        Ks.append(info["K"])
    S.close()
    metas = [_meta(q) for q in qs]
    ref = oracle_yK_multi(g, metas, Ks)
    exact = oracle_exact_multi(g, metas)
    for j, q in enumerate(qs):
        y = ys[j].double().cpu().numpy()
        m = compare(y, ref[:, j])
        assert m["l1"] <= f32_bar(Ks[j], *metas[j][:2]), (j, Ks[j], m)
        assert E.l1(y, exact[:, j]) <= q.tol + f32_bar(Ks[j], *metas[j][:2]), (j, q.tol)


def test_server_cancel_busy_and_budget(torch, graph):
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    G = gpu_graph(g)
    with pytest.raises(cp.ChebypropError) as ei:
        cp.Server(G, hbm_budget_bytes=1000, prec="f32")
    assert ei.value.status == cp.CP_ENOMEM
    S = cp.Server(G, hbm_budget_bytes=1 << 40, max_slots=16, max_queue=4, prec="f64")
    assert S.stats()["slots"] == 16
    s0 = int(synth.sources(g, 1, seed=9)[0])
    slow = cp.make_query("ppr", 0.001, s0, 1e-12)  # long-running (K in the hundreds)
    ys = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in range(21)]
    print("CASE server-cancel", flush=True)
    tickets = [S.submit(slow, ys[i]) for i in range(20)]
    with pytest.raises(cp.ChebypropError) as ei:
        S.submit(slow, ys[20])
    assert ei.value.status == cp.CP_EBUSY
    # cancel one queued (the last) and one running (the first) query
    assert S.cancel(tickets[-1]) == cp.CP_OK
    t0 = time.time()
    while S.stats()["active"] == 0 and time.time() - t0 < 10:
        time.sleep(0.0005)
    assert S.cancel(tickets[0]) == cp.CP_OK
    assert S.wait(tickets[-1])[0] == cp.CP_ECANCELLED
    assert S.wait(tickets[0])[0] == cp.CP_ECANCELLED
    assert S.cancel(tickets[0]) == cp.CP_ENOTFOUND
    for t in tickets[1:-1]:
        st, info = S.wait(t, timeout_ms=120_000)
        assert st == cp.CP_OK
    r = G.power("ppr", 0.001, s0, tol=1e-12, prec="f64")
    np.testing.assert_allclose(ys[1].cpu().numpy(), r.y.cpu().numpy(), atol=1e-14, rtol=1e-12)
    with pytest.raises(cp.ChebypropError) as ei:
        S.submit(cp.make_query("ppr", 0.2, g.n + 1, 1e-6), ys[20])
    assert ei.value.status == cp.CP_ESOURCE
    assert S.poll(123456789)[0] == cp.CP_ENOTFOUND
    S.close()


@pytest.mark.slow
def test_server_full_size_mixed_stream_f32(torch):
    """The served workload at full size, with the server configured as the
    benchmark runs it: Chung-Lu n=4M, ~35M edges, exponent 2.3, XCD-striped
    graph, FP32 state, 512 slots; mixed PPR (alpha 0.1, 0.2) and HKPR
    (t 3, 5, 10) queries with tolerances log-uniform in [1e-9, 1e-4] (a
    wider range than the served trace's [1e-7, 1e-4]), some submitted while
    others run.  Every result equals the single-source run of its query
    (same K) to FP32 rounding and matches the FP64 oracle's Alg. 3 at its
    K."""
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.chung_lu(4_000_000, 35_000_000, 2.3, seed=2)
    G = gpu_graph(g, stripes=True)
    S = cp.Server(G, hbm_budget_bytes=16 << 30, max_slots=512, max_queue=100000, prec="f32")
    qs = _mixed_queries(g, 24, seed=7)
    ys = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in qs]
    print("CASE server-full-size", flush=True)
    tickets = []
    for i, (q, y) in enumerate(zip(qs, ys)):
        tickets.append(S.submit(q, y))
        if i % 8 == 7:
            time.sleep(0.01)  # later queries join running batches
    infos = []
    for t in tickets:
        st, info = S.wait(t, timeout_ms=120_000)
        assert st == cp.CP_OK, st
        infos.append(info)
    S.close()
    torch.cuda.synchronize()
    ymat = [y.double().cpu().numpy() for y in ys]
    for q, y, info in zip(qs, ymat, infos):
        kind = "hkpr" if q.kind == 1 else "ppr"
        r = G.power(kind, q.param, q.source, tol=q.tol, prec="f32")
        assert r.info["K"] == info["K"]
        assert compare(y, r.y.double().cpu().numpy())["l1"] <= f32_bar(info["K"], kind, q.param)
    # every result against the FP64 oracle's Alg. 3 at its K; with the certified K
    # (tail_bound_l1 <= tol, pinned on the CPU) this bounds the distance to the
    # exact vector by tol + the rounding bar
    metas = [_meta(q) for q in qs]
    ref = oracle_yK_multi(g, metas, [i["K"] for i in infos])
    worst = 0.0
    for j, q in enumerate(qs):
        m = compare(ymat[j], ref[:, j])
        worst = max(worst, m["l1"])
        assert m["l1"] <= f32_bar(infos[j]["K"], *metas[j][:2]), (j, infos[j]["K"], m)
        assert infos[j]["tail_bound_l1"] <= q.tol
    print("server full size: worst FP32 l1 against Alg. 3 at the same K", worst, flush=True)


def test_server_destroy_releases_blocked_waiters(torch, graph):
    """cp_server_destroy cancels what is left and lets threads blocked in
    cp_server_wait return before it frees the server."""
    import threading

    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    G = gpu_graph(g)
    S = cp.Server(G, hbm_budget_bytes=1 << 40, max_slots=16, max_queue=64, prec="f64")
    s0 = int(synth.sources(g, 1, seed=9)[0])
    slow = cp.make_query("ppr", 0.001, s0, 1e-12)  # long-running (K in the hundreds)
    ys = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in range(24)]
    tickets = [S.submit(slow, y) for y in ys]
    results = {}

    def waiter(i):
        results[i] = S.wait(tickets[i])[0]

    print("CASE server-destroy-with-waiters", flush=True)
    threads = [threading.Thread(target=waiter, args=(i,)) for i in (0, 23)]  # running, queued
    for t in threads:
        t.start()
    t0 = time.time()
    while S.stats()["waiters"] < 2 and time.time() - t0 < 30:
        time.sleep(0.001)
    assert S.stats()["waiters"] == 2
    S.close()
    for t in threads:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in threads)
    assert results[23] == cp.CP_ECANCELLED
    assert results[0] in (cp.CP_OK, cp.CP_ECANCELLED)


def test_idle_server_runs_single_source_path(torch, graph):
    """A query that reaches an idle server runs on the single-source path:
    its result is bitwise the cp_power result; a burst that arrives while it
    runs is batched (stats: direct count, batched launches); the queue limit
    of the single-source path starts at 3 and stays within [1, 16] once
    both paths have been timed."""
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    G = gpu_graph(g, stripes=True)
    S = cp.Server(G, hbm_budget_bytes=1 << 30, max_slots=64, prec="f32")
    qs = _mixed_queries(g, 30, seed=11)
    y = torch.empty(g.n, dtype=torch.float32, device="cuda")
    print("CASE server direct path", flush=True)
    st, info = S.wait(S.submit(qs[0], y), timeout_ms=60_000)
    assert st == cp.CP_OK and S.stats()["direct"] == 1 and S.stats()["ticks"] == 0
    assert S.stats()["direct_limit"] == 3  # no batched step timed yet
    q = qs[0]
    r = G.power("hkpr" if q.kind == 1 else "ppr", q.param, q.source, tol=q.tol, prec="f32")
    assert torch.equal(y, r.y) and info["K"] == r.info["K"]
    ys = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in qs[1:]]
    tickets = [S.submit(q, yy) for q, yy in zip(qs[1:], ys)]
    for t in tickets:
        assert S.wait(t, timeout_ms=60_000)[0] == cp.CP_OK
    stats = S.stats()
    assert stats["completed"] == 30 and stats["ticks"] > 0 and stats["direct"] < 30
    assert 1 <= stats["direct_limit"] <= 16
    S.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f32f"])
def test_narrow_launches_of_the_first_slots(torch, graph, prec):
    """A few queries arriving together take the first slots, so the batched
    launches update only those (narrow launches of 8 or 16 lanes over the
    first tile); their results equal single-source runs (FP64) or the FP64
    oracle at the same K (float storage), and a larger burst runs whole-tile
    launches too."""
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    G = gpu_graph(g, stripes=True)
    S = cp.Server(G, hbm_budget_bytes=1 << 30, max_slots=64, prec=prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    bw = S.stats()["tile_width"]
    for nq in (6, 12, 40):
        qs = _mixed_queries(g, nq, seed=50 + nq)
        ys = [torch.empty(g.n, dtype=dt, device="cuda") for _ in qs]
        before = S.stats()
        print("CASE server narrow", prec, nq, flush=True)
        got = [S.wait(t, timeout_ms=60_000) for t in [S.submit(q, y) for q, y in zip(qs, ys)]]
        assert all(st == cp.CP_OK for st, _ in got)
        st = S.stats()
        narrow, ticks = st["narrow_ticks"] - before["narrow_ticks"], st["ticks"] - before["ticks"]
        if nq == 6 or (nq == 12 and bw > 16):
            assert narrow > 0 and narrow == ticks, (nq, narrow, ticks)
        else:
            assert ticks > narrow, (nq, narrow, ticks)
        metas = [("hkpr" if q.kind == 1 else "ppr", q.param, q.source) for q in qs]
        Ks = [info["K"] for _, info in got]
        if prec == "f64":
            for q, y, (_, info) in zip(qs, ys, got):
                r = G.power("hkpr" if q.kind == 1 else "ppr", q.param, q.source, tol=q.tol, prec="f64")
                assert r.info["K"] == info["K"]
                np.testing.assert_allclose(y.cpu().numpy(), r.y.cpu().numpy(), atol=1e-14, rtol=1e-12)
        else:
            ref = oracle_yK_multi(g, metas, Ks)
            bar = f32f_bar if prec == "f32f" else (lambda K, kind, param: f32_bar(K, kind, param))
            for j, y in enumerate(ys):
                m = compare(y.double().cpu().numpy(), ref[:, j])
                b = bar(Ks[j]) if prec == "f32f" else bar(Ks[j], metas[j][0], metas[j][1])
                assert m["l1"] <= b, (prec, nq, j, Ks[j], m)
    S.close()
