"""Batched ChebyPower (cp_power_batch) against the FP64 oracle and against
single-source runs: every column must be the single-source result of its
own query (same K), whatever the source-tile width."""

import numpy as np
import pytest

import synth
from gpu_util import BF16_L1, compare, f32_bar, gpu_graph, oracle_exact_multi, oracle_yK, oracle_yK_multi, require_gpu
from oracle import errors as E
from oracle import propagation as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _queries(g, nq, seed, tol_choices=(1e-4, 1e-6, 1e-8)):
    from paper_2412_10789_amd import chebyprop as cp

    srcs = synth.sources(g, nq, seed=seed)
    tols = synth.tolerance_choice(seed, nq, tol_choices)
    kinds = [("ppr", 0.2), ("ppr", 0.1), ("hkpr", 5.0), ("hkpr", 3.0)]
    qs, meta = [], []
    for i in range(nq):
        kind, param = kinds[i % len(kinds)]
        qs.append(cp.make_query(kind, param, int(srcs[i]), float(tols[i])))
        meta.append((kind, param, int(srcs[i])))
    return qs, meta


@pytest.fixture(scope="module")
def mid_graph():
    return synth.chung_lu(150_000, 1_500_000, 2.2, seed=31)


@pytest.fixture(scope="module")
def mid_oracle(mid_graph):
    """The oracle's vectors for the mixed queries of each width's seed."""
    return {}


@pytest.mark.parametrize("bw", [8, 16, 32, 64])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_batch_columns_match_oracle(torch, mid_graph, mid_oracle, bw, prec):
    """Every column of a 37-query batch (ragged last tile for every width)
    against Alg. 3 in FP64 at its K and against the converged vector."""
    g = mid_graph
    G = gpu_graph(g, reorder=(bw in (16, 64)))
    nq = 37
    qs, meta = _queries(g, nq, seed=bw)
    G.set_batch_width(nq, prec, bw)
    print("CASE batch", prec, bw, flush=True)
    Y, infos = G.power_batch(qs, prec=prec)
    Y = Y.double().cpu().numpy()
    Ks = [i["K"] for i in infos]
    assert len(set(Ks)) > 1, "queries must differ in K"
    key = (bw, tuple(Ks))
    if key not in mid_oracle:
        mid_oracle[key] = (oracle_yK_multi(g, meta, Ks), oracle_exact_multi(g, meta))
    ref, exact = mid_oracle[key]
    for j in range(nq):
        m = compare(Y[:, j], ref[:, j])
        ex = E.l1(Y[:, j], exact[:, j])
        if prec == "f64":
            assert m["max_abs"] <= 1e-13, (j, m)
            assert ex <= qs[j].tol, (j, ex, qs[j].tol)
        elif prec == "f32":
            assert m["l1"] <= f32_bar(Ks[j], *meta[j][:2]), (j, Ks[j], m)
            assert ex <= qs[j].tol + f32_bar(Ks[j], *meta[j][:2]), (j, ex, qs[j].tol)
        else:  # BF16 storage: reported, about 1e-3
            assert m["l1"] <= BF16_L1, (j, m)


@pytest.mark.parametrize("stripes", [False, True])
def test_batch_equals_single_source_f64(torch, mid_graph, stripes):
    """Batch columns equal single-source runs on the same graph; on the
    XCD-striped layout the single runs take the striped step kernels and the
    batch the row-tiled ones over the same relabelled CSR."""
    g = mid_graph
    G = gpu_graph(g, stripes=stripes)
    qs, meta = _queries(g, 12, seed=5)
    print("CASE batch-vs-single", stripes, flush=True)
    Y, infos = G.power_batch(qs, prec="f64")
    for j, (kind, param, s) in enumerate(meta):
        r = G.power(kind, param, s, tol=qs[j].tol, prec="f64")
        assert r.info["K"] == infos[j]["K"]
        np.testing.assert_allclose(Y[:, j].cpu().numpy(), r.y.cpu().numpy(), atol=1e-14, rtol=1e-12)


def test_batch_hub_split(torch):
    leaves = 40_000
    base = synth.erdos_renyi(1_500, 0.005, seed=9)
    e = [(0, i) for i in range(1, leaves + 1)]
    rows = np.repeat(np.arange(base.n), base.degrees)
    e += [(int(a) + 1, int(b) + 1) for a, b in zip(rows, base.col_idx) if a < b]
    g = synth.from_edges(leaves + 1, e, name="hub")
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g)
    from paper_2412_10789_amd import chebyprop as cp

    srcs = [0, 3, 17, leaves, 1200, 5]
    qs = [cp.make_query("hkpr", 3.0, s, 1e-9) for s in srcs] + [cp.make_query("ppr", 0.2, s, 1e-7) for s in srcs]
    for bw in (8, 16):
        G.set_batch_width(len(qs), "f64", bw)
        print("CASE batch-hub", bw, flush=True)
        Y, infos = G.power_batch(qs, prec="f64")
        Y = Y.cpu().numpy()
        for j, q in enumerate(qs):
            kind = "hkpr" if q.kind == 1 else "ppr"
            ref = oracle_yK(g, q.source, kind, q.param, infos[j]["K"], P)
            assert compare(Y[:, j], ref)["max_abs"] <= 1e-11


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_deep_gathers_long_rows_and_hubs(torch, prec):
    """Tiles of 32 and 64 sources on a graph of 80 arcs a row take the
    16-deep gather form of the step kernel (stream rows, long rows and the
    segments of a 20,000-arc hub); every column against Alg. 3 in FP64 at
    its K."""
    base = synth.chung_lu(30_000, 1_200_000, 1.9, seed=5)
    n0 = base.n
    rows = np.repeat(np.arange(n0), base.degrees)
    e = [(int(a), int(b)) for a, b in zip(rows, base.col_idx) if a < b]
    e += [(n0, i) for i in range(20_000)]
    g = synth.from_edges(n0 + 1, e, name="dense-hub")
    assert g.nnz / g.n > 32 and int(g.degrees.max()) == 20_000
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g)
    from paper_2412_10789_amd import chebyprop as cp

    srcs = [n0, 0, 1, 7] + [int(s) for s in synth.sources(g, 36, seed=8)]
    kinds = [("ppr", 0.2), ("hkpr", 5.0), ("ppr", 0.1), ("hkpr", 3.0)]
    qs = [cp.make_query(*kinds[i % 4], s, 1e-7) for i, s in enumerate(srcs)]
    for bw in (32, 64):
        G.set_batch_width(len(qs), prec, bw)
        print("CASE deep gathers", prec, bw, flush=True)
        Y, infos = G.power_batch(qs, prec=prec)
        Y = Y.double().cpu().numpy()
        for j, q in enumerate(qs):
            kind = "hkpr" if q.kind == 1 else "ppr"
            ref = oracle_yK(g, q.source, kind, q.param, infos[j]["K"], P)
            m = compare(Y[:, j], ref)
            if prec == "f64":
                assert m["max_abs"] <= 1e-11, (bw, j, m)
            else:
                assert m["l1"] <= f32_bar(infos[j]["K"], kind, q.param), (bw, j, m)


def test_batch_edge_cases(torch):
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.chung_lu(5_000, 20_000, 2.5, seed=3)
    G = gpu_graph(g)
    s = int(synth.sources(g, 1, seed=1)[0])
    print("CASE batch-edge", flush=True)
    # one query, and duplicated sources with different parameters
    Y1, _ = G.power_batch([cp.make_query("ppr", 0.2, s, 1e-8)], prec="f64")
    r = G.power("ppr", 0.2, s, tol=1e-8, prec="f64")
    np.testing.assert_allclose(Y1[:, 0].cpu().numpy(), r.y.cpu().numpy(), atol=1e-15)
    qs = [cp.make_query("ppr", 0.2, s, 1e-8), cp.make_query("hkpr", 5.0, s, 1e-8),
          cp.make_query("ppr", 0.2, s, 1e-8)]
    Y, infos = G.power_batch(qs, prec="f64")
    np.testing.assert_array_equal(Y[:, 0].cpu().numpy(), Y[:, 2].cpu().numpy())
    # an invalid query anywhere rejects the whole batch
    Yb = torch.full((g.n, 3), 7.0, dtype=torch.float64, device="cuda")
    bad = [qs[0], cp.make_query("ppr", 0.2, g.n + 5, 1e-6), qs[1]]
    with pytest.raises(cp.ChebypropError) as ei:
        G.power_batch(bad, prec="f64", Y=Yb)
    assert ei.value.status == cp.CP_ESOURCE
    assert bool(torch.all(Yb == 7.0))
    with pytest.raises(cp.ChebypropError):
        G.set_batch_width(3, "f32", 12)


def test_autotune_picks_a_width(torch, mid_graph):
    g = mid_graph
    G = gpu_graph(g)
    qs, _ = _queries(g, 32, seed=8)
    print("CASE autotune", flush=True)
    bw = G.autotune_batch(qs, prec="f32")
    assert bw in (8, 16, 32)
    Y, infos = G.power_batch(qs, prec="f32")
    assert infos[0]["K"] > 0


@pytest.mark.slow
def test_orkut_shape_3m_full_size_batch_f32(torch):
    """The batched workload at full size, as the benchmark runs it: Chung-Lu
    n=3M, ~117M edges, exponent 2.2; 64 PPR alpha=0.2 sources with
    tolerances drawn from {1e-4, 1e-6, 1e-7}, certified K, FP32 storage,
    autotuned source-tile width.  The largest-K column of each tolerance
    class against the FP64 oracle at the same K; every column against the
    FP64 batch and Def. 3's fixed-point certificate, and for mass."""
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.chung_lu(3_000_000, 117_000_000, 2.2, seed=3)
    G = gpu_graph(g, reorder=True)
    srcs = [int(s) for s in synth.sources(g, 64, seed=3)]
    tols = [float(t) for t in synth.tolerance_choice(3, 64, (1e-4, 1e-6, 1e-7))]
    qs = [cp.make_query("ppr", 0.2, s, t) for s, t in zip(srcs, tols)]
    bw = G.autotune_batch(qs, prec="f32")
    print("CASE batch 3M width", bw, flush=True)
    Y, infos = G.power_batch(qs, prec="f32")
    Y = Y.double().cpu().numpy()
    Ks = [i["K"] for i in infos]
    print("CASE batch 3M f64", flush=True)
    Y64, infos64 = G.power_batch(qs, prec="f64")
    Y64 = Y64.cpu().numpy()
    G.close()
    assert [i["K"] for i in infos64] == Ks
    # the largest K of each tolerance class against the oracle's Alg. 3 at that K
    pick = sorted({max((j for j in range(64) if tols[j] == t), key=lambda j: Ks[j]) for t in set(tols)})
    ref = oracle_yK_multi(g, [("ppr", 0.2, srcs[j]) for j in pick], [Ks[j] for j in pick])
    for i, j in enumerate(pick):
        m = compare(Y[:, j], ref[:, i])
        m64 = compare(Y64[:, j], ref[:, i])
        print("batch 3M column", j, tols[j], Ks[j], m, "f64", m64, flush=True)
        assert m["l1"] <= f32_bar(Ks[j]), (j, m)
        assert m64["max_abs"] <= 1e-13, (j, m64)
    # every column: FP32 storage against the FP64 path (pinned to the oracle above and in the
    # smaller tests) to FP32 rounding, and Def. 3's fixed-point certificate
    from oracle import native as NO

    res = NO.ppr_residual_multi(g.row_ptr, g.col_idx, srcs, [0.2] * 64, Y)
    for j in range(64):
        d = E.l1(Y[:, j], Y64[:, j])
        assert d <= f32_bar(Ks[j]), (j, d)
        # ||res||_1 <= (2 - alpha) ||pi - y||_1, and ||pi - y||_1 <= tol + FP32 rounding
        assert res[j] / 0.2 <= 9.0 * (tols[j] + f32_bar(Ks[j])), (j, res[j], tols[j])
        assert abs(Y[:, j].sum() - 1.0) <= tols[j] + f32_bar(Ks[j]), j


@pytest.mark.parametrize("hot_nodes,stripes", [(None, False), (2000, False), (0, False), (3000, True)])
def test_hot_split_batch_matches_oracle(torch, mid_graph, monkeypatch, hot_nodes, stripes):
    """CP_GRAPH_HOT_SPLIT: the batched step sums each row's arcs into the
    hot_nodes highest-degree nodes in one pass and the rest in a second; every
    column still matches the oracle (all nodes hot, a few thousand hot, none
    hot, and the striped relabelling), in FP64 and FP32."""
    g = mid_graph
    if hot_nodes is not None:
        monkeypatch.setenv("CHEBYPROP_HOT_NODES", str(hot_nodes))
    else:
        monkeypatch.delenv("CHEBYPROP_HOT_NODES", raising=False)
    G = gpu_graph(g, hot_split=True, stripes=stripes)
    st = G.stats
    want = g.n if hot_nodes is None else min(hot_nodes, g.n)
    assert st["hot_nodes"] == want and st["reordered"] == 1
    assert (st["hot_arcs"] == g.nnz) if want == g.n else (0 <= st["hot_arcs"] < g.nnz)
    qs, meta = _queries(g, 21, seed=13)
    for prec in ("f64", "f32"):
        for bw in (8, 32):
            G.set_batch_width(21, prec, bw)
            print("CASE hot split", hot_nodes, stripes, prec, bw, flush=True)
            Y, infos = G.power_batch(qs, prec=prec)
            Y = Y.double().cpu().numpy()
            Ks = [i["K"] for i in infos]
            ref = oracle_yK_multi(g, meta, Ks)
            for j in range(len(qs)):
                m = compare(Y[:, j], ref[:, j])
                if prec == "f64":
                    assert m["max_abs"] <= 1e-13, (j, m)
                else:
                    assert m["l1"] <= f32_bar(Ks[j], *meta[j][:2]), (j, Ks[j], m)
    G.close()


def test_hot_split_hubs_server_and_propagate(torch, monkeypatch):
    """The split with hub rows (a 40,000-arc row whose cold part is split into
    segments, and 40,000 rows whose only arc is hot), through the batch, the
    server and feature propagation (forward and Clenshaw), against the
    unsplit graph's results and the oracle."""
    from paper_2412_10789_amd import chebyprop as cp

    leaves = 40_000
    base = synth.erdos_renyi(1_500, 0.005, seed=9)
    e = [(0, i) for i in range(1, leaves + 1)]
    rows = np.repeat(np.arange(base.n), base.degrees)
    e += [(int(a) + 1, int(b) + 1) for a, b in zip(rows, base.col_idx) if a < b]
    g = synth.from_edges(leaves + 1, e, name="hub")
    monkeypatch.setenv("CHEBYPROP_HOT_NODES", "100")
    Gs = gpu_graph(g, hot_split=True)
    monkeypatch.delenv("CHEBYPROP_HOT_NODES")
    G0 = gpu_graph(g, reorder=True)
    assert Gs.stats["hot_nodes"] == 100 and 0 < Gs.stats["hot_arcs"] < g.nnz
    srcs = [0, 3, 17, leaves, 1200, 5]
    qs = [cp.make_query("hkpr", 3.0, s, 1e-9) for s in srcs] + [cp.make_query("ppr", 0.2, s, 1e-7) for s in srcs]
    metas = [("hkpr", 3.0, s) for s in srcs] + [("ppr", 0.2, s) for s in srcs]
    print("CASE hot split hub batch", flush=True)
    Ys, infos = Gs.power_batch(qs, prec="f64")
    Y0, _ = G0.power_batch(qs, prec="f64")
    ref = oracle_yK_multi(g, metas, [i["K"] for i in infos])
    Ys, Y0 = Ys.cpu().numpy(), Y0.cpu().numpy()
    for j in range(len(qs)):
        assert compare(Ys[:, j], ref[:, j])["max_abs"] <= 1e-11, j
        assert compare(Ys[:, j], Y0[:, j])["max_abs"] <= 1e-12, j
    print("CASE hot split hub server", flush=True)
    S = cp.Server(Gs, hbm_budget_bytes=1 << 30, max_slots=16, prec="f64")
    ys = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in qs]
    tickets = [S.submit(q, y) for q, y in zip(qs, ys)]
    for j, t in enumerate(tickets):
        st, info = S.wait(t, timeout_ms=60_000)
        assert st == cp.CP_OK
        assert compare(ys[j].cpu().numpy(), ref[:, j])["max_abs"] <= 1e-11, j
    S.close()
    X = (torch.rand((g.n, 5), generator=torch.Generator().manual_seed(3), dtype=torch.float64) - 0.5).cuda()
    for method in ("cheby", "clenshaw"):
        print("CASE hot split propagate", method, flush=True)
        Zs, _ = Gs.propagate(X, "ppr", 0.2, a=0.5, K=12, kmode="fixed", prec="f64", method=method)
        Z0, _ = G0.propagate(X, "ppr", 0.2, a=0.5, K=12, kmode="fixed", prec="f64", method=method)
        d = (Zs - Z0).abs().max().item()
        assert d <= 1e-12 * Z0.abs().max().item(), (method, d)
    Gs.close()
    G0.close()


@pytest.mark.parametrize("shape", ["powerlaw", "hub"])
def test_autotune_row_splits(torch, shape):
    """cp_autotune_batch and cp_autotune_single time several row-split plans
    (long-row cuts, hub cut and segment size) and install the fastest: the
    stats report a candidate plan, results match the default plan's to FP64
    rounding (only the order of the sums of split rows changes) and the
    oracle, and a workspace sized before tuning stays valid."""
    from paper_2412_10789_amd import chebyprop as cp

    if shape == "powerlaw":
        g = synth.chung_lu(200_000, 2_400_000, 2.1, seed=12)
    else:
        leaves = 40_000
        base = synth.erdos_renyi(1_500, 0.005, seed=9)
        e = [(0, i) for i in range(1, leaves + 1)] + [(1, i) for i in range(2, 9_000)]
        rows = np.repeat(np.arange(base.n), base.degrees)
        e += [(int(a) + 1, int(b) + 1) for a, b in zip(rows, base.col_idx) if a < b]
        g = synth.from_edges(leaves + 1, e, name="hubs")
    G0 = gpu_graph(g)
    G = gpu_graph(g)
    qs, meta = _queries(g, 16, seed=21)
    ws_before, _ = G.workspace(16, cp.CP_F64)
    Y0, infos = G0.power_batch(qs, prec="f64")
    print("CASE autotune row splits", shape, flush=True)
    bw = G.autotune_batch(qs, prec="f64")
    st = G.stats
    print("autotuned", shape, "width", bw, "batch plan", st["batch_long_cut"], st["batch_hub_cut"],
          st["batch_hub_seg"], flush=True)
    assert st["batch_long_cut"] in (64, 128, 256, 512, 1024)
    assert (st["batch_hub_cut"], st["batch_hub_seg"]) in ((16384, 8192), (4096, 2048), (65536, 16384))
    ws_after, nbytes = G.workspace(16, cp.CP_F64)
    assert ws_after.numel() == ws_before.numel()  # sized for every candidate plan
    Y1, _ = G.power_batch(qs, prec="f64")
    Y0, Y1 = Y0.cpu().numpy(), Y1.cpu().numpy()
    ref = oracle_yK_multi(g, meta, [i["K"] for i in infos])
    for j in range(len(qs)):
        assert compare(Y1[:, j], Y0[:, j])["max_abs"] <= 1e-13 * max(1.0, np.abs(Y0[:, j]).max()), j
        assert compare(Y1[:, j], ref[:, j])["max_abs"] <= 1e-12, j
    kind, param, s = meta[0]
    r0 = G0.power(kind, param, s, tol=1e-9, prec="f64")
    st = G.autotune_single(kind, param, s, tol=1e-9, prec="f64")
    print("autotuned", shape, "single plan", st["single_long_cut"], st["single_hub_cut"], st["single_hub_seg"],
          flush=True)
    assert st["single_long_cut"] in (256, 512, 1024, 2048)
    r1 = G.power(kind, param, s, tol=1e-9, prec="f64")
    assert compare(r1.y.cpu().numpy(), r0.y.cpu().numpy())["max_abs"] <= 1e-13
    # striped graphs keep their stripe tiles
    Gs = gpu_graph(g, stripes=True)
    before = dict(Gs.stats)
    assert Gs.autotune_single(kind, param, s, tol=1e-9, prec="f64") == before
    for x in (G0, G, Gs):
        x.close()
