"""CP_F32F, FP32 storage with FP32 arithmetic (float sums, float partials and
a float estimate), through the C ABI against the FP64 oracle: single-source
queries on every layout (Alg. 3 and Alg. 1), batches with and without the
hot/cold split, the server, feature-matrix propagation, and the benchmark's
16 sources at full LiveJournal size."""

import numpy as np
import pytest

import synth
from gpu_util import compare, f32f_bar, gpu_graph, oracle_exact_multi, oracle_yK, oracle_yK_multi, require_gpu
from oracle import coefficients as C
from oracle import errors as E
from oracle import generalized as GG
from oracle import propagation as PR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def mid_graph():
    return synth.chung_lu(150_000, 1_500_000, 2.2, seed=31)


KINDS = [("ppr", 0.2), ("ppr", 0.1), ("hkpr", 5.0), ("hkpr", 10.0)]


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.mark.parametrize("layout", ["native", "degree", "stripes"])
def test_single_source_every_layout(torch, mid_graph, layout):
    """Every query against Alg. 3 in FP64 at its K and against the converged
    vector; the float path differs from CP_F32's double one, and a PwMethod
    query against Alg. 1 in FP64 at its N."""
    g = mid_graph
    G = gpu_graph(g, reorder=layout != "native", stripes=layout == "stripes")
    srcs = [int(s) for s in synth.sources(g, 8, seed=6)]
    metas = [(*KINDS[i % 4], s) for i, s in enumerate(srcs)]
    ys, Ks, same = [], [], 0
    for kind, param, s in metas:
        _case("f32f single", layout, kind, param, s)
        r = G.power(kind, param, s, tol=1e-6, prec="f32f")
        r32 = G.power(kind, param, s, tol=1e-6, prec="f32")
        assert r.info["K"] == r32.info["K"]
        same += int(torch.equal(r.y, r32.y))
        ys.append(r.y.double().cpu().numpy())
        Ks.append(r.info["K"])
    assert same == 0, "FP32 arithmetic gave the double-arithmetic results"
    ref = oracle_yK_multi(g, metas, Ks)
    exact = oracle_exact_multi(g, metas)
    for j, (kind, param, s) in enumerate(metas):
        m = compare(ys[j], ref[:, j])
        assert m["l1"] <= f32f_bar(Ks[j]), (kind, param, s, Ks[j], m)
        assert E.l1(ys[j], exact[:, j]) <= 1e-6 + f32f_bar(Ks[j]), (kind, param, s)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    kind, param, s = metas[0]
    _case("f32f pwmethod", layout, s)
    r = G.power(kind, param, s, tol=1e-6, prec="f32f", method="power")
    N = r.info["K"]
    ref = PR.power_method(P, s, C.taylor_coeffs(kind, param, N), N)
    assert compare(r.y.double().cpu().numpy(), ref)["l1"] <= f32f_bar(N)


@pytest.mark.parametrize("hot_split", [False, True])
def test_batch_columns(torch, mid_graph, hot_split, monkeypatch):
    """37 queries (a ragged last tile) at widths 8 and 32, every column
    against Alg. 3 in FP64 at its K; with the hot/cold split the hot pass's
    partials are float too."""
    g = mid_graph
    if hot_split:
        monkeypatch.setenv("CHEBYPROP_HOT_NODES", "4096")
    G = gpu_graph(g, reorder=True, hot_split=hot_split)
    from paper_2412_10789_amd import chebyprop as cp

    srcs = [int(s) for s in synth.sources(g, 37, seed=9)]
    metas = [(*KINDS[i % 4], s) for i, s in enumerate(srcs)]
    tols = synth.tolerance_choice(9, 37, (1e-4, 1e-6))
    qs = [cp.make_query(k, p, s, float(t)) for (k, p, s), t in zip(metas, tols)]
    for bw in (8, 32):
        G.set_batch_width(len(qs), "f32f", bw)
        _case("f32f batch", hot_split, bw)
        Y, infos = G.power_batch(qs, prec="f32f")
        Y = Y.double().cpu().numpy()
        Ks = [i["K"] for i in infos]
        ref = oracle_yK_multi(g, metas, Ks)
        for j in range(len(qs)):
            m = compare(Y[:, j], ref[:, j])
            assert m["l1"] <= f32f_bar(Ks[j]), (bw, j, Ks[j], m)


def test_hub_rows(torch):
    """A 40,000-arc hub row (split into segments whose float partials the
    last workgroup adds) on the single CSR, the XCD stripes and in a batch;
    against Alg. 3 in FP64 at the same K."""
    leaves = 40_000
    base = synth.erdos_renyi(1_500, 0.005, seed=9)
    e = [(0, i) for i in range(1, leaves + 1)]
    rows = np.repeat(np.arange(base.n), base.degrees)
    e += [(int(a) + 1, int(b) + 1) for a, b in zip(rows, base.col_idx) if a < b]
    g = synth.from_edges(leaves + 1, e, name="hub")
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    from paper_2412_10789_amd import chebyprop as cp

    srcs = [0, 3, leaves, 1200]
    for stripes in (False, True):
        G = gpu_graph(g, stripes=stripes)
        if not stripes:
            assert G.stats["hub_rows"] > 0
        for s in srcs:
            _case("f32f hub single", stripes, s)
            r = G.power("hkpr", 3.0, s, tol=1e-7, prec="f32f")
            ref = oracle_yK(g, s, "hkpr", 3.0, r.info["K"], P)
            assert compare(r.y.double().cpu().numpy(), ref)["l1"] <= f32f_bar(r.info["K"]), (stripes, s)
        G.close()
    G = gpu_graph(g)
    qs = [cp.make_query("ppr", 0.2, s, 1e-7) for s in srcs]
    _case("f32f hub batch")
    Y, infos = G.power_batch(qs, prec="f32f")
    Y = Y.double().cpu().numpy()
    for j, s in enumerate(srcs):
        ref = oracle_yK(g, s, "ppr", 0.2, infos[j]["K"], P)
        assert compare(Y[:, j], ref)["l1"] <= f32f_bar(infos[j]["K"]), s
    G.close()


def test_server(torch, mid_graph):
    """Served CP_F32F queries (batched launches and the idle server's
    single-source path) against Alg. 3 in FP64 at their K."""
    g = mid_graph
    G = gpu_graph(g, stripes=True)
    from paper_2412_10789_amd import chebyprop as cp

    S = cp.Server(G, hbm_budget_bytes=1 << 30, max_slots=64, prec="f32f")
    assert S.stats()["tile_width"] == 32
    srcs = [int(s) for s in synth.sources(g, 40, seed=12)]
    metas = [(*KINDS[i % 4], s) for i, s in enumerate(srcs)]
    ys = [torch.empty(g.n, dtype=torch.float32, device="cuda") for _ in metas]
    _case("f32f server")
    tickets = [S.submit(cp.make_query(k, p, s, 1e-6), y) for (k, p, s), y in zip(metas, ys)]
    got = [S.wait(t, timeout_ms=60_000) for t in tickets]
    assert all(st == cp.CP_OK for st, _ in got)
    Ks = [info["K"] for _, info in got]
    ref = oracle_yK_multi(g, metas, Ks)
    for j, y in enumerate(ys):
        m = compare(y.double().cpu().numpy(), ref[:, j])
        assert m["l1"] <= f32f_bar(Ks[j]), (j, Ks[j], m)
    S.close()


def test_propagate(torch, mid_graph):
    """A feature matrix in forward and Clenshaw form against Def. 8 in FP64:
    column l1 relative to the column's l1."""
    g = mid_graph
    G = gpu_graph(g)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((g.n, 5)).astype(np.float32)
    Xd = torch.tensor(X, device="cuda")
    Xref = Xd.double().cpu().numpy()
    for method in ("cheby", "clenshaw"):
        _case("f32f propagate", method)
        Z, info = G.propagate(Xd, "ppr", 0.2, a=0.5, kmode="fixed", K=20, prec="f32f", method=method)
        ref = GG.generalized_gp(g.row_ptr, g.col_idx, Xref, 0.5, "ppr", 0.2, 20, method=method)
        Z = Z.double().cpu().numpy()
        for j in range(5):
            rel = np.abs(Z[:, j] - ref[:, j]).sum() / np.abs(ref[:, j]).sum()
            assert rel <= 1e-6, (method, j, rel)


@pytest.mark.slow
def test_livejournal_shape_4m_sixteen_sources(torch):
    """The benchmark's 16 HKPR t = 5 sources on the 4M-node graph (XCD
    stripes), every result against Alg. 3 in FP64 at its K and against the
    converged vector (tolerance 1e-6 plus the rounding bar)."""
    g = synth.chung_lu(4_000_000, 35_000_000, 2.3, seed=2)
    srcs = [int(s) for s in synth.sources(g, 16, seed=2)]
    G = gpu_graph(g, stripes=True)
    ys, Ks = [], []
    for s in srcs:
        _case("f32f 4M", s)
        r = G.power("hkpr", 5.0, s, tol=1e-6, prec="f32f")
        ys.append(r.y.double().cpu().numpy())
        Ks.append(r.info["K"])
    G.close()
    metas = [("hkpr", 5.0, s) for s in srcs]
    ref = oracle_yK_multi(g, metas, Ks)
    exact = oracle_exact_multi(g, metas)
    for j, s in enumerate(srcs):
        m = compare(ys[j], ref[:, j])
        ex = E.l1(ys[j], exact[:, j])
        print("f32f 4M", s, Ks[j], m, "vs exact", ex, flush=True)
        assert m["l1"] <= f32f_bar(Ks[j]), (s, m)
        assert ex <= 1e-6 + f32f_bar(Ks[j]), (s, ex)
