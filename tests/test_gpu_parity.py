"""GPU ChebyPower (HIP library through the C ABI) against the FP64 oracle.

Tolerances: FP64 vectors are compared element by element with the oracle's
Alg. 3 at the same K to 1e-12 (only summation order differs).  FP32 storage
rounds each stored value to 2^-24 relative while the sums run in double;
measured l1 deviations are about 6e-8 at 4M nodes and smaller on smaller
graphs, and the tests allow F32_L1 = 1.2e-7 up to K = 30, in proportion to
K beyond, twice that for HKPR with t > 5 (float sums, measured 1.7e-7 for
t = 5 at K = 17, fail it).  BF16 storage measures 1.5e-3 to 5e-3 and is held to 8e-3.  The
contract against the exact vector (l1 <= tol) is checked with the certified
K, plus the rounding bar for FP32.
"""

import numpy as np
import pytest

import synth
from gpu_util import BF16_L1, F32_L1, compare, f32_bar, gpu_graph, oracle_exact_multi, oracle_yK, oracle_yK_multi, require_gpu
from oracle import errors as E
from oracle import propagation as PR

pytestmark = pytest.mark.gpu


def _print_case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def test_star_example_f64(torch):
    """Sec. 4.2 star, source v1: Alg. 3 with K = 1..3 against the oracle."""
    g = synth.star(3)
    G = gpu_graph(g)
    for K in (1, 2, 3):
        _print_case("star", K)
        r = G.power("ppr", 0.2, 1, prec="f64", kmode="fixed", K=K)
        ref = oracle_yK(g, 1, "ppr", 0.2, K)
        np.testing.assert_allclose(r.y.cpu().numpy(), ref, atol=1e-15)
        assert r.info["K"] == K and r.info["steps"] == K - 1


@pytest.mark.parametrize("kind,param", [("ppr", 0.2), ("ppr", 0.05), ("hkpr", 5.0), ("hkpr", 0.7)])
def test_tiny_graphs_f64(torch, kind, param):
    import pins

    for g in pins.tiny_graphs():
        s = int(np.flatnonzero(g.degrees > 0)[2])
        _print_case("tiny", g.name, kind, param, s)
        G = gpu_graph(g, validate=True)
        r = G.power(kind, param, s, tol=1e-12, prec="f64")
        ref = oracle_yK(g, s, kind, param, r.info["K"])
        np.testing.assert_allclose(r.y.cpu().numpy(), ref, atol=1e-13, rtol=1e-12)


def test_chung_lu_20k_f64(torch):
    """n=20,000 Chung-Lu, avg degree 10, exponent 2.5, PPR alpha=0.2, FP64,
    K certified for l1 <= 1e-8 against the exact vector."""
    g = synth.chung_lu(20_000, 100_000, 2.5, seed=1)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g)
    for s in synth.sources(g, 4, seed=1):
        _print_case("20k", int(s))
        r = G.power("ppr", 0.2, int(s), tol=1e-8, prec="f64", flags=1)
        y = r.y.cpu().numpy()
        ref_K = oracle_yK(g, s, "ppr", 0.2, r.info["K"], P)
        exact = PR.ground_truth(P, int(s), "ppr", 0.2)
        np.testing.assert_allclose(y, ref_K, atol=1e-14, rtol=1e-12)
        assert E.l1(y, exact) <= 1e-8
        assert abs(r.info["mass"] - 1.0) < 1e-8


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_powerlaw_tiles_and_long_rows(torch, prec, reorder):
    """200k-node power-law graph: thousands of stream tiles, a ragged last
    tile, rows longer than one tile (whole-workgroup rows)."""
    g = synth.chung_lu(200_000, 2_400_000, 2.1, seed=12)
    assert g.degrees.max() > 2048, "graph must contain long rows"
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, reorder=reorder)
    assert G.stats["long_rows"] > 0
    for kind, param in [("ppr", 0.2), ("hkpr", 5.0)]:
        for s in synth.sources(g, 2, seed=3):
            _print_case("powerlaw", prec, reorder, kind, int(s))
            r = G.power(kind, param, int(s), tol=1e-6, prec=prec)
            y = r.y.cpu().numpy()
            ref = oracle_yK(g, s, kind, param, r.info["K"], P)
            m = compare(y, ref)
            if prec == "f64":
                assert m["max_abs"] <= 1e-13, m
            else:
                assert m["l1"] <= f32_bar(r.info["K"], kind, param), m
            exact = PR.ground_truth(P, int(s), kind, param)
            assert E.l1(y, exact) <= 1e-6 + (0 if prec == "f64" else f32_bar(r.info["K"], kind, param))


def test_hub_rows_split_f64(torch):
    """A hub of degree 40,000 (split over several workgroups, combined in
    segment order) plus a random graph among its leaves."""
    leaves = 40_000
    rng_edges = synth.erdos_renyi(2_000, 0.004, seed=5)
    e = [(0, i) for i in range(1, leaves + 1)]
    rows = np.repeat(np.arange(rng_edges.n), rng_edges.degrees)
    e += [(int(a) + 1, int(b) + 1) for a, b in zip(rows, rng_edges.col_idx) if a < b]
    g = synth.from_edges(leaves + 1, e, name="hub")
    G = gpu_graph(g)
    assert G.stats["hub_rows"] == 1
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    for s in (0, 5, leaves):
        for prec in ("f64", "f32"):
            _print_case("hub", s, prec)
            r = G.power("hkpr", 3.0, s, tol=1e-10, prec=prec)
            ref = oracle_yK(g, s, "hkpr", 3.0, r.info["K"], P)
            m = compare(r.y.cpu().numpy(), ref)
            # a 40,000-term row sum: rounding up to d * eps * sum|x| (about 1e-11
            # in FP64, 1e-6 in FP32 relative to the hub value)
            assert m["max_abs"] <= (1e-11 if prec == "f64" else 1e-6), m


def test_isolated_nodes_and_errors(torch):
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.from_edges(8, [(0, 1), (1, 2), (2, 0), (4, 5)], name="with isolated")
    G = gpu_graph(g, validate=True)
    _print_case("isolated")
    r = G.power("ppr", 0.3, 0, tol=1e-12, prec="f64")
    y = r.y.cpu().numpy()
    assert np.all(y[[3, 6, 7]] == 0.0) and np.all(y[[4, 5]] == 0.0)
    ref = oracle_yK(g, 0, "ppr", 0.3, r.info["K"])
    np.testing.assert_allclose(y, ref, atol=1e-15)
    with pytest.raises(cp.ChebypropError) as ei:
        G.power("ppr", 0.3, 3)
    assert ei.value.status == cp.CP_EISOLATED
    with pytest.raises(cp.ChebypropError) as ei:
        G.power("ppr", 0.3, 8)
    assert ei.value.status == cp.CP_ESOURCE
    with pytest.raises(cp.ChebypropError) as ei:
        G.power("ppr", 1.5, 0)
    assert ei.value.status == cp.CP_EINVAL
    with pytest.raises(cp.ChebypropError) as ei:
        G.power("ppr", 0.2, 0, kmode="fixed", K=0)
    assert ei.value.status == cp.CP_EINVAL
    q = cp.make_query("ppr", 0.2, 0, 1e-6)
    y = torch.empty(g.n, dtype=torch.float32, device="cuda")
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_power(G.handle, q, cp.CP_F32, y.data_ptr(), 0, 0, 0)
    assert ei.value.status == cp.CP_EWORKSPACE


@pytest.mark.parametrize("layout", ["native", "degree", "stripes"])
def test_edgeless_graph(torch, layout):
    """Nodes and no edges: every node is isolated, so single-source, batched,
    push and walk queries report CP_EISOLATED, and feature propagation
    returns zeros (degree-0 rows are outside the propagation)."""
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.CSRGraph(np.zeros(6, dtype=np.int64), np.zeros(0, dtype=np.int32), name="edgeless")
    _print_case("edgeless", layout)
    G = gpu_graph(g, reorder=layout == "degree", stripes=layout == "stripes")
    assert G.stats["n"] == 5 and G.stats["nnz"] == 0
    calls = [lambda: G.power("ppr", 0.2, 2), lambda: G.power_batch([cp.make_query("ppr", 0.2, 1, 1e-6)]),
             lambda: G.push("ppr", 0.2, 0, 1e-6), lambda: G.push_rw(0.2, 3, 0.5, 1e-3, seed=1)]
    for call in calls:
        with pytest.raises(cp.ChebypropError) as ei:
            call()
        assert ei.value.status == cp.CP_EISOLATED
    X = torch.ones((5, 3), dtype=torch.float32, device="cuda")
    for method in ("cheby", "clenshaw"):
        Z, info = G.propagate(X, "ppr", 0.2, kmode="fixed", K=4, method=method)
        assert info["K"] == 4 and bool(torch.all(Z == 0))


@pytest.mark.parametrize("kind,param", [("ppr", 0.01), ("ppr", 0.003), ("hkpr", 20.0), ("hkpr", 60.0)])
def test_long_recurrences_f64(torch, kind, param):
    """Small alpha and large t (K from about 30 to several hundred) in FP64,
    single-source on the striped layout and batched, against the oracle's
    Alg. 3 at the same K (only summation order differs)."""
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.chung_lu(50_000, 300_000, 2.3, seed=13)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    srcs = [int(x) for x in synth.sources(g, 3, seed=8)]
    G = gpu_graph(g, stripes=True)
    _print_case("long", kind, param)
    r = G.power(kind, param, srcs[0], tol=1e-10, prec="f64")
    ref = oracle_yK(g, srcs[0], kind, param, r.info["K"], P)
    assert compare(r.y.cpu().numpy(), ref)["max_abs"] <= 1e-12 * np.abs(ref).max(), r.info["K"]
    Y, infos = G.power_batch([cp.make_query(kind, param, x, 1e-10) for x in srcs], prec="f64")
    for j, x in enumerate(srcs):
        ref = oracle_yK(g, x, kind, param, infos[j]["K"], P)
        assert compare(Y[:, j].cpu().numpy(), ref)["max_abs"] <= 1e-12 * np.abs(ref).max(), (j, infos[j]["K"])


def test_validation_rejects_bad_csr(torch):
    from paper_2412_10789_amd import chebyprop as cp

    rp = np.array([0, 1, 2, 2], np.int64)
    ci = np.array([1, 2], np.int32)  # 0->1, 1->2: not symmetric
    with pytest.raises(cp.ChebypropError) as ei:
        cp.Graph(rp, ci, validate=True)
    assert ei.value.status == cp.CP_EGRAPH
    rp = np.array([0, 1, 2], np.int64)
    ci = np.array([0, 1], np.int32)  # self-loops
    with pytest.raises(cp.ChebypropError) as ei:
        cp.Graph(rp, ci, validate=True)
    assert ei.value.status == cp.CP_EGRAPH


def test_decreasing_offsets_rejected_without_validation(torch):
    """Offsets that decrease (a negative degree) are rejected on every create,
    validation flag or not, for host and device inputs."""
    from paper_2412_10789_amd import chebyprop as cp

    rp = np.array([0, 2, 1, 3], np.int64)
    ci = np.array([1, 2, 0], np.int32)
    for host in (True, False):
        with pytest.raises(cp.ChebypropError) as ei:
            cp.Graph(rp, ci, host_input=host)
        assert ei.value.status == cp.CP_EINVAL


@pytest.mark.parametrize("layout", ["native", "degree", "stripes"])
def test_host_and_device_inputs_build_the_same_graph(torch, layout):
    """A graph created from host arrays (CP_GRAPH_HOST) and one created from
    device arrays give the same layout and bitwise the same results, single
    source and batched."""
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.chung_lu(200_000, 2_400_000, 2.1, seed=12)
    kw = dict(reorder=layout == "degree", stripes=layout == "stripes")
    Gh = gpu_graph(g, **kw)
    Gd = gpu_graph(g, host_input=False, **kw)
    assert Gh.stats == Gd.stats
    srcs = [int(s) for s in synth.sources(g, 3, seed=9)]
    for s in srcs:
        _print_case("host/device input", layout, s)
        for prec in ("f64", "f32"):
            a = Gh.power("hkpr", 5.0, s, tol=1e-7, prec=prec).y
            b = Gd.power("hkpr", 5.0, s, tol=1e-7, prec=prec).y
            assert torch.equal(a, b), (layout, s, prec)
    qs = [cp.make_query("ppr", 0.2, s, 1e-6) for s in srcs]
    Ya, _ = Gh.power_batch(qs, prec="f32")
    Yb, _ = Gd.power_batch(qs, prec="f32")
    assert torch.equal(Ya, Yb)
    Gh.close()
    Gd.close()


def test_bitwise_reproducible_and_timing(torch):
    g = synth.chung_lu(100_000, 900_000, 2.3, seed=2)
    G = gpu_graph(g)
    s = int(synth.sources(g, 1, seed=4)[0])
    _print_case("repro", s)
    a = G.power("hkpr", 5.0, s, tol=1e-6, prec="f32").y.clone()
    b = G.power("hkpr", 5.0, s, tol=1e-6, prec="f32", flags=2)
    assert torch.equal(a, b.y)
    assert b.info["elapsed_ms"] > 0 and 0 < b.info["step_ms"] <= b.info["elapsed_ms"]


@pytest.mark.parametrize("stripes", [False, True])
def test_bf16_storage_error_reported(torch, stripes):
    g = synth.chung_lu(100_000, 900_000, 2.3, seed=2)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, stripes=stripes)
    s = int(synth.sources(g, 1, seed=4)[0])
    _print_case("bf16", stripes, s)
    for kind, param in (("ppr", 0.2), ("hkpr", 5.0)):
        r = G.power(kind, param, s, tol=1e-6, prec="bf16")
        ref = oracle_yK(g, s, kind, param, r.info["K"], P)
        m = compare(r.y.cpu().numpy(), ref)
        print("bf16 storage error vs FP64 oracle:", kind, stripes, m)
        assert m["l1"] <= BF16_L1, m


@pytest.mark.slow
def test_livejournal_shape_4m_full_size_f32(torch):
    """Chung-Lu n=4M, ~35M edges, exponent 2.3; HKPR t=5, FP32, l1 tol 1e-6:
    on the XCD-striped layout (the one the benchmark times) all 16 of the
    benchmark's sources, on the other layouts two, each full vector against
    Alg. 3 in FP64 at its K and against the converged vector."""
    g = synth.chung_lu(4_000_000, 35_000_000, 2.3, seed=2)
    srcs16 = [int(s) for s in synth.sources(g, 16, seed=2)]
    for layout in ("stripes", "native", "degree"):
        G = gpu_graph(g, reorder=layout == "degree", stripes=layout == "stripes")
        if layout == "stripes":
            assert G.stats["stripe_packed"] == 1 and G.stats["stripe_count"] == 4
        srcs = srcs16 if layout == "stripes" else srcs16[:2]
        ys, Ks = [], []
        for s in srcs:
            _print_case("4M", layout, s)
            r = G.power("hkpr", 5.0, s, tol=1e-6, prec="f32")
            ys.append(r.y.double().cpu().numpy())
            Ks.append(r.info["K"])
        G.close()
        metas = [("hkpr", 5.0, s) for s in srcs]
        ref = oracle_yK_multi(g, metas, Ks)
        exact = oracle_exact_multi(g, metas)
        for j, s in enumerate(srcs):
            m = compare(ys[j], ref[:, j])
            ex = E.l1(ys[j], exact[:, j])
            print("4M", layout, s, Ks[j], m, "vs exact", ex, flush=True)
            assert m["l1"] <= F32_L1, (s, m)
            assert ex <= 1e-6, (s, ex)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_xcd_striped_layout(torch, prec):
    """XCD-striped single-source steps (8 column stripes, partial sums
    combined in stripe order) against the oracle: many row tiles, rows
    whose stripe segment exceeds one LDS tile, ragged stripes (n % 8 != 0)."""
    g = synth.chung_lu(150_003, 2_400_000, 2.0, seed=17)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, stripes=True)
    assert G.stats["stripe_tiles"] > 0 and G.stats["reordered"] == 1 and G.stats["stripe_packed"] == 1
    assert G.stats["stripe_count"] == 2
    for kind, param in [("ppr", 0.2), ("hkpr", 5.0)]:
        for s in synth.sources(g, 2, seed=7):
            _print_case("striped", prec, kind, int(s))
            r = G.power(kind, param, int(s), tol=1e-7, prec=prec)
            ref = oracle_yK(g, s, kind, param, r.info["K"], P)
            m = compare(r.y.cpu().numpy(), ref)
            assert m["max_abs"] <= (1e-13 if prec == "f64" else 1e-8), m
            assert m["l1"] <= (1e-12 if prec == "f64" else 2e-7), m


@pytest.mark.parametrize("n_total,stripes", [(3_000_003, 4), (6_000_005, 8)])
def test_xcd_stripe_counts(torch, n_total, stripes):
    """The stripe count follows n (the fewest of 2, 4, 8 whose FP32 slice of
    the vector fits 4 MiB); a 100k-node power-law core padded with isolated
    nodes runs with 4 and with 8 stripes in the packed form."""
    core = synth.chung_lu(100_000, 800_000, 2.1, seed=29)
    rp = np.concatenate([core.row_ptr, np.full(n_total - core.n, core.nnz, dtype=np.int64)])
    g = synth.CSRGraph(rp, core.col_idx, name="core + isolated")
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, stripes=True)
    assert G.stats["stripe_count"] == stripes and G.stats["stripe_packed"] == 1
    s = int(synth.sources(core, 1, seed=4)[0])
    for prec in ("f64", "f32"):
        for kind, param in [("ppr", 0.2), ("hkpr", 5.0)]:
            _print_case("stripe-count", stripes, prec, kind, s)
            r = G.power(kind, param, s, tol=1e-7, prec=prec)
            ref = oracle_yK(g, s, kind, param, r.info["K"], P)
            m = compare(r.y.cpu().numpy(), ref)
            assert m["max_abs"] <= (1e-13 if prec == "f64" else 1e-8), m
            assert m["l1"] <= (1e-12 if prec == "f64" else 2e-7), m
    G.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_xcd_striped_plain_form_above_2_24_nodes(torch, prec):
    """Stripes of more than 2^21 nodes keep plain column ids (no packed
    form): a 100k-node power-law core padded with isolated nodes to
    n = 2^24 + 9."""
    core = synth.chung_lu(100_000, 800_000, 2.1, seed=23)
    n = (1 << 24) + 9
    rp = np.concatenate([core.row_ptr, np.full(n - core.n, core.nnz, dtype=np.int64)])
    g = synth.CSRGraph(rp, core.col_idx, name="core + isolated")
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, stripes=True)
    assert G.stats["stripe_tiles"] > 0 and G.stats["stripe_packed"] == 0 and G.stats["stripe_count"] == 8
    for kind, param in [("ppr", 0.2), ("hkpr", 5.0)]:
        s = int(synth.sources(core, 1, seed=3)[0])
        _print_case("striped-plain", prec, kind, s)
        r = G.power(kind, param, s, tol=1e-7, prec=prec)
        ref = oracle_yK(g, s, kind, param, r.info["K"], P)
        m = compare(r.y.cpu().numpy(), ref)
        assert m["max_abs"] <= (1e-13 if prec == "f64" else 1e-8), m
        assert m["l1"] <= (1e-12 if prec == "f64" else 2e-7), m
    G.close()


def test_xcd_striped_hub_and_tiny(torch):
    from paper_2412_10789_amd import chebyprop as cp  # noqa: F401

    leaves = 40_000
    e = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, leaves, 3)]
    g = synth.from_edges(leaves + 1, e, name="hub+chain")
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, stripes=True)
    for s in (0, 7, leaves):
        _print_case("striped-hub", s)
        r = G.power("hkpr", 3.0, s, tol=1e-10, prec="f64")
        ref = oracle_yK(g, s, "hkpr", 3.0, r.info["K"], P)
        assert compare(r.y.cpu().numpy(), ref)["max_abs"] <= 1e-11
    for gg in (synth.star(3), synth.path(5), synth.complete(9)):
        G = gpu_graph(gg, stripes=True)
        for K in (1, 2, 5):
            _print_case("striped-tiny", gg.name, K)
            r = G.power("ppr", 0.2, 1, prec="f64", kmode="fixed", K=K)
            np.testing.assert_allclose(r.y.cpu().numpy(), oracle_yK(gg, 1, "ppr", 0.2, K), atol=1e-15)
