"""ChebyPush (Alg. 4) on the GPU (cp_push through the C ABI) against the
oracle's Alg. 4.

Selection is a floating-point decision (|r(u)| > eps_k d_u) and the GPU sums
each row's pushed values in another order than the oracle, so the two sides
can only disagree on a node whose residual sits on its threshold to
rounding.  Each
case checks the oracle's smallest relative distance of a residual to its
threshold first (well above 1e-9 here); then the GPU must take the same
decisions (same number of pushes and arcs) and match to FP64 rounding."""

import numpy as np
import pytest

import synth
from gpu_util import gpu_graph, oracle_yK, require_gpu
from oracle import coefficients as C
from oracle import propagation as PR
from oracle import push as PU
from oracle import truncation as T

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _check(G, g, s, kind, param, K, eps_a, a=0.0):
    c = C.chebyshev_coeffs(kind, param, K)
    ref, tr = PU.cheby_push(g.row_ptr, g.col_idx, s, c, K, eps_a, trace=True)
    assert tr["margin"] > 1e-9, ("decision on the threshold", tr["margin"])
    r = G.push(kind, param, s, eps_a, kmode="fixed", K=K, a=a, flags=1)
    assert r.info["K"] == K and r.info["steps"] == K - 1
    assert r.info["pushes"] == sum(len(S) for S in tr["sets"])
    assert r.info["arcs"] == sum(int(g.degrees[S].sum()) for S in tr["sets"])
    if a != 0.0:
        from oracle import generalized as GG

        ref = GG.single_source_generalized(g.row_ptr, g.col_idx, s, a, ref)
    y = r.y.cpu().numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-15 * max(1.0, np.abs(ref).max()))
    assert abs(r.info["mass"] - ref.sum()) <= 1e-12 * max(1.0, abs(ref.sum()))
    return r, tr


def test_tiny_graphs(torch):
    import pins

    for g in pins.tiny_graphs():
        G = gpu_graph(g)
        s = int(np.flatnonzero(g.degrees > 0)[2])
        for kind, param, K in (("ppr", 0.2, 12), ("hkpr", 3.0, 9)):
            for eps_a in (3e-2, 1e-3, 1e-5):
                _case("push-tiny", g.name, kind, eps_a)
                _check(G, g, s, kind, param, K, eps_a)


@pytest.mark.parametrize("layout", ["native", "degree", "stripes"])
def test_chung_lu_20k(torch, layout):
    """n=20,000 Chung-Lu: local (small eps_a frontier) and nearly global runs,
    in three graph layouts (results in caller ids)."""
    g = synth.chung_lu(20_000, 100_000, 2.5, seed=1)
    G = gpu_graph(g, reorder=layout == "degree", stripes=layout == "stripes")
    for s in synth.sources(g, 2, seed=5):
        for kind, param, eps_a in (("ppr", 0.2, 1e-4), ("hkpr", 5.0, 1e-5), ("ppr", 0.1, 1e-7)):
            K = T.choose_K(kind, param, eps_a / 2, mode="tail")
            _case("push-20k", layout, int(s), kind, eps_a)
            _check(G, g, int(s), kind, param, K, eps_a)


def test_degree_normalized_error_and_output_space(torch):
    """Thm. 4 on a 200k-node power-law graph (long rows, hubs in the
    frontier), and the Def. 8 output space."""
    g = synth.chung_lu(200_000, 2_400_000, 2.1, seed=12)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, reorder=True)
    s = int(synth.sources(g, 1, seed=4)[0])
    for kind, param, eps_a in (("ppr", 0.2, 1e-6), ("hkpr", 5.0, 1e-7)):
        K = T.choose_K(kind, param, eps_a / 2, mode="tail")
        _case("push-200k", kind, eps_a)
        r, tr = _check(G, g, s, kind, param, K, eps_a)
        exact = PR.ground_truth(P, s, kind, param)
        assert PU.degree_normalized_error(exact, r.y.cpu().numpy(), g.degrees) < eps_a
        assert r.info["arcs"] < (K - 1) * g.nnz  # local: less than the global iteration
    _case("push-200k a=1/2")
    _check(G, g, s, "ppr", 0.2, 20, 1e-5, a=0.5)


@pytest.mark.parametrize("n_total,stripes", [(3_000_003, 4), (6_000_005, 8)])
def test_striped_dense_pulls_with_4_and_8_stripes(torch, n_total, stripes):
    """Dense iterations pull through the XCD-striped step kernels with the
    graph's own stripe count: a 100k-node power-law core padded with
    isolated nodes to 4 and 8 stripes, at thresholds that make some
    iterations dense (vol(S_k) > nnz/128) and others sparse."""
    core = synth.chung_lu(100_000, 800_000, 2.1, seed=33)
    rp = np.concatenate([core.row_ptr, np.full(n_total - core.n, core.nnz, dtype=np.int64)])
    g = synth.CSRGraph(rp, core.col_idx, name="core + isolated")
    G = gpu_graph(g, stripes=True)
    assert G.stats["stripe_count"] == stripes
    s = int(synth.sources(core, 1, seed=6)[0])
    for kind, param, eps_a in (("ppr", 0.2, 1e-6), ("hkpr", 5.0, 1e-8)):
        K = T.choose_K(kind, param, eps_a / 2, mode="tail")
        _case("push-stripes", stripes, kind, eps_a)
        r, tr = _check(G, g, s, kind, param, K, eps_a)
        vols = [int(g.degrees[S].sum()) for S in tr["sets"]]
        assert max(vols) * 128 > g.nnz and min(vols) * 128 <= g.nnz, vols  # both forms ran


def test_hub_and_isolated_nodes(torch):
    leaves = 40_000
    e = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, leaves, 3)]
    g = synth.from_edges(leaves + 3, e, name="hub+chain+2 isolated")
    G = gpu_graph(g)
    for s, eps_a in ((0, 1e-6), (7, 1e-8)):
        _case("push-hub", s, eps_a)
        r, _ = _check(G, g, s, "hkpr", 3.0, 10, eps_a)
        assert np.all(r.y.cpu().numpy()[leaves + 1:] == 0.0)


def test_without_threshold_equals_first_K_terms_of_alg3(torch):
    """eps_a = 0: every non-zero residual is pushed, which is Alg. 3 with the
    terms c_0..c_{K-1}; compared with cp_power at K - 1 on the same graph."""
    g = synth.chung_lu(60_000, 400_000, 2.2, seed=21)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g)
    s = int(synth.sources(g, 1, seed=9)[0])
    K = 15
    _case("push-eps0")
    r = G.push("ppr", 0.2, s, 0.0, kmode="fixed", K=K)
    c = C.chebyshev_coeffs("ppr", 0.2, K)
    ref = PR.cheby_power(P, s, c[:K], K - 1)
    np.testing.assert_allclose(r.y.cpu().numpy(), ref, rtol=1e-11, atol=1e-16)
    assert abs(oracle_yK(g, s, "ppr", 0.2, K, P) - ref).max() > 0  # the dropped term is real


def test_push_argument_errors(torch):
    from paper_2412_10789_amd import chebyprop as cp

    g = synth.star(4)
    G = gpu_graph(g)
    for kw, status in [(dict(eps_a=-1.0), cp.CP_EINVAL), (dict(eps_a=float("nan")), cp.CP_EINVAL),
                       (dict(eps_a=1e-3, flags=cp.CP_Q_PWMETHOD), cp.CP_EINVAL),
                       (dict(eps_a=1e-3, source=9), cp.CP_ESOURCE)]:
        src = kw.pop("source", 1)
        with pytest.raises(cp.ChebypropError) as ei:
            G.push("ppr", 0.2, src, **kw)
        assert ei.value.status == status, kw
