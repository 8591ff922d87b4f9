"""Generalized graph propagation on the GPU (Def. 8, Thm. 5) against the
oracle: single-source outputs in the D^{-a} A D^{-b} space (cp_query.a) for
single, batched and served queries, and feature matrices through
cp_propagate (Alg. 3, its Clenshaw form and Alg. 1 from dense start vectors
D^{a} x_j).

Tolerances: FP64 results differ from the oracle only in summation order
(max-abs within 1e-11 of the column's largest entry); FP32 storage rounds
every stored iterate to 2^-24 relative, so columns are compared in relative
l1 (5e-6)."""

import numpy as np
import pytest

import synth
from gpu_util import gpu_graph, oracle_yK, require_gpu
from oracle import generalized as GG
from oracle import propagation as PR

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def graph():
    return synth.chung_lu(60_000, 400_000, 2.2, seed=21)


def _features(n, k, seed):
    return (synth.uniform01(seed, n * k) - 0.5).reshape(n, k)


def _check_cols(Z, ref, prec, what):
    for j in range(ref.shape[1]):
        scale = np.max(np.abs(ref[:, j]))
        if prec == "f64":
            err = np.max(np.abs(Z[:, j] - ref[:, j]))
            assert err <= 1e-11 * scale + 1e-300, (what, j, err, scale)
        else:
            rel = np.sum(np.abs(Z[:, j] - ref[:, j])) / np.sum(np.abs(ref[:, j]))
            assert rel <= 5e-6, (what, j, rel)


@pytest.mark.parametrize("stripes", [False, True])
def test_single_source_output_space(torch, graph, stripes):
    """cp_query.a: z = d_s^a D^{-a} y (the single-source form of Thm. 5)."""
    g = graph
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, stripes=stripes)
    s = int(synth.sources(g, 1, seed=2)[0])
    for kind, param in (("ppr", 0.2), ("hkpr", 5.0)):
        for a in (0.5, 1.0, 0.3):
            _case("out-space", stripes, kind, a)
            r = G.power(kind, param, s, tol=1e-9, prec="f64", a=a, flags=1)
            y = oracle_yK(g, s, kind, param, r.info["K"], P)
            ref = GG.single_source_generalized(g.row_ptr, g.col_idx, s, a, y)
            z = r.y.cpu().numpy()
            assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))
            assert abs(r.info["mass"] - ref.sum()) <= 1e-10 * abs(ref.sum())


def test_batch_and_server_output_space(torch, graph):
    from paper_2412_10789_amd import chebyprop as cp

    g = graph
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    G = gpu_graph(g, reorder=True)
    srcs = synth.sources(g, 19, seed=6)
    avals = [0.0, 0.5, 1.0, 0.25]
    qs = [cp.make_query("ppr" if i % 2 else "hkpr", 0.15 if i % 2 else 3.0, int(srcs[i]), 1e-9,
                        a=avals[i % 4], method="power" if i % 3 == 2 else "cheby") for i in range(19)]
    _case("out-space batch")
    Y, infos = G.power_batch(qs, prec="f64")
    Y = Y.cpu().numpy()
    S = cp.Server(G, hbm_budget_bytes=2 << 30, max_slots=16, prec="f64")
    ys = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in qs]
    tickets = [S.submit(q, y) for q, y in zip(qs, ys)]
    for j, q in enumerate(qs):
        st, info = S.wait(tickets[j], timeout_ms=60_000)
        assert st == cp.CP_OK
        kind = "hkpr" if q.kind == 1 else "ppr"
        K = infos[j]["K"]
        if q.flags & cp.CP_Q_PWMETHOD:
            from oracle import coefficients as C

            y = PR.power_method(P, q.source, C.taylor_coeffs(kind, q.param, K), K)
        else:
            y = oracle_yK(g, q.source, kind, q.param, K, P)
        ref = GG.single_source_generalized(g.row_ptr, g.col_idx, q.source, q.a, y)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(Y[:, j] - ref)) <= 1e-12 * scale, ("batch", j)
        assert np.max(np.abs(ys[j].cpu().numpy() - ref)) <= 1e-12 * scale, ("server", j)
    S.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 5, 37])
def test_propagate_feature_matrix(torch, graph, prec, k):
    """Z = f(D^{-a} A D^{-b}) X for k columns (ragged last tile for k = 37)."""
    g = graph
    G = gpu_graph(g, reorder=k == 5)
    X = _features(g.n, k, seed=k)
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    Xref = Xd.double().cpu().numpy()  # the values the GPU reads
    for kind, param, K in (("ppr", 0.2, 25), ("hkpr", 5.0, 18)):
        for a in (0.0, 0.5, 1.0):
            _case("propagate", prec, k, kind, a)
            Z, info = G.propagate(Xd, kind, param, a=a, kmode="fixed", K=K, prec=prec)
            assert info["K"] == K and info["steps"] == K
            ref = GG.generalized_gp(g.row_ptr, g.col_idx, Xref, a, kind, param, K)
            _check_cols(Z.double().cpu().numpy(), ref, prec, (kind, a))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 37])
def test_propagate_clenshaw(torch, graph, prec, k):
    """CP_Q_CLENSHAW: Alg. 3's series by Clenshaw's backward recurrence
    against the oracle's Clenshaw form; FP64 also against the GPU's forward
    form (the same series, other rounding).  FP32 keeps b_k in float, whose
    rounding is carried by later steps like the forward form's r_k."""
    g = graph
    G = gpu_graph(g, reorder=k == 37)
    X = _features(g.n, k, seed=k + 100)
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    Xref = Xd.double().cpu().numpy()
    for kind, param, K in (("ppr", 0.2, 25), ("hkpr", 5.0, 18), ("ppr", 0.1, 1), ("hkpr", 3.0, 2)):
        for a in (0.0, 0.5, 1.0):
            _case("clenshaw", prec, k, kind, K, a)
            Z, info = G.propagate(Xd, kind, param, a=a, kmode="fixed", K=K, prec=prec, method="clenshaw")
            assert info["K"] == K and info["steps"] == K
            ref = GG.generalized_gp(g.row_ptr, g.col_idx, Xref, a, kind, param, K, method="clenshaw")
            _check_cols(Z.double().cpu().numpy(), ref, prec, ("clenshaw", kind, K, a))
            if prec == "f64":
                Zf, _ = G.propagate(Xd, kind, param, a=a, kmode="fixed", K=K, prec=prec)
                _check_cols(Z.cpu().numpy(), Zf.cpu().numpy(), prec, ("clenshaw vs forward", kind, K, a))


def test_propagate_pwmethod_tail_rule_and_in_place(torch, graph):
    """Alg. 1 from D^{a} x_j with N from the exact Taylor tail; Z may be X."""
    from oracle import truncation as T

    g = graph
    G = gpu_graph(g, stripes=True)
    X = _features(g.n, 8, seed=3)
    Xd = torch.tensor(X, dtype=torch.float64, device="cuda")
    _case("propagate pw")
    Z, info = G.propagate(Xd, "ppr", 0.2, a=0.5, tol=1e-10, prec="f64", method="power")
    N = info["K"]
    assert N == T.pwmethod_steps("ppr", 0.2, 1e-10)
    ref = GG.generalized_gp(g.row_ptr, g.col_idx, X, 0.5, "ppr", 0.2, N, method="power")
    _check_cols(Z.cpu().numpy(), ref, "f64", "pw")
    # in place, Chebyshev, tail rule
    K = T.choose_K("hkpr", 3.0, 1e-10, mode="tail")
    _case("propagate in place")
    Z2, info2 = G.propagate(Xd, "hkpr", 3.0, a=1.0, tol=1e-10, kmode="tail", prec="f64", Z=Xd)
    assert info2["K"] == K and Z2.data_ptr() == Xd.data_ptr()
    ref2 = GG.generalized_gp(g.row_ptr, g.col_idx, X, 1.0, "hkpr", 3.0, K)
    _check_cols(Xd.cpu().numpy(), ref2, "f64", "in place")


def test_propagate_degree_zero_nodes_and_hubs(torch):
    """Degree-0 rows of Z are 0 whatever X holds there; a hub row split over
    workgroups."""
    leaves = 30_000
    e = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, leaves, 4)]
    g = synth.from_edges(leaves + 5, e, name="hub+chain+4 isolated")
    G = gpu_graph(g)
    X = _features(g.n, 3, seed=4) + 1.0
    Xd = torch.tensor(X, dtype=torch.float64, device="cuda")
    _case("propagate hub/isolated")
    Z, _ = G.propagate(Xd, "ppr", 0.3, a=0.5, kmode="fixed", K=20, prec="f64")
    Z = Z.cpu().numpy()
    assert np.all(Z[leaves + 1:] == 0.0)
    ref = GG.generalized_gp(g.row_ptr, g.col_idx, X, 0.5, "ppr", 0.3, 20)
    _check_cols(Z, ref, "f64", "hub")


def test_propagate_argument_errors(torch, graph):
    from paper_2412_10789_amd import chebyprop as cp

    G = gpu_graph(synth.star(4))
    Xd = torch.zeros((5, 2), dtype=torch.float32, device="cuda")
    for kw, status in [(dict(kmode="certified"), cp.CP_EINVAL), (dict(a=1.5, kmode="fixed", K=3), cp.CP_EINVAL),
                       (dict(kmode="fixed", K=5000), cp.CP_EKMAX),
                       (dict(kmode="fixed", K=3, flags=cp.CP_Q_STATS), cp.CP_EINVAL),
                       (dict(kmode="fixed", K=3, flags=cp.CP_Q_CLENSHAW | cp.CP_Q_PWMETHOD), cp.CP_EINVAL)]:
        with pytest.raises(cp.ChebypropError) as ei:
            G.propagate(Xd, "ppr", 0.2, **kw)
        assert ei.value.status == status, kw
    with pytest.raises(cp.ChebypropError) as ei:
        G.power("ppr", 0.2, 1, a=-0.1)
    assert ei.value.status == cp.CP_EINVAL
    with pytest.raises(cp.ChebypropError) as ei:  # Clenshaw is for cp_propagate only
        G.power("ppr", 0.2, 1, method="clenshaw")
    assert ei.value.status == cp.CP_EINVAL
