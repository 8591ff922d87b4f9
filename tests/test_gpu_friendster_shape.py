"""The Friendster-sized workload's shape on the GPU: n near 2^26 nodes and
3.6 billion arcs (int64 row offsets, int32 columns).

1. A circulant graph with n = 2^26 nodes and offsets -27..27 (0 excluded)
   has 3,623,878,656 arcs.  On the XCD-striped layout it runs with 8
   stripes of plain column ids (each stripe's arcs start past 2^31 in the
   concatenated stripe CSR); it also runs on the single CSR and as a batch
   of 8 sources.  Every result is checked against the oracle's DFT closed
   forms: Algorithm 3's output at the GPU's K (rounding of the precision)
   and the exact vector f(P) e_s (the certified tolerance).
2. The seeded Chung-Lu graph the benchmark's headline runs on (n = 65M
   target nodes, 1.8 billion edges, exponent 2.1, with 11,945 rows above
   16,384 arcs split over several workgroups): its 8-source PPR batch in
   degree order with the hot/cold split, as the headline runs it, and one
   source on the striped layout, each checked against
   Def. 3's fixed-point equation (plain-C FP64 residual / alpha, a bound on
   the l1 distance to the exact vector) and for mass, and one batch column
   against plain-C FP64 Algorithm 3 at the same K.
"""

import numpy as np
import pytest

from gpu_util import require_gpu
from oracle import circulant as CI
from oracle import coefficients as C
from oracle import errors as E

pytestmark = pytest.mark.gpu

N = 1 << 26
H = 27
TOL = 1e-6


def _case(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def circulant():
    offs = CI.offsets_band(H)
    rp, ci = CI.csr(N, offs)
    assert rp[-1] == N * 2 * H and rp[-1] > 3 * 2**30
    return offs, rp, ci


_series_cache = {}


def _forms(offs, kind, param, K):
    """Alg. 3's output and the exact vector from node 0; other sources are
    rotations of these (the graph is vertex-transitive)."""
    key = (kind, param, K)
    if key not in _series_cache:
        _series_cache[key] = (CI.cheby_truncated(N, offs, 0, C.chebyshev_coeffs(kind, param, K)),
                              CI.exact(N, offs, 0, kind, param))
    return _series_cache[key]


def _check(y, offs, s, kind, param, K, prec):
    yK0, ex0 = _forms(offs, kind, param, K)
    yK, ex = np.roll(yK0, s), np.roll(ex0, s)
    y = np.asarray(y, dtype=np.float64)
    m = {"l1_vs_series": E.l1(y, yK), "max_abs": E.max_abs(y, yK), "l1_vs_exact": E.l1(y, ex)}
    print("circulant 2^26", prec, kind, param, s, "K", K, m, flush=True)
    if prec == "f64":
        # only the summation order differs; the DFT forms carry ~1e-17 per entry
        assert m["l1_vs_series"] <= 1e-9 and m["max_abs"] <= 1e-13, m
    else:
        # FP32 storage, double sums: measured l1 about 3e-8 at this size
        assert m["l1_vs_series"] <= 2e-7, m
    assert m["l1_vs_exact"] <= TOL, m


def test_striped_plain_ids_8_stripes(torch, circulant):
    from paper_2412_10789_amd.chebyprop import Graph

    offs, rp, ci = circulant
    _case("2^26 stripes create")
    G = Graph(rp, ci, stripes=True)
    try:
        st = G.stats
        assert st["stripe_count"] == 8 and st["stripe_packed"] == 0 and st["nnz"] == rp[-1]
        for s, kind, param, prec in ((3, "ppr", 0.2, "f32"), (N // 2 + 77, "hkpr", 5.0, "f32"),
                                     (N - 2, "hkpr", 5.0, "f64")):
            _case("2^26 stripes", prec, kind, s)
            r = G.power(kind, param, s, tol=TOL, prec=prec)
            _check(r.y.cpu().numpy(), offs, s, kind, param, r.info["K"], prec)
    finally:
        G.close()
        torch.cuda.empty_cache()


def test_single_csr_and_batch_of_8(torch, circulant):
    from paper_2412_10789_amd import chebyprop as cp

    offs, rp, ci = circulant
    _case("2^26 single CSR create")
    G = cp.Graph(rp, ci)
    try:
        _case("2^26 single CSR f32")
        r = G.power("ppr", 0.2, 11, tol=TOL, prec="f32")
        _check(r.y.cpu().numpy(), offs, 11, "ppr", 0.2, r.info["K"], "f32")
        srcs = [0, 1, 5, N // 3, N // 2, N // 2 + 1, N - 27, N - 1]
        for prec in ("f32", "f64"):
            qs = [cp.make_query("ppr", 0.2, s, TOL) for s in srcs]
            _case("2^26 batch of 8", prec)
            Y, infos = G.power_batch(qs, prec=prec)
            Yh = Y.cpu().numpy()
            del Y
            Ks = {i["K"] for i in infos}
            assert len(Ks) == 1  # a regular graph: the certified K does not depend on the source
            for j, s in enumerate(srcs):
                _check(Yh[:, j], offs, s, "ppr", 0.2, infos[j]["K"], prec)
            del Yh
    finally:
        G.close()
        torch.cuda.empty_cache()


@pytest.mark.slow
def test_friendster_shaped_chung_lu_batch_and_stripes(torch):
    import synth
    from oracle import native as NO
    from paper_2412_10789_amd import chebyprop as cp

    _case("friendster-shaped graph generate")
    g = synth.chung_lu(65_000_000, 1_800_000_000, 2.1, seed=5, tune_passes=0)
    assert g.nnz > 2**31 + 2**30
    alpha = 0.2
    srcs = [int(s) for s in synth.sources(g, 8, seed=5)]
    _case("friendster-shaped degree-order create, hot/cold split as the benchmark's headline")
    G = cp.Graph(g.row_ptr, g.col_idx, reorder=True, hot_split=True)
    try:
        assert G.stats["hub_rows"] > 1000 and G.stats["hot_nodes"] == 524_288
        assert 0.3 < G.stats["hot_arcs"] / g.nnz < 0.5
        _case("friendster-shaped batch of 8 f32")
        Y, infos = G.power_batch([cp.make_query("ppr", alpha, s, TOL) for s in srcs], prec="f32")
        Yh = Y.double().cpu().numpy()
        del Y
    finally:
        G.close()
        torch.cuda.empty_cache()
    _case("friendster-shaped striped create")
    Gs = cp.Graph(g.row_ptr, g.col_idx, stripes=True)
    try:
        assert Gs.stats["stripe_count"] == 8 and Gs.stats["stripe_packed"] == 0
        _case("friendster-shaped striped f32", srcs[0])
        r = Gs.power("ppr", alpha, srcs[0], tol=TOL, prec="f32")
        ys = r.y.double().cpu().numpy()
    finally:
        Gs.close()
        torch.cuda.empty_cache()
    _case("friendster-shaped fixed-point residuals")
    cols = np.concatenate([Yh, ys[:, None]], axis=1)
    res = NO.ppr_residual_multi(g.row_ptr, g.col_idx, srcs + [srcs[0]], [alpha] * 9, cols)
    bound = res / alpha
    mass = cols.sum(axis=0)
    print("friendster-shaped l1 bounds", bound.tolist(), "mass", mass.tolist(), flush=True)
    # ||res||_1 <= (2 - alpha) ||pi - y||_1, so a result within tol (plus FP32
    # rounding) of pi has a certificate within (2 - alpha) / alpha times that
    assert np.all(bound <= (2 - alpha) / alpha * (TOL + 2e-7)), bound
    # mass of a truncated PPR series is 1 - (truncated terms' mass), within tol
    assert np.all(np.abs(mass - 1.0) <= TOL), mass
    # batch column 0 and the striped single-source run are the same query
    assert E.l1(cols[:, 0], cols[:, 8]) <= 3e-7
    # batch column 0 against plain-C FP64 Alg. 3 at the same K (rounding of FP32 storage)
    _case("friendster-shaped plain-C oracle", srcs[0], infos[0]["K"])
    K = infos[0]["K"]
    ref = NO.cheby_power(g.row_ptr, g.col_idx, srcs[0], C.ppr_chebyshev_coeffs(alpha, K), K)
    m = (E.l1(cols[:, 0], ref), E.max_abs(cols[:, 0], ref))
    print("friendster-shaped batch column 0 vs FP64 Alg. 3:", m, flush=True)
    assert m[0] <= 2e-7, m
