"""CSR row offsets beyond 2^31 (int64 offsets, int32 columns).

A circulant graph with n = 2^22 nodes and offsets -257..257 (0 excluded)
has 2,155,872,256 arcs, so the stream tiles past the 2^31-th arc start at
offsets that do not fit 32 bits.  The single-CSR layout, the XCD-striped
layout and the batched kernel run on it, and every result is checked
against the oracle's DFT closed forms: Algorithm 3's output at the GPU's K
(rounding error of FP32 storage) and the exact vector f(P) e_s (the
certified tolerance).  FP64 ChebyPower and ChebyPush without a threshold
(Alg. 4 with eps_a = 0, which is Algorithm 3 with the terms c_0..c_{K-1})
run on the same graph.  Sources sit next to the wrap-around rows, whose
columns are not sorted, and in the middle of the ring."""

import numpy as np
import pytest

from gpu_util import require_gpu
from oracle import circulant as CI
from oracle import coefficients as C
from oracle import errors as E

pytestmark = pytest.mark.gpu

N = 1 << 22
H = 257
SOURCES = (5, N // 2 + 12345)
QUERIES = (("ppr", 0.2), ("hkpr", 5.0))
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
    assert rp[-1] > 2**31 and ci.shape[0] == rp[-1]
    return offs, rp, ci


def _check(y, offs, s, kind, param, K):
    yK = CI.cheby_truncated(N, offs, s, C.chebyshev_coeffs(kind, param, K))
    ex = CI.exact(N, offs, s, kind, param)
    y = np.asarray(y, dtype=np.float64)
    m = {"l1_vs_series": E.l1(y, yK), "max_abs": E.max_abs(y, yK), "l1_vs_exact": E.l1(y, ex)}
    print("circulant 2^22", kind, param, s, "K", K, m, flush=True)
    assert m["l1_vs_series"] <= 1e-6, m  # FP32 storage against the FP64 series
    assert m["l1_vs_exact"] <= TOL, m


@pytest.mark.parametrize("layout", ["native", "stripes"])
def test_single_source_beyond_2_31_arcs(torch, circulant, layout):
    from paper_2412_10789_amd.chebyprop import Graph

    offs, rp, ci = circulant
    _case("large offsets create", layout)
    G = Graph(rp, ci, stripes=layout == "stripes")
    try:
        assert G.stats["nnz"] == rp[-1]
        if layout == "stripes":
            assert G.stats["stripe_count"] == 4 and G.stats["stripe_packed"] == 1
        for s in SOURCES:
            for kind, param in QUERIES:
                _case("large offsets", layout, s, kind)
                r = G.power(kind, param, s, tol=TOL, prec="f32")
                _check(r.y.cpu().numpy(), offs, s, kind, param, r.info["K"])
    finally:
        G.close()
        torch.cuda.empty_cache()


def test_batch_beyond_2_31_arcs(torch, circulant):
    from paper_2412_10789_amd import chebyprop as cp

    offs, rp, ci = circulant
    _case("large offsets batch create")
    G = cp.Graph(rp, ci)
    try:
        qs = [cp.make_query(kind, param, s, TOL) for s in SOURCES for kind, param in QUERIES]
        _case("large offsets batch", len(qs))
        Y, infos = G.power_batch(qs, prec="f32")
        Yh = Y.cpu().numpy()
        for j, q in enumerate(qs):
            kind = "hkpr" if q.kind == 1 else "ppr"
            _check(Yh[:, j], offs, q.source, kind, q.param, infos[j]["K"])
    finally:
        G.close()
        torch.cuda.empty_cache()


def test_f64_and_chebypush_beyond_2_31_arcs(torch, circulant):
    from paper_2412_10789_amd.chebyprop import CP_Q_STATS, Graph

    offs, rp, ci = circulant
    _case("large offsets f64/push create")
    G = Graph(rp, ci)
    try:
        s = SOURCES[0]
        _case("large offsets f64", s)
        r = G.power("hkpr", 5.0, s, tol=1e-9, prec="f64")
        K = r.info["K"]
        yK = CI.cheby_truncated(N, offs, s, C.chebyshev_coeffs("hkpr", 5.0, K))
        y = r.y.cpu().numpy()
        # the DFT form itself carries about 1e-17 of rounding per entry
        assert E.l1(y, yK) <= 1e-9 and E.max_abs(y, yK) <= 1e-13, (E.l1(y, yK), E.max_abs(y, yK))
        assert E.l1(y, CI.exact(N, offs, s, "hkpr", 5.0)) <= 1e-9
        # K = 80: the frontier passes nnz / 128 of volume, so late iterations are dense
        for kind, param, K in (("ppr", 0.2, 80), ("hkpr", 5.0, 14)):
            _case("large offsets push eps 0", kind, s)
            r = G.push(kind, param, s, 0.0, kmode="fixed", K=K, flags=CP_Q_STATS)
            ref = CI.cheby_truncated(N, offs, s, C.chebyshev_coeffs(kind, param, K)[:K])
            y = r.y.cpu().numpy()
            m = (E.l1(y, ref), E.max_abs(y, ref))
            print("circulant 2^22 push eps 0", kind, K, m, r.info["pushes"], r.info["arcs"], flush=True)
            assert m[0] <= 1e-9 and m[1] <= 1e-13, m
            assert r.info["arcs"] == r.info["pushes"] * 2 * H
    finally:
        G.close()
        torch.cuda.empty_cache()
