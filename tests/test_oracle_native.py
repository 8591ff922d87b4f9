"""The plain-C oracle against the pinned Python oracle and the paper's
worked example (CPU only)."""

import numpy as np
import pytest

import synth
from conftest import load_golden
from oracle import coefficients as C
from oracle import native as NO
from oracle import propagation as PR
from oracle import truncation as T


@pytest.fixture(scope="module", autouse=True)
def _built():
    NO.build(force=False)


def test_star_example():
    """Sec. 4.2: with c = e_k, Alg. 3 returns T_k(P) e_{v1}."""
    gold = load_golden("star_example.txt")
    g = synth.star(3)
    for k, key in [(1, "T1"), (2, "T2"), (3, "T3")]:
        c = np.zeros(k + 1)
        c[k] = 1.0
        np.testing.assert_allclose(NO.cheby_power(g.row_ptr, g.col_idx, 1, c, k), gold[key], atol=1e-15)


@pytest.mark.parametrize("kind,param", [("ppr", 0.2), ("ppr", 0.05), ("hkpr", 5.0)])
def test_matches_python_oracle(kind, param):
    g = synth.chung_lu(30_000, 200_000, 2.2, seed=6)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    for s in synth.sources(g, 2, seed=1):
        K = T.choose_K(kind, param, 1e-9, vol=g.nnz, d_s=g.degrees[s])
        c = C.chebyshev_coeffs(kind, param, K)
        a = NO.cheby_power(g.row_ptr, g.col_idx, int(s), c, K)
        b = PR.cheby_power(P, int(s), c, K)
        np.testing.assert_allclose(a, b, atol=1e-15, rtol=1e-12)
        N = T.pwmethod_steps(kind, param, 1e-10)
        z = C.taylor_coeffs(kind, param, N)
        np.testing.assert_allclose(NO.power_method(g.row_ptr, g.col_idx, int(s), z, N),
                                   PR.power_method(P, int(s), z, N), atol=1e-15, rtol=1e-12)


def test_isolated_nodes_and_mass():
    g = synth.from_edges(6, [(0, 1), (1, 2), (2, 0)], name="triangle+isolated")
    c = C.ppr_chebyshev_coeffs(0.3, 40)
    y = NO.cheby_power(g.row_ptr, g.col_idx, 0, c, 40)
    assert np.all(y[3:] == 0.0) and abs(y.sum() - 1.0) < 1e-12
    with pytest.raises(RuntimeError):
        NO.cheby_power(g.row_ptr, g.col_idx, 9, c, 40)


def test_matches_circulant_closed_form():
    """Plain-C Alg. 3 (and Alg. 1) on a circulant graph with 2^16 nodes and
    offsets -40..40 against the DFT closed forms (independent of any sparse
    product), with the unsorted wrap-around rows of the CSR builder."""
    from oracle import circulant as CI

    n, offs = 1 << 16, CI.offsets_band(40)
    rp, ci = CI.csr(n, offs)
    for kind, param, K in (("ppr", 0.2, 30), ("hkpr", 5.0, 18)):
        c = C.chebyshev_coeffs(kind, param, K)
        for s in (3, n // 2):
            y = NO.cheby_power(rp, ci, s, c, K)
            ref = CI.cheby_truncated(n, offs, s, c)
            assert np.abs(y - ref).sum() <= 1e-11, (kind, s)
            N = T.pwmethod_steps(kind, param, 1e-13)
            yp = NO.power_method(rp, ci, s, C.taylor_coeffs(kind, param, N), N)
            assert np.abs(yp - CI.exact(n, offs, s, kind, param)).sum() <= 1e-11, (kind, s)


def test_multi_source_columns_match_single_source():
    """Alg. 3 for several sources in one pass per step: every column equals
    the single-source run (same sums in the same order), with different K
    and coefficient rows per column, a repeated source and K = 1."""
    g = synth.chung_lu(30_000, 200_000, 2.2, seed=6)
    srcs = [int(s) for s in synth.sources(g, 5, seed=2)] + [0]
    srcs[5] = srcs[1]
    Ks = [3, 17, 25, 1, 9, 31]
    kinds = [("hkpr", 5.0), ("ppr", 0.2), ("ppr", 0.05), ("hkpr", 3.0), ("ppr", 0.2), ("hkpr", 5.0)]
    cs = [C.chebyshev_coeffs(k, p, K) for (k, p), K in zip(kinds, Ks)]
    Y = NO.cheby_power_multi(g.row_ptr, g.col_idx, srcs, cs, Ks)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    for j in range(len(srcs)):
        np.testing.assert_array_equal(Y[:, j], NO.cheby_power(g.row_ptr, g.col_idx, srcs[j], cs[j], Ks[j]))
        np.testing.assert_allclose(Y[:, j], PR.cheby_power(P, srcs[j], cs[j], Ks[j]), atol=1e-15, rtol=1e-12)


def test_multi_source_against_circulant_closed_form():
    """The multi-source form on a circulant graph (2^15 nodes, offsets
    -20..20) against the DFT form of Alg. 3's output, thread count 1 and
    the default (the sums do not depend on it)."""
    from oracle import circulant as CI

    n, offs = 1 << 15, CI.offsets_band(20)
    rp, ci = CI.csr(n, offs)
    srcs, Ks = [7, n // 3, n - 1], [12, 30, 5]
    cs = [C.chebyshev_coeffs("ppr", 0.2, 30)[:13], C.chebyshev_coeffs("ppr", 0.2, 30),
          C.chebyshev_coeffs("hkpr", 5.0, 5)]
    Y = NO.cheby_power_multi(rp, ci, srcs, cs, Ks)
    NO.set_threads(1)
    try:
        Y1 = NO.cheby_power_multi(rp, ci, srcs, cs, Ks)
    finally:
        NO.set_threads(0)
    np.testing.assert_array_equal(Y, Y1)
    for j, s in enumerate(srcs):
        ref = CI.cheby_truncated(n, offs, s, cs[j][:Ks[j] + 1])
        assert np.abs(Y[:, j] - ref).sum() <= 1e-11, j


def test_pwmethod_multi_columns_match_single_source_and_closed_form():
    """Alg. 1 for several sources in one pass per step: every column equals
    the single-source run bit for bit, with its own N and weights; on a
    circulant graph the columns match the DFT form of f(P) e_s to the exact
    Taylor tail."""
    g = synth.chung_lu(30_000, 200_000, 2.2, seed=6)
    srcs = [int(s) for s in synth.sources(g, 4, seed=3)]
    kinds = [("hkpr", 5.0), ("ppr", 0.2), ("hkpr", 3.0), ("ppr", 0.1)]
    Ns = [T.pwmethod_steps(k, p, 1e-10) for k, p in kinds]
    Ns[2] = 1
    zs = [C.taylor_coeffs(k, p, N) for (k, p), N in zip(kinds, Ns)]
    Y = NO.power_method_multi(g.row_ptr, g.col_idx, srcs, zs, Ns)
    for j in range(len(srcs)):
        np.testing.assert_array_equal(Y[:, j], NO.power_method(g.row_ptr, g.col_idx, srcs[j], zs[j], Ns[j]))
    from oracle import circulant as CI

    n, offs = 1 << 15, CI.offsets_band(20)
    rp, ci = CI.csr(n, offs)
    srcs = [5, n // 2]
    kinds = [("ppr", 0.2), ("hkpr", 5.0)]
    Ns = [T.pwmethod_steps(k, p, 1e-13) for k, p in kinds]
    Y = NO.power_method_multi(rp, ci, srcs, [C.taylor_coeffs(k, p, N) for (k, p), N in zip(kinds, Ns)], Ns)
    for j, ((k, p), s) in enumerate(zip(kinds, srcs)):
        assert np.abs(Y[:, j] - CI.exact(n, offs, s, k, p)).sum() <= 1e-11, j


def test_ppr_residual_multi_is_the_fixed_point_residual():
    """The residual of Def. 3's fixed-point equation: about zero at the exact
    PPR vector (dense solve), equal to the Python certificate times alpha on
    perturbed vectors, and (divided by alpha) never below the true l1 error."""
    from oracle import dense as D
    from oracle import errors as E

    g = synth.chung_lu(150, 600, 2.3, seed=4)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    srcs = [int(s) for s in synth.sources(g, 3, seed=5)]
    alphas = [0.2, 0.05, 0.5]
    A = D.adjacency(g.row_ptr, g.col_idx)
    exact = np.stack([D.ppr_solve(A, s, a) for s, a in zip(srcs, alphas)], axis=1)
    res0 = NO.ppr_residual_multi(g.row_ptr, g.col_idx, srcs, alphas, exact)
    assert np.all(res0 <= 1e-13), res0
    rng = np.random.default_rng(0)
    Yp = exact + rng.uniform(-1e-4, 1e-4, size=exact.shape)
    res = NO.ppr_residual_multi(g.row_ptr, g.col_idx, srcs, alphas, Yp)
    for j, (s, a) in enumerate(zip(srcs, alphas)):
        assert res[j] == pytest.approx(a * E.ppr_certificate(P, s, a, Yp[:, j]), rel=1e-12, abs=1e-15)
        assert res[j] / a >= E.l1(exact[:, j], Yp[:, j])
    # a truncated series: the bound holds and shrinks with K
    big = synth.chung_lu(30_000, 200_000, 2.2, seed=6)
    s = int(synth.sources(big, 1, seed=8)[0])
    ys = np.stack([NO.cheby_power(big.row_ptr, big.col_idx, s, C.ppr_chebyshev_coeffs(0.2, K), K)
                   for K in (10, 20, 30)], axis=1)
    rk = NO.ppr_residual_multi(big.row_ptr, big.col_idx, [s] * 3, [0.2] * 3, ys)
    assert rk[0] > rk[1] > rk[2] > 0.0
