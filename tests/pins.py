"""Pins for the oracle: each function checks one part of the oracle against
something the paper or the mathematics fixes independently of it, and
raises AssertionError when the oracle disagrees.

test_oracle_pins.py asserts that they all pass; test_oracle_planted.py
plants plausible mistakes in the oracle and asserts that each one makes at
least one pin fail.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.special as ss

import synth
from conftest import load_golden
from oracle import bidirectional as BI
from oracle import circulant as CI
from oracle import coefficients as C
from oracle import dense as D
from oracle import errors as E
from oracle import generalized as GG
from oracle import propagation as PR
from oracle import push as PU
from oracle import truncation as T

GP_CASES = [("ppr", 0.2), ("ppr", 0.05), ("ppr", 0.5), ("hkpr", 0.7), ("hkpr", 5.0), ("hkpr", 12.0)]


def tiny_graphs():
    """Small graphs with varied spectra: irregular, bipartite, long-diameter."""
    return [
        synth.erdos_renyi(40, 0.15, seed=3),
        synth.barbell_with_tail(6, 5),
        synth.star(7),
        synth.path(9),
        synth.erdos_renyi(120, 0.05, seed=11),
    ]


def _connected_node(g, seed=0):
    deg = g.degrees
    return int(np.flatnonzero(deg > 0)[seed % int(np.sum(deg > 0))])


# ---------------------------------------------------------------- recurrence


def pin_star_example():
    """Sec. 4.2 worked example (tests/golden/star_example.txt)."""
    gold = load_golden("star_example.txt")
    g = synth.star(3)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    r = PR.chebyshev_vectors(P, 1, 3)
    np.testing.assert_allclose(-r[0], gold["minus_T0"], atol=1e-15)
    np.testing.assert_allclose(r[1], gold["T1"], atol=1e-15)
    np.testing.assert_allclose(r[2], gold["T2"], atol=1e-15)
    np.testing.assert_allclose(r[3], gold["T3"], atol=1e-15)


def pin_chebyshev_vectors_eigen():
    """T_k(P) e_s from the recurrence vs cos(k arccos lambda) on A~'s
    spectrum (Def. 6 + Lemma 1 proof), irregular graphs."""
    for g in tiny_graphs():
        A = D.adjacency(g.row_ptr, g.col_idx)
        if np.any(A.sum(0) == 0):
            continue
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        s = _connected_node(g, 5)
        r = PR.chebyshev_vectors(P, s, 12)
        for k in range(13):
            Tk = D.chebyshev_matrix_eigen(A, k)
            np.testing.assert_allclose(r[k], Tk[:, s], atol=1e-11, err_msg=f"{g.name} k={k}")


def pin_mass():
    """Property 1: sum_u T_k(P) e_s (u) = 1 for every k."""
    g = synth.chung_lu(3000, 12000, 2.4, seed=5)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = _connected_node(g, 17)
    _, st = PR.cheby_power(P, s, C.chebyshev_coeffs("ppr", 0.2, 30), 30, stats=True)
    np.testing.assert_allclose(st["sum_r"], 1.0, atol=1e-10)


def pin_cycle_closed_form():
    """Cycle C_n: P is the circulant (shift + shift^-1)/2 with eigenvalues
    cos(2 pi j / n); f(P) e_s(u) = (1/n) sum_j f(cos(2 pi j/n)) cos(2 pi j (u-s)/n)."""
    n = 17
    g = synth.cycle(n)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = 4
    for kind, p in [("ppr", 0.15), ("hkpr", 3.0)]:
        f = C.gp_function(kind, p)
        j = np.arange(n)
        u = np.arange(n)
        exact = (f(np.cos(2 * np.pi * j / n))[None, :] *
                 np.cos(2 * np.pi * np.outer(u - s, j) / n)).sum(1) / n
        K = T.choose_K(kind, p, 1e-14, mode="tail")
        y = PR.cheby_power(P, s, C.chebyshev_coeffs(kind, p, K), K)
        np.testing.assert_allclose(y, exact, atol=1e-13)


def pin_circulant_closed_forms():
    """Circulant graphs (a band and an irregular symmetric offset set, n a
    power of two and not): the DFT forms of f(P) e_s and of
    sum_k c_k T_k(P) e_s against the dense definitions (Def. 3 solve,
    Def. 4 expm) and against Algorithm 3 with sparse products; the CSR
    builder against the edge set it should hold."""
    for n, offs in ((64, CI.offsets_band(3)), (50, np.array([-12, -5, -1, 1, 5, 12]))):
        rp, ci = CI.csr(n, offs)
        want = {(v, (v + int(o)) % n) for v in range(n) for o in offs}
        got = {(v, int(c)) for v in range(n) for c in ci[rp[v]:rp[v + 1]]}
        assert got == want and len(got) == ci.shape[0]
        assert all((b, a) in got for a, b in got) and all(a != b for a, b in got)
        A = D.adjacency(rp, ci)
        P = PR.transition_matrix(rp, ci)
        for s in (0, 7):
            np.testing.assert_allclose(CI.exact(n, offs, s, "ppr", 0.2), D.ppr_solve(A, s, 0.2), atol=1e-13)
            np.testing.assert_allclose(CI.exact(n, offs, s, "hkpr", 3.0), D.hkpr_expm(A, s, 3.0), atol=1e-13)
            for kind, p, K in (("ppr", 0.2, 6), ("hkpr", 5.0, 11)):
                c = C.chebyshev_coeffs(kind, p, K)
                np.testing.assert_allclose(CI.cheby_truncated(n, offs, s, c), PR.cheby_power(P, s, c, K),
                                           atol=1e-13)


def pin_complete_closed_form():
    """K_n: P = (J - I)/(n-1), eigenvalue 1 on the constant vector and
    -1/(n-1) elsewhere: f(P) e_s = f(1)/n 1 + f(-1/(n-1)) (e_s - 1/n)."""
    n = 9
    g = synth.complete(n)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = 2
    for kind, p in [("ppr", 0.3), ("hkpr", 2.0)]:
        f = C.gp_function(kind, p)
        e = np.zeros(n)
        e[s] = 1.0
        exact = f(1.0) / n + f(-1.0 / (n - 1)) * (e - 1.0 / n)
        K = T.choose_K(kind, p, 1e-14, mode="tail")
        y = PR.cheby_power(P, s, C.chebyshev_coeffs(kind, p, K), K)
        np.testing.assert_allclose(y, exact, atol=1e-13)


# ---------------------------------------------------------------- coefficients


def pin_ppr_closed_values():
    """Lemma 2 at alpha = 0.2 (tests/golden/ppr_alpha_0_2.txt)."""
    gold = load_golden("ppr_alpha_0_2.txt")
    g, b = C.ppr_gamma_beta(0.2)
    assert abs(g - gold["gamma"][0]) < 1e-15 and abs(b - gold["beta"][0]) < 1e-15
    np.testing.assert_allclose(C.ppr_chebyshev_coeffs(0.2, 4), gold["c0_to_c4"], rtol=1e-14)
    c = C.ppr_chebyshev_coeffs(0.2, 200)
    alt = np.sum(c * (-1.0) ** np.arange(201))
    assert abs(alt - gold["f_minus_one"][0]) < 1e-14


def _gauss_legendre(fn, a: float, b: float, nodes: int) -> float:
    x, w = ss.roots_legendre(nodes)
    t = 0.5 * (b - a) * x + 0.5 * (b + a)
    return float(0.5 * (b - a) * np.sum(w * fn(t)))


def pin_coefficient_integrals():
    """Lemma 1's definition integrated numerically in theta = arccos x:
    c_k = (2/pi) int_0^pi f(cos th) cos(k th) dth (1/pi for k = 0), by
    Gauss-Legendre quadrature (a method independent of the trapezoid rule
    and the recurrences the oracle uses) at 96 and 128 nodes; the two must
    agree (the integrand is analytic, so the rule has converged) before the
    value is compared."""
    for kind, p in GP_CASES:
        f = C.gp_function(kind, p)
        c = C.chebyshev_coeffs(kind, p, 12)
        for k in range(13):
            def fn(th, k=k):
                return np.asarray(f(np.cos(th)), dtype=np.float64) * np.cos(k * th)

            v1 = _gauss_legendre(fn, 0.0, math.pi, 96)
            v2 = _gauss_legendre(fn, 0.0, math.pi, 128)
            assert abs(v1 - v2) <= 1e-13, (kind, p, k, v1, v2)
            ref = v2 * (1.0 if k == 0 else 2.0) / math.pi
            assert abs(c[k] - ref) <= 1e-13 + 1e-11 * abs(ref), (kind, p, k, c[k], ref)


def pin_hkpr_library():
    """Lemma 3 vs scipy's exponentially scaled Bessel function ive."""
    for t in (0.3, 1.0, 5.0, 10.0, 30.0):
        c = C.hkpr_chebyshev_coeffs(t, 60)
        ref = np.r_[ss.ive(0, t), 2.0 * ss.ive(np.arange(1, 61), t)]
        np.testing.assert_allclose(c, ref, atol=2e-15, rtol=1e-12)


def pin_coefficient_sums():
    """f(1) = 1 (coefficients sum to one, Lemma 4 proof) and
    sum (-1)^k c_k = f(-1) (T_k(-1) = (-1)^k)."""
    for kind, p in GP_CASES:
        f = C.gp_function(kind, p)
        K = T.choose_K(kind, p, 1e-14, mode="tail") + 10
        c = C.chebyshev_coeffs(kind, p, K)
        assert abs(c.sum() - 1.0) < 1e-13, (kind, p, c.sum())
        assert abs(np.sum(c * (-1.0) ** np.arange(K + 1)) - float(f(-1.0))) < 1e-13


def pin_expansion_pointwise():
    """Lemma 1: |f(l) - sum_{k<=K} c_k T_k(l)| <= tail(K) on [-1, 1], with
    T_k(l) = cos(k arccos l) (Def. 6 closed form, not the recurrence)."""
    lam = np.linspace(-1.0, 1.0, 201)
    for kind, p in GP_CASES:
        f = C.gp_function(kind, p)
        tails = T.chebyshev_tails(kind, p, 40)
        c = C.chebyshev_coeffs(kind, p, 40)
        for K in (1, 2, 5, 10, 20, 40):
            approx = sum(c[k] * np.cos(k * np.arccos(lam)) for k in range(K + 1))
            err = np.max(np.abs(f(lam) - approx))
            assert err <= tails[K] * (1 + 1e-9) + 1e-14, (kind, p, K, err, tails[K])


def pin_taylor_sums():
    """Def. 3 / Def. 4 Taylor coefficients sum to f(1) = 1."""
    for kind, p in GP_CASES:
        N = T.pwmethod_steps(kind, p, 1e-16)
        z = C.taylor_coeffs(kind, p, N + 50)
        assert abs(z.sum() - 1.0) < 1e-13


# ---------------------------------------------------------------- results


def pin_dense_definitions():
    """ChebyPower (Alg. 3) at a K whose tail is 1e-14 vs the definitions:
    dense inverse (Def. 3), expm (Def. 4), eigen route (Lemma 1)."""
    for g in tiny_graphs():
        A = D.adjacency(g.row_ptr, g.col_idx)
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        s = _connected_node(g, 3)
        for kind, p in GP_CASES:
            L = T.certified_multiplier(g.nnz, g.degrees[s])
            K = T.choose_K(kind, p, 1e-13, mode="certified", vol=g.nnz, d_s=g.degrees[s])
            y = PR.cheby_power(P, s, C.chebyshev_coeffs(kind, p, K), K)
            ref = D.ppr_solve(A, s, p) if kind == "ppr" else D.hkpr_expm(A, s, p)
            eig = D.matrix_function_eigen(A, s, C.gp_function(kind, p))
            assert E.l1(y, ref) < 1e-12, (g.name, kind, p, E.l1(y, ref))
            assert E.l1(eig, ref) < 1e-11, (g.name, kind, p)
            assert L >= 1.0


def pin_truncated_series_eigen():
    """y^_K of Alg. 3 equals sum_{k<=K} c_k T_k(P) e_s, formed on A~'s
    spectrum with T_k(l) = cos(k arccos l), for every small K."""
    for g in tiny_graphs()[:3]:
        A = D.adjacency(g.row_ptr, g.col_idx)
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        s = _connected_node(g, 1)
        for kind, p in [("ppr", 0.2), ("hkpr", 5.0)]:
            for K in range(1, 9):
                c = C.chebyshev_coeffs(kind, p, K)
                pK = lambda lam, c=c, K=K: sum(c[k] * np.cos(k * np.arccos(lam)) for k in range(K + 1))
                ref = D.matrix_function_eigen(A, s, pK)
                y = PR.cheby_power(P, s, c, K)
                np.testing.assert_allclose(y, ref, atol=1e-12, err_msg=f"{g.name} {kind} K={K}")


def pin_pwmethod_exact_tail():
    """Alg. 1 after N terms misses exactly sum_{k>=N} zeta_k in l1."""
    g = synth.erdos_renyi(60, 0.12, seed=8)
    A = D.adjacency(g.row_ptr, g.col_idx)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = _connected_node(g, 2)
    for kind, p in [("ppr", 0.2), ("hkpr", 4.0)]:
        ref = D.ppr_solve(A, s, p) if kind == "ppr" else D.hkpr_expm(A, s, p)
        for N in (3, 10, 25):
            y = PR.power_method(P, s, C.taylor_coeffs(kind, p, N), N)
            tail = T.taylor_tail(kind, p, N)
            assert abs(E.l1(y, ref) - tail) <= 1e-12 + 1e-9 * tail, (kind, N, E.l1(y, ref), tail)
            assert np.all(ref - y >= -1e-14)


def pin_certified_bound_and_certificate():
    """||y - y^_K||_1 <= sqrt(vol/d_s) tail(K) for all K, and the PPR
    fixed-point certificate bounds the true l1 error from above."""
    g = synth.chung_lu(2000, 9000, 2.3, seed=21)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = _connected_node(g, 40)
    for kind, p in [("ppr", 0.2), ("hkpr", 5.0)]:
        ref = PR.ground_truth(P, s, kind, p)
        tails = T.chebyshev_tails(kind, p, 40)
        L = T.certified_multiplier(g.nnz, g.degrees[s])
        for K in (2, 5, 10, 20, 30):
            y = PR.cheby_power(P, s, C.chebyshev_coeffs(kind, p, K), K)
            err = E.l1(y, ref)
            assert err <= L * tails[K] + 1e-13, (kind, K, err, L * tails[K])
            if kind == "ppr":
                cert = E.ppr_certificate(P, s, p, y)
                assert cert >= err * (1 - 1e-9) - 1e-15, (K, cert, err)


def pin_convergence_rate():
    """Lemma 4: l1 error falls like beta^K.  On a bipartite graph
    (eigenvalue -1 present) the error after K terms is dominated by
    c_{K+1} T_{K+1}(-1), so log(err) has slope log(beta) in K."""
    g = synth.star(5)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    A = D.adjacency(g.row_ptr, g.col_idx)
    s = 2
    for alpha in (0.2, 0.05):
        ref = D.ppr_solve(A, s, alpha)
        _, beta = C.ppr_gamma_beta(alpha)
        Ks = np.arange(6, 30, 2)
        errs = [E.l1(PR.cheby_power(P, s, C.ppr_chebyshev_coeffs(alpha, K), K), ref) for K in Ks]
        slope = np.polyfit(Ks, np.log(errs), 1)[0]
        assert abs(slope - math.log(beta)) < 0.05 * abs(math.log(beta)), (alpha, slope, math.log(beta))


# ---------------------------------------------------------------- Def. 8 / Thm. 5


def _features(n, k, seed):
    return (synth.uniform01(seed, n * k) - 0.5).reshape(n, k)


def pin_generalized_definition():
    """Z = f(D^{-a} A D^{-b}) X, b = 1 - a, formed densely from Def. 8, against
    Thm. 5's route (the series of Alg. 3 and of Alg. 1 on D^{a} X, then
    D^{-a}) for several a, on graphs without degree-0 nodes."""
    for g in tiny_graphs()[:4]:
        A = D.adjacency(g.row_ptr, g.col_idx)
        X = _features(g.n, 3, seed=g.n)
        for kind, p, K in [("ppr", 0.2, 60), ("hkpr", 3.0, 40)]:
            N = T.pwmethod_steps(kind, p, 1e-15)
            for a in (0.0, 0.3, 0.5, 1.0):
                ref = D.generalized_definition(A, X, a, kind, p)
                Zc = GG.generalized_gp(g.row_ptr, g.col_idx, X, a, kind, p, K, method="cheby")
                Zp = GG.generalized_gp(g.row_ptr, g.col_idx, X, a, kind, p, N, method="power")
                assert np.max(np.abs(Zc - ref)) < 1e-11, (g.name, kind, a, np.max(np.abs(Zc - ref)))
                assert np.max(np.abs(Zp - ref)) < 1e-11, (g.name, kind, a, np.max(np.abs(Zp - ref)))


def pin_clenshaw_truncated_series():
    """Clenshaw's backward form equals sum_{k<=K} c_k T_k(P) x with T_k(P)
    formed on A~'s spectrum (cos(k arccos lambda)), for every K <= 9 and
    random coefficients and start vectors; and Def. 8 at a large K."""
    for g in tiny_graphs()[:4]:
        A = D.adjacency(g.row_ptr, g.col_idx)
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        Tk = [D.chebyshev_matrix_eigen(A, k) for k in range(10)]
        x = _features(g.n, 1, seed=g.n + 7)[:, 0]
        c = _features(10, 1, seed=g.n + 8)[:, 0]
        for K in range(1, 10):
            ref = sum(c[k] * (Tk[k] @ x) for k in range(K + 1))
            got = GG.clenshaw_vector(P, x, c, K)
            assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))), (g.name, K)
        X = _features(g.n, 2, seed=g.n)
        for kind, p, K in [("ppr", 0.2, 60), ("hkpr", 3.0, 40)]:
            for a in (0.0, 0.5, 1.0):
                ref = D.generalized_definition(A, X, a, kind, p)
                Z = GG.generalized_gp(g.row_ptr, g.col_idx, X, a, kind, p, K, method="clenshaw")
                assert np.max(np.abs(Z - ref)) < 1e-11, (g.name, kind, a)


def pin_generalized_symmetric_half():
    """a = 1/2: f(D^{-1/2} A D^{-1/2}) is a symmetric matrix, so Z for X = I
    is symmetric (and not for a = 0 on an irregular graph)."""
    g = synth.barbell_with_tail(5, 4)
    X = np.eye(g.n)
    Z = GG.generalized_gp(g.row_ptr, g.col_idx, X, 0.5, "ppr", 0.15, 80)
    assert np.max(np.abs(Z - Z.T)) < 1e-12
    Z0 = GG.generalized_gp(g.row_ptr, g.col_idx, X, 0.0, "ppr", 0.15, 80)
    assert np.max(np.abs(Z0 - Z0.T)) > 1e-3


def pin_generalized_single_source():
    """X = e_s: Thm. 5 reduces to the single-source form d_s^{a} D^{-a} f(P) e_s,
    and for a = 0 to Alg. 3 itself."""
    g = synth.erdos_renyi(40, 0.15, seed=3)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = _connected_node(g, 5)
    for kind, p, K in [("ppr", 0.1, 30), ("hkpr", 5.0, 25)]:
        y = PR.cheby_power(P, s, C.chebyshev_coeffs(kind, p, K), K)
        for a in (0.0, 0.5, 0.8):
            Z = GG.generalized_gp(g.row_ptr, g.col_idx, PR.one_hot(g.n, s), a, kind, p, K)[:, 0]
            np.testing.assert_allclose(Z, GG.single_source_generalized(g.row_ptr, g.col_idx, s, a, y),
                                       rtol=1e-12, atol=1e-15)
            if a == 0.0:
                np.testing.assert_allclose(Z, y, rtol=0, atol=0)


def pin_generalized_degree_zero_reading():
    """Degree-0 nodes (reading: outside the propagation) get Z = 0, and the
    other rows equal Def. 8 on the graph without them."""
    core = synth.erdos_renyi(30, 0.2, seed=4)
    assert np.all(core.degrees > 0)
    n = core.n + 2
    rows = np.repeat(np.arange(core.n), core.degrees)
    g = synth.from_edges(n, [(int(u), int(v)) for u, v in zip(rows, core.col_idx) if u < v], name="core+2")
    X = _features(n, 2, seed=9)
    Z = GG.generalized_gp(g.row_ptr, g.col_idx, X, 0.5, "hkpr", 2.0, 40)
    assert np.all(Z[core.n:] == 0.0)
    ref = D.generalized_definition(D.adjacency(core.row_ptr, core.col_idx), X[: core.n], 0.5, "hkpr", 2.0)
    assert np.max(np.abs(Z[: core.n] - ref)) < 1e-11


# ---------------------------------------------------------------- Sec. 4 (ChebyPush)


def pin_chebypush_worked_example():
    """Sec. 4.2 illustrative example (tests/golden/star_example.txt): star with
    centre v0, source v1, c = e_3 (f = T_3), eps_k = 1/3; the state after
    each iteration's pushes and the final r_cur = [5/3, 0, 0, 0].  Only the
    squared, inclusive threshold reproduces the printed steps."""
    gold = load_golden("star_example.txt")
    g = synth.star(3)
    c = np.array([0.0, 0.0, 0.0, 1.0])
    y, tr = PU.cheby_push(g.row_ptr, g.col_idx, 1, c, 3, np.full(4, 1.0 / 3.0), rule="squared_inclusive",
                          trace=True)
    assert [list(S) for S in tr["sets"]] == [[0], [2, 3]]
    np.testing.assert_allclose(tr["states"][0][0], gold["push_k1_r_cur_after"], atol=1e-15)
    np.testing.assert_allclose(tr["states"][0][1], gold["push_k1_r_new_after"], atol=1e-15)
    np.testing.assert_allclose(tr["states"][1][0], gold["push_k2_r_cur_after"], atol=1e-15)
    np.testing.assert_allclose(tr["states"][1][1], gold["push_k2_r_new_after"], atol=1e-15)
    np.testing.assert_allclose(tr["r_cur"], gold["chebypush_T3_threshold_1_3"], atol=1e-15)
    np.testing.assert_allclose(y, 0.0, atol=0)  # c_1 = c_2 = 0 and Alg. 4 never adds c_K


def _push_cases():
    for g in tiny_graphs()[:4]:
        s = _connected_node(g, 2)
        for kind, p, K in (("ppr", 0.2, 12), ("hkpr", 3.0, 10)):
            for eps_a in (3e-2, 1e-3):
                for rule in ("linear", "squared_inclusive"):
                    yield g, s, kind, p, K, eps_a, rule


def pin_push_form_is_subset_recurrence():
    """Lemma 6: after iteration k of the push form, r_cur = r^_{k+1} of Def. 7
    (formed from the same sets) and r_new = -r^_k|S_k + r^_k|(V - S_k)."""
    for g, s, kind, p, K, eps_a, rule in _push_cases():
        c = C.chebyshev_coeffs(kind, p, K)
        _, tr = PU.cheby_push(g.row_ptr, g.col_idx, s, c, K, eps_a, rule=rule, trace=True)
        r_hat = PU.subset_recurrence(g.row_ptr, g.col_idx, s, tr["sets"])
        for k, ((rc, rn), S) in enumerate(zip(tr["states"], tr["sets"]), start=1):
            on = np.zeros(g.n, dtype=bool)
            on[S] = True
            np.testing.assert_allclose(rn, r_hat[k + 1], atol=1e-14)
            np.testing.assert_allclose(rc, np.where(on, -r_hat[k], r_hat[k]), atol=1e-14)
        assert any(len(S) < np.count_nonzero(r_hat[k + 1]) for k, S in enumerate(tr["sets"])) or eps_a < 1e-2


def pin_subset_recurrence_deviation_identity():
    """Lemma 5: r_k = r^_k + 2 sum_{l=1}^{k-1} T_{k-l}(P) delta_l, with the
    exact T_j(P) formed on A~'s spectrum (Def. 6, Lemma 1 proof)."""
    for g, s, kind, p, K, eps_a, rule in _push_cases():
        if rule != "linear":
            continue
        A = D.adjacency(g.row_ptr, g.col_idx)
        c = C.chebyshev_coeffs(kind, p, K)
        _, tr = PU.cheby_push(g.row_ptr, g.col_idx, s, c, K, eps_a, trace=True)
        r_hat = PU.subset_recurrence(g.row_ptr, g.col_idx, s, tr["sets"])
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        r = PR.chebyshev_vectors(P, s, len(r_hat) - 1)
        Tm = [D.chebyshev_matrix_eigen(A, j) for j in range(len(r_hat))]
        delta = [None]
        for l, S in enumerate(tr["sets"], start=1):
            off = np.ones(g.n, dtype=bool)
            off[S] = False
            delta.append(np.where(off, r_hat[l], 0.0))
        for k in range(2, len(r_hat)):
            rhs = r_hat[k] + 2.0 * sum(Tm[k - l] @ delta[l] for l in range(1, k))
            np.testing.assert_allclose(rhs, r[k], atol=1e-11, err_msg=f"{g.name} {kind} k={k}")


def pin_chebypush_without_threshold():
    """eps_a = 0 pushes every node with a non-zero residual, so the subset
    recurrence is the exact one (Def. 7 with S_k = V) and Alg. 4 returns the
    first K terms c_0..c_{K-1} of Alg. 3 (its loop stops before c_K)."""
    for g in tiny_graphs():
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        s = _connected_node(g, 1)
        for kind, p in (("ppr", 0.2), ("hkpr", 5.0)):
            K = 9
            c = C.chebyshev_coeffs(kind, p, K)
            y = PU.cheby_push(g.row_ptr, g.col_idx, s, c, K, 0.0)
            ref = PR.cheby_power(P, s, c[:K], K - 1)
            np.testing.assert_allclose(y, ref, atol=1e-14, err_msg=g.name)


def pin_chebypush_degree_normalized_error():
    """Thm. 4: max_u |y(u) - y^(u)| / d_u < eps_a with K from Thm. 2's tail at
    eps_a / 2 (the theorem rests on the stability assumption of Sec. 4.3,
    which these graphs satisfy closely enough)."""
    for g in tiny_graphs():
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
        s = _connected_node(g, 2)
        for kind, p in (("ppr", 0.2), ("hkpr", 5.0)):
            exact = PR.ground_truth(P, s, kind, p)
            for eps_a in (1e-2, 1e-4, 1e-6):
                K = T.choose_K(kind, p, eps_a / 2, mode="tail")
                y = PU.cheby_push(g.row_ptr, g.col_idx, s, C.chebyshev_coeffs(kind, p, K), K, eps_a)
                err = PU.degree_normalized_error(exact, y, g.degrees)
                assert err < eps_a, (g.name, kind, eps_a, err)


def pin_chebypush_locality():
    """Lemma 7's locality bound, iteration by iteration: vol(S_k) eps_k is at
    most the selected residual mass, sum_{u in S_k} |r^_k(u)| with Alg. 4's
    test and sum_{u in S_k} r^_k(u)^2 with the squared one."""
    graphs = tiny_graphs() + [synth.chung_lu(20_000, 100_000, 2.5, seed=1)]
    for g in graphs:
        s = _connected_node(g, 2)
        for kind, p in (("ppr", 0.2), ("hkpr", 5.0)):
            for eps_a in (1e-2, 1e-4):
                K = T.choose_K(kind, p, eps_a / 2, mode="tail")
                c = C.chebyshev_coeffs(kind, p, K)
                for rule in ("linear", "squared_inclusive"):
                    _, tr = PU.cheby_push(g.row_ptr, g.col_idx, s, c, K, eps_a, rule=rule, trace=True)
                    r_hat = PU.subset_recurrence(g.row_ptr, g.col_idx, s, tr["sets"])
                    for k, S in enumerate(tr["sets"], start=1):
                        mass = np.abs(r_hat[k][S]) if rule == "linear" else r_hat[k][S] ** 2
                        assert g.degrees[S].sum() * tr["eps"][k] <= mass.sum() * (1 + 1e-12), (g.name, k, rule)


def pin_chebypush_candidates():
    """Locality of Alg. 4: every pushed node of iteration k is a neighbour of
    S_{k-1} or a node of S_{k-2} (with S_0 = {s}, N(S_0) = N(s), S_{-1}
    empty), because only S's sign flips and the pushes into N(S) change
    residuals and eps_k does not decrease with k."""
    graphs = tiny_graphs() + [synth.chung_lu(20_000, 100_000, 2.5, seed=1),
                              synth.chung_lu(30_000, 300_000, 2.1, seed=5)]
    for g in graphs:
        s = _connected_node(g, 2)
        for kind, p in (("ppr", 0.2), ("hkpr", 5.0), ("ppr", 0.05)):
            for eps_a in (1e-2, 1e-4, 1e-6):
                K = T.choose_K(kind, p, eps_a / 2, mode="tail")
                c = C.chebyshev_coeffs(kind, p, K)
                assert np.all(np.diff(PU.thresholds(c, K, eps_a)[1:K]) >= 0)  # entries 1..K-1 are used
                _, tr = PU.cheby_push(g.row_ptr, g.col_idx, s, c, K, eps_a, trace=True)
                sets = [np.array([s])] + tr["sets"]  # sets[k] = S_k
                for k in range(1, len(sets)):
                    prev = sets[k - 1]
                    nbr = np.zeros(g.n, dtype=bool)
                    for u in prev:
                        nbr[g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]] = True
                    cand = nbr.copy()
                    if k >= 2:
                        cand[sets[k - 2]] = True
                    assert np.all(cand[sets[k]]), (g.name, kind, eps_a, k)


# ---------------------------------------------------------------- Sec. 5.2 (ChebyPush + walks)


def pin_splitmix64_published_outputs():
    """The walk generator is SplitMix64: its first outputs from state 0 equal
    the published reference values (tests/golden/splitmix64_seed0.txt)."""
    import os
    from conftest import HERE

    with open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")) as fh:
        line = [ln for ln in fh if ln.startswith("outputs:")][0]
    want = [int(x.strip(), 16) for x in line.split(":", 1)[1].split(",")]
    assert [BI.splitmix64(0, i) for i in range(len(want))] == want


def _ppr_matrix(g, alpha):
    A = D.adjacency(g.row_ptr, g.col_idx)
    P = D.random_walk_matrix(A)
    return alpha * np.linalg.inv(np.eye(g.n) - (1.0 - alpha) * P)  # column v is pi_v


def pin_residual_invariant():
    """Lemma 9: after the push phase, pi_s = pi^ + sum_v r(v) pi_v, with the
    residual r = e_s - alpha^{-1} [I - (1 - alpha) P] pi^ and the exact pi_v."""
    for g in tiny_graphs()[:4]:
        s = _connected_node(g, 1)
        alpha = 0.2
        Pi = _ppr_matrix(g, alpha)
        for eps_a in (1e-2, 1e-4):
            K = 12
            pi_hat = PU.cheby_push(g.row_ptr, g.col_idx, s, C.ppr_chebyshev_coeffs(alpha, K), K, eps_a)
            r = BI.residual(g.row_ptr, g.col_idx, s, alpha, pi_hat)
            np.testing.assert_allclose(pi_hat + Pi @ r, Pi[:, s], atol=1e-12, err_msg=g.name)
            assert np.max(np.abs(r)) > 1e-6  # the push left mass to the walks


def pin_alpha_walk_end_distribution():
    """An alpha-random walk from v ends at u with probability pi_v(u) (the
    walk reading of Def. 3): 40,000 seeded walks against the exact vector,
    every node within 5 binomial standard deviations."""
    g = synth.barbell_with_tail(5, 4)
    alpha = 0.25
    Pi = _ppr_matrix(g, alpha)
    v = 3
    M = 40_000
    key = BI.splitmix64(123, v)
    ends = np.bincount([BI.walk_terminal(g.row_ptr, g.col_idx, key, j, v, alpha) for j in range(M)],
                       minlength=g.n)
    p = Pi[:, v]
    sd = np.sqrt(p * (1 - p) / M) + 1e-12
    assert np.all(np.abs(ends / M - p) <= 5 * sd + 1e-9), np.max(np.abs(ends / M - p) / sd)


def pin_push_rw_accuracy():
    """Alg. 5 end to end, with a threshold large enough that the walks carry
    most of the mass: |pi^(u) - pi_s(u)| < eps_r pi_s(u) wherever
    pi_s(u) > delta (the guarantee holds with high probability; seeded)."""
    g = synth.erdos_renyi(60, 0.12, seed=8)
    s = _connected_node(g, 2)
    alpha, eps_r = 0.2, 0.3
    delta = 1.0 / g.n
    Pi = _ppr_matrix(g, alpha)
    pi_hat, tr = BI.push_rw(g.row_ptr, g.col_idx, s, alpha, 4, eps_r, delta, seed=7, trace=True, r_max=1e-2)
    walked = float(np.sum(np.abs(tr["residual"])))
    assert walked > 0.5  # most of the mass went through the walks
    big = Pi[:, s] > delta
    rel = np.abs(pi_hat[big] - Pi[big, s]) / Pi[big, s]
    assert np.max(rel) < eps_r, np.max(rel)
    assert np.max(rel) > 1e-6  # not exact: the walks are sampled


ALL_PINS = [
    pin_star_example,
    pin_chebyshev_vectors_eigen,
    pin_mass,
    pin_cycle_closed_form,
    pin_complete_closed_form,
    pin_circulant_closed_forms,
    pin_ppr_closed_values,
    pin_coefficient_integrals,
    pin_hkpr_library,
    pin_coefficient_sums,
    pin_expansion_pointwise,
    pin_taylor_sums,
    pin_dense_definitions,
    pin_truncated_series_eigen,
    pin_pwmethod_exact_tail,
    pin_certified_bound_and_certificate,
    pin_convergence_rate,
    pin_generalized_definition,
    pin_clenshaw_truncated_series,
    pin_generalized_symmetric_half,
    pin_generalized_single_source,
    pin_generalized_degree_zero_reading,
    pin_chebypush_worked_example,
    pin_push_form_is_subset_recurrence,
    pin_subset_recurrence_deviation_identity,
    pin_chebypush_without_threshold,
    pin_chebypush_degree_normalized_error,
    pin_chebypush_locality,
    pin_chebypush_candidates,
    pin_splitmix64_published_outputs,
    pin_residual_invariant,
    pin_alpha_walk_end_distribution,
    pin_push_rw_accuracy,
]


def failing_pins(pins=None):
    """Names of the pins that raise AssertionError (or any error)."""
    bad = []
    for fn in pins or ALL_PINS:
        try:
            fn()
        except Exception:  # noqa: BLE001 - a planted mistake may break in any way
            bad.append(fn.__name__)
    return bad
