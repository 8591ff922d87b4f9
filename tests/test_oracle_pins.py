"""The oracle against what the paper and the mathematics fix (CPU only)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import pins
import synth
from oracle import coefficients as C
from oracle import errors as E
from oracle import propagation as PR
from oracle import truncation as T


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_chung_lu_20k_against_krylov_solve():
    """Chung-Lu n=20,000, avg degree 10, exponent 2.5, PPR alpha=0.2:
    ChebyPower at the certified K meets l1 <= 1e-8 against a Krylov (GMRES)
    solve of Def. 3's linear system, whose own l1 error is bounded by the
    fixed-point certificate; the certified PwMethod agrees to 1e-13."""
    g = synth.chung_lu(20_000, 100_000, 2.5, seed=1)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = int(synth.sources(g, 1, seed=1)[0])
    alpha = 0.2
    n = g.n
    M = (sp.identity(n, format="csc") - (1 - alpha) * P.tocsc())
    e = np.zeros(n)
    e[s] = 1.0
    x, info = spla.gmres(M, e, rtol=1e-15, atol=0.0, restart=200, maxiter=50)
    assert info == 0
    y_lu = alpha * x
    assert E.ppr_certificate(P, s, alpha, y_lu) <= 1e-13
    K = T.choose_K("ppr", alpha, 1e-8, mode="certified", vol=g.nnz, d_s=g.degrees[s])
    y = PR.cheby_power(P, s, C.ppr_chebyshev_coeffs(alpha, K), K)
    assert E.l1(y, y_lu) <= 1e-8
    y_pw = PR.ground_truth(P, s, "ppr", alpha)
    assert E.l1(y_pw, y_lu) <= 1e-13
    # the paper-tail rule is weaker than the certified one on irregular graphs
    assert T.choose_K("ppr", alpha, 1e-8, mode="tail") < K


def test_hkpr_two_algorithms_agree():
    """HKPR t=5 on a 20k-node power-law graph: ChebyPower (Alg. 3) at a
    tiny certified tolerance vs PwMethod (Alg. 1) with an exact 1e-15 tail
    vs scipy's expm_multiply of -t(I-P)."""
    g = synth.chung_lu(20_000, 170_000, 2.3, seed=4)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    s = int(synth.sources(g, 1, seed=9)[0])
    K = T.choose_K("hkpr", 5.0, 1e-12, mode="certified", vol=g.nnz, d_s=g.degrees[s])
    y = PR.cheby_power(P, s, C.hkpr_chebyshev_coeffs(5.0, K), K)
    y_pw = PR.ground_truth(P, s, "hkpr", 5.0)
    n = g.n
    e = np.zeros(n)
    e[s] = 1.0
    y_ex = spla.expm_multiply(-5.0 * (sp.identity(n, format="csr") - P), e)
    assert E.l1(y, y_pw) <= 1e-12
    assert E.l1(y_ex, y_pw) <= 1e-10


def test_k_rules_match_closed_forms():
    """K from the summed tail equals the K from Lemma 4's exact PPR tail
    2 gamma beta^{K+1} / (1 - beta), at many tolerances and alphas."""
    for alpha in (0.01, 0.1, 0.2, 0.5, 0.9):
        gm, b = C.ppr_gamma_beta(alpha)
        for tol in (1e-3, 1e-6, 1e-9, 1e-12):
            K = T.choose_K("ppr", alpha, tol, mode="tail")
            closed = lambda K: 2 * gm * b ** (K + 1) / (1 - b)
            assert closed(K) <= tol * (1 + 1e-9)
            assert K == 1 or closed(K - 1) > tol * (1 - 1e-9)


def test_k_paper_mode_values():
    """The experiments' K = (1/sqrt(alpha)) ln(1/eps) and sqrt(t) ln(1/eps)."""
    assert T.choose_K("ppr", 0.2, 1e-6, mode="paper") == 31
    assert T.choose_K("hkpr", 5.0, 1e-6, mode="paper") == 31


def test_invalid_parameters():
    with pytest.raises(ValueError):
        C.chebyshev_coeffs("ppr", 1.0, 3)
    with pytest.raises(ValueError):
        C.chebyshev_coeffs("hkpr", 0.0, 3)
    g = synth.star(3)
    P = PR.transition_matrix(g.row_ptr, g.col_idx)
    with pytest.raises(ValueError):
        PR.cheby_power(P, 1, [1.0], 0)


def test_error_measures_def5():
    y = np.array([0.5, 0.25, 0.25])
    yh = np.array([0.4, 0.3, 0.25])
    assert abs(E.l1(y, yh) - 0.15) < 1e-15
    assert abs(E.l2(y, yh) - np.sqrt(0.01 + 0.0025)) < 1e-15
    assert abs(E.degree_normalized(y, yh, [2, 1, 1]) - 0.05) < 1e-15
