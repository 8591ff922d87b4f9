"""Host-side parts of the HIP library, runnable without a GPU: the shared
library loads and exports every symbol its header declares; coefficients
and truncation steps agree with the oracle (CPU only)."""

import os
import re

import numpy as np
import pytest
import scipy.special as ss

from oracle import coefficients as C
from oracle import truncation as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cp():
    from paper_2412_10789_amd import chebyprop

    chebyprop.load()
    return chebyprop


def _declared():
    with open(os.path.join(ROOT, "include", "chebyprop.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:cp_status|size_t|const char\*|int32_t)\s+(cp_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(cp):
    names = _declared()
    assert len(names) >= 13
    lib = cp.load()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(cp.EXPORTED) == names


def test_status_strings(cp):
    for code in range(0, -13, -1):
        assert cp.cp_status_str(code) not in ("", "unknown status")
    assert cp.cp_status_str(-99) == "unknown status"
    assert "gfx950" in cp.cp_version()


@pytest.mark.parametrize("alpha", [0.01, 0.1, 0.2, 0.5, 0.9])
def test_ppr_coefficients_match_oracle(cp, alpha):
    np.testing.assert_allclose(cp.cp_coeffs(cp.CP_PPR, alpha, 60), C.ppr_chebyshev_coeffs(alpha, 60),
                               rtol=1e-13, atol=0)


@pytest.mark.parametrize("t", [0.3, 1.0, 5.0, 10.0, 40.0])
def test_hkpr_coefficients_match_oracle_and_library(cp, t):
    c = cp.cp_coeffs(cp.CP_HKPR, t, 80)
    np.testing.assert_allclose(c, C.hkpr_chebyshev_coeffs(t, 80), atol=2e-15, rtol=1e-12)
    ref = np.r_[ss.ive(0, t), 2 * ss.ive(np.arange(1, 81), t)]
    big = ref > 1e-290
    np.testing.assert_allclose(c[big], ref[big], rtol=1e-12)


@pytest.mark.parametrize("mode,omode", [(0, "certified"), (1, "tail"), (2, "paper")])
def test_truncation_step_matches_oracle(cp, mode, omode):
    cases = [("ppr", 0.2), ("ppr", 0.1), ("ppr", 0.02), ("hkpr", 3.0), ("hkpr", 5.0), ("hkpr", 10.0)]
    for kind, p in cases:
        for tol in (1e-4, 1e-6, 1e-7, 1e-9):
            for vol, ds in ((7e7, 8.0), (2e5, 1.0), (1e3, 900.0)):
                K, tail = cp.cp_choose_K(cp.KINDS[kind], p, tol, mode, 0, vol, ds)
                Ko = T.choose_K(kind, p, tol, mode=omode, vol=vol, d_s=ds)
                # the oracle's HKPR tails come from quadrature with ~1e-16 absolute
                # noise per coefficient (~1e-13 summed); the library's from
                # Miller's recurrence (relative accuracy).  K may differ only
                # where the tail sits within that noise of the threshold.
                noise = 1e-13 if kind == "hkpr" else 1e-16
                L = np.sqrt(vol / ds) if omode == "certified" else 1.0
                if K != Ko:
                    tails = T.chebyshev_tails(kind, p, max(K, Ko) + 1)
                    assert abs(tails[min(K, Ko)] - tol / L) <= 1e-9 * tol / L + noise, (kind, p, tol, K, Ko)
                if omode != "paper":
                    assert abs(tail - T.chebyshev_tails(kind, p, K + 1)[K]) <= 1e-12 * tail + noise


def test_argument_errors_without_gpu(cp):
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_coeffs(cp.CP_PPR, 1.0, 3)
    assert ei.value.status == cp.CP_EINVAL
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_choose_K(cp.CP_PPR, 0.2, 1e-6, cp.CP_K_FIXED, 0)
    assert ei.value.status == cp.CP_EINVAL
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_choose_K(cp.CP_PPR, 0.2, 1e-6, cp.CP_K_FIXED, 5000, K_max=100)
    assert ei.value.status == cp.CP_EKMAX
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_choose_K(cp.CP_HKPR, 5.0, 1.5)
    assert ei.value.status == cp.CP_EINVAL
    assert cp.cp_workspace_bytes(0, 1, cp.CP_F32) == 0
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_graph_create(0, 0, 0, 0, 0, 0)
    assert ei.value.status == cp.CP_EINVAL


@pytest.mark.parametrize("kind,param", [("ppr", 0.01), ("ppr", 0.2), ("ppr", 0.9), ("hkpr", 0.5), ("hkpr", 5.0),
                                        ("hkpr", 40.0)])
def test_taylor_weights_match_oracle(cp, kind, param):
    """Def. 3 / Def. 4 weights of PwMethod (Alg. 1)."""
    z = cp.cp_taylor(cp.KINDS[kind], param, 300)
    ref = C.taylor_coeffs(kind, param, 300)
    big = ref > 1e-290
    np.testing.assert_allclose(z[big], ref[big], rtol=1e-12)
    assert np.all(z[~big] < 1e-280)
    assert cp.cp_taylor(cp.KINDS[kind], param, 0).size == 0


def test_pwmethod_terms_match_oracle(cp):
    for kind, p in [("ppr", 0.2), ("ppr", 0.1), ("ppr", 0.01), ("hkpr", 0.3), ("hkpr", 3.0), ("hkpr", 10.0),
                    ("hkpr", 60.0)]:
        for tol in (0.5, 1e-4, 1e-6, 1e-9, 1e-12):
            for mode in (cp.CP_K_CERTIFIED, cp.CP_K_TAIL, cp.CP_K_PAPER):
                N, tail = cp.cp_choose_N(cp.KINDS[kind], p, tol, mode)
                No = T.pwmethod_steps(kind, p, tol)
                if N != No:  # only where the tail sits on the threshold to rounding
                    assert abs(T.taylor_tail(kind, p, min(N, No)) - tol) <= 1e-12 * tol, (kind, p, tol, N, No)
                assert abs(tail - T.taylor_tail(kind, p, N)) <= 1e-12 * tail + 1e-300
                assert tail <= tol and (N == 1 or T.taylor_tail(kind, p, N - 1) > tol * (1 - 1e-12))


def test_pwmethod_term_errors(cp):
    N, tail = cp.cp_choose_N(cp.CP_PPR, 0.2, 0.0, cp.CP_K_FIXED, 7)
    assert N == 7 and abs(tail - 0.8**7) < 1e-15
    for args, status in [((cp.CP_PPR, 0.2, 1e-6, cp.CP_K_FIXED, 0), cp.CP_EINVAL),
                         ((cp.CP_PPR, 0.2, 1e-6, cp.CP_K_FIXED, 500, 100), cp.CP_EKMAX),
                         ((cp.CP_PPR, 0.001, 1e-9, cp.CP_K_CERTIFIED, 0, 1000), cp.CP_EKMAX),
                         ((cp.CP_HKPR, 5000.0, 1e-6, cp.CP_K_CERTIFIED, 0, 4096), cp.CP_EKMAX),
                         ((cp.CP_HKPR, 5.0, 1.0), cp.CP_EINVAL),
                         ((cp.CP_PPR, 1.0, 1e-6), cp.CP_EINVAL)]:
        with pytest.raises(cp.ChebypropError) as ei:
            cp.cp_choose_N(*args)
        assert ei.value.status == status, args
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_taylor(cp.CP_HKPR, -1.0, 3)
    assert ei.value.status == cp.CP_EINVAL


@pytest.mark.parametrize("t", [100.0, 500.0, 700.0])
def test_hkpr_coefficients_large_t(cp, t):
    """Large heat-kernel times: Miller's recurrence keeps every coefficient
    finite and matches the scaled Bessel functions; the coefficients sum to
    f(1) = 1 and alternate to f(-1) = e^{-2t} (Lemma 3's series at
    lambda = +-1)."""
    K = int(t + 40 * np.sqrt(t) + 50)
    c = cp.cp_coeffs(cp.CP_HKPR, t, K)
    assert np.all(np.isfinite(c)) and np.all(c >= 0)
    ref = np.r_[ss.ive(0, t), 2 * ss.ive(np.arange(1, K + 1), t)]
    big = ref > 1e-250
    np.testing.assert_allclose(c[big], ref[big], rtol=1e-10)
    assert abs(c.sum() - 1.0) <= 1e-12
    alt = np.sum(c * (-1.0) ** np.arange(K + 1))
    assert abs(alt - np.exp(-2 * t)) <= 1e-12


@pytest.mark.parametrize("alpha", [1e-4, 0.999])
def test_ppr_coefficients_extreme_alpha(cp, alpha):
    """Near the ends of (0, 1): the series sums to f(1) = 1 and alternates to
    f(-1) = alpha / (2 - alpha) (Def. 3 at lambda = +-1), up to its tail."""
    K = 4000 if alpha < 0.01 else 40
    c = cp.cp_coeffs(cp.CP_PPR, alpha, K)
    assert np.all(np.isfinite(c))
    tail = T.chebyshev_tails("ppr", alpha, K + 1)[K]
    assert abs(c.sum() - 1.0) <= tail + 1e-12
    alt = np.sum(c * (-1.0) ** np.arange(K + 1))
    assert abs(alt - alpha / (2 - alpha)) <= tail + 1e-12


def test_truncation_step_limits(cp):
    """A K beyond the library's cap gives CP_EKMAX rather than a wrong K."""
    K, _ = cp.cp_choose_K(cp.CP_PPR, 0.2, 1e-9, 1, 0, 1e6, 1.0)
    assert 1 <= K < 200
    with pytest.raises(cp.ChebypropError) as ei:
        cp.cp_choose_K(cp.CP_PPR, 1e-7, 1e-14, 0, 0, 1e9, 1.0)
    assert ei.value.status == cp.CP_EKMAX
