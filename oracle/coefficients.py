"""Expansion coefficients of the two GP functions (oracle, test-only).

Paper passages:
  Def. 3  SSPPR: Taylor coefficients zeta_k = alpha (1-alpha)^k,
          f(x) = alpha / (1 - (1-alpha) x).
  Def. 4  HKPR:  zeta_k = e^{-t} t^k / k!,  f(x) = e^{-t(1-x)}.
  Lemma 1 Chebyshev coefficients c_k = (2/pi) int f T_k / sqrt(1-x^2),
          c_0 with 1/pi.
  Lemma 2 SSPPR closed form: gamma = alpha / sqrt(2 alpha - alpha^2),
          beta = (1 - sqrt(2 alpha - alpha^2)) / (1 - alpha);
          c_0 = gamma, c_k = 2 gamma beta^k.
  Lemma 3 HKPR: c_0 = e^{-t} I_0(t), c_k = 2 e^{-t} I_k(t), with
          I_n(t) = (1/pi) int_0^pi e^{t cos th} cos(n th) dth.

The HKPR coefficients are computed from that integral definition by the
trapezoid rule in theta.  The integrand is smooth and 2 pi-periodic, so the
rule converges geometrically; e^{-t} is folded into the exponent
(e^{t (cos th - 1)}) so nothing overflows.
"""

from __future__ import annotations

import math

import numpy as np

PPR = "ppr"
HKPR = "hkpr"


def check_param(kind: str, param: float) -> None:
    if kind == PPR:
        if not (0.0 < param < 1.0):
            raise ValueError("SSPPR needs alpha in (0, 1) (Def. 3)")
    elif kind == HKPR:
        if not (param > 0.0):
            raise ValueError("HKPR needs t > 0 (Def. 4 states t > 1; the expansion holds for t > 0)")
    else:
        raise ValueError(f"unknown GP kind {kind!r}")


def gp_function(kind: str, param: float):
    """The scalar GP function f of Def. 3 / Def. 4 (vectorised)."""
    check_param(kind, param)
    if kind == PPR:
        a = param
        return lambda x: a / (1.0 - (1.0 - a) * np.asarray(x, dtype=np.float64))
    t = param
    return lambda x: np.exp(-t * (1.0 - np.asarray(x, dtype=np.float64)))


def taylor_coeffs(kind: str, param: float, N: int) -> np.ndarray:
    """zeta_0 .. zeta_{N-1} (Def. 3 / Def. 4)."""
    check_param(kind, param)
    k = np.arange(N, dtype=np.float64)
    if kind == PPR:
        a = param
        return a * (1.0 - a) ** k
    t = param
    # e^{-t} t^k / k! via logs (lgamma) to stay finite for large k.
    return np.exp(-t + k * math.log(t) - np.array([math.lgamma(x + 1.0) for x in k]))


def ppr_gamma_beta(alpha: float) -> tuple[float, float]:
    """gamma and beta of Lemma 2."""
    check_param(PPR, alpha)
    root = math.sqrt(2.0 * alpha - alpha * alpha)
    gamma = alpha / root
    beta = (1.0 - root) / (1.0 - alpha)
    return gamma, beta


def ppr_chebyshev_coeffs(alpha: float, K: int) -> np.ndarray:
    """c_0 .. c_K of Lemma 2."""
    gamma, beta = ppr_gamma_beta(alpha)
    c = np.empty(K + 1, dtype=np.float64)
    c[0] = gamma
    for k in range(1, K + 1):
        c[k] = 2.0 * gamma * beta**k
    return c


def scaled_bessel_I(t: float, nmax: int, panels: int | None = None) -> np.ndarray:
    """e^{-t} I_n(t), n = 0..nmax, from the integral in Lemma 3.

    (1/pi) int_0^pi g(th) dth with g(th) = e^{t (cos th - 1)} cos(n th),
    trapezoid rule with ``panels`` equal panels on [0, pi].
    """
    if panels is None:
        panels = 2 * (nmax + int(math.ceil(2.0 * t))) + 256
    th = np.linspace(0.0, math.pi, panels + 1)
    w = np.full(panels + 1, 1.0 / panels)
    w[0] = w[-1] = 0.5 / panels
    env = np.exp(t * (np.cos(th) - 1.0)) * w
    n = np.arange(nmax + 1, dtype=np.float64)[:, None]
    return np.cos(n * th[None, :]) @ env


def hkpr_chebyshev_coeffs(t: float, K: int) -> np.ndarray:
    """c_0 .. c_K of Lemma 3."""
    check_param(HKPR, t)
    i_scaled = scaled_bessel_I(t, K)
    c = 2.0 * i_scaled
    c[0] = i_scaled[0]
    return c


def chebyshev_coeffs(kind: str, param: float, K: int) -> np.ndarray:
    if kind == PPR:
        return ppr_chebyshev_coeffs(param, K)
    return hkpr_chebyshev_coeffs(param, K)
