"""Truncation steps (oracle, test-only).

Paper passages:
  Thm. 2   ChebyPower's error is governed by the coefficient tail
           sum_{k>K} |c_k|.
  Lemma 4  K = O((1/sqrt(alpha)) log 1/eps) for SSPPR and
           O(sqrt(t) log 1/eps) for HKPR; the experiments (Sec. 6.1, 6.2)
           use K = (1/sqrt(alpha)) log(1/eps) and sqrt(t) log(1/eps).
  Sec. 3.2 PwMethod needs N = O((1/alpha) log 1/eps) (SSPPR) and
           O(2t log 1/eps) (HKPR) for l1 error eps.

Reading used here (the paper's l2 argument leans on ||T_k(P)||_2 <= 1,
which only holds for regular graphs): since T_k(P) = D^{1/2} T_k(A~) D^{-1/2}
with ||T_k(A~)||_2 <= 1, Cauchy-Schwarz gives
  ||T_k(P) e_s||_1 <= sqrt(vol(G) / d_s),
so  ||y - y_K||_1 <= sqrt(vol / d_s) * tail(K).
"certified" mode picks the smallest K >= 1 with sqrt(vol/d_s) tail(K) <= tol;
"tail" mode is Thm. 2 as printed (multiplier 1); "paper" mode is the
experiments' formula with the natural logarithm.

Tails are summed term by term from the coefficient definitions (never as
1 - partial sum), far enough that the neglected remainder is below 1e-300.
"""

from __future__ import annotations

import math

import numpy as np

from .coefficients import HKPR, PPR, check_param, chebyshev_coeffs, taylor_coeffs

CERTIFIED = "certified"
TAIL = "tail"
PAPER = "paper"


def _coeff_horizon(kind: str, param: float) -> int:
    """A K beyond which every |c_k| is below 1e-300."""
    if kind == PPR:
        from .coefficients import ppr_gamma_beta

        _, beta = ppr_gamma_beta(param)
        return int(math.ceil(math.log(1e-300) / math.log(beta))) + 2
    # e^{-t} I_k(t) <= (t/2)^k / k!  (series bound); find where it drops below 1e-300
    k = 1
    while (k * math.log(param / 2.0) - math.lgamma(k + 1.0)) > math.log(1e-300) or k < 2 * param:
        k += 1
    return k + 2


def chebyshev_tails(kind: str, param: float, K_max: int) -> np.ndarray:
    """tail[K] = sum_{k > K} |c_k| for K = 0..K_max."""
    check_param(kind, param)
    H = max(_coeff_horizon(kind, param), K_max + 2)
    c = np.abs(chebyshev_coeffs(kind, param, H))
    # suffix sums, smallest terms first
    suffix = np.cumsum(c[::-1])[::-1]  # suffix[j] = sum_{k >= j}
    return np.array([suffix[K + 1] for K in range(K_max + 1)])


def certified_multiplier(vol: float, d_s: float) -> float:
    return math.sqrt(vol / d_s)


def choose_K(kind: str, param: float, tol: float, mode: str = CERTIFIED,
             vol: float = 1.0, d_s: float = 1.0, K_max: int = 10000) -> int:
    """Smallest K >= 1 whose tail bound meets ``tol`` (see module doc)."""
    if not (0.0 < tol < 1.0):
        raise ValueError("tolerance must be in (0, 1)")
    if mode == PAPER:
        if kind == PPR:
            return max(1, int(math.ceil(math.log(1.0 / tol) / math.sqrt(param))))
        return max(1, int(math.ceil(math.sqrt(param) * math.log(1.0 / tol))))
    L = certified_multiplier(vol, d_s) if mode == CERTIFIED else 1.0
    # beyond the horizon every tail is below 1e-300, so no larger K is needed
    tails = chebyshev_tails(kind, param, min(K_max, _coeff_horizon(kind, param)))
    for K in range(1, len(tails)):
        if tails[K] * L <= tol:
            return K
    raise ValueError("no K <= K_max meets the tolerance")


def taylor_tail(kind: str, param: float, N: int) -> float:
    """sum_{k >= N} zeta_k: the exact l1 error of PwMethod after N terms,
    because every P^k e_s is a probability vector and zeta_k >= 0."""
    check_param(kind, param)
    if kind == PPR:
        return (1.0 - param) ** N
    # sum Poisson(t) pmf from N upward until negligible
    terms = taylor_coeffs(kind, param, N + int(10 * param) + 400)
    return float(np.sum(terms[N:][::-1]))


def pwmethod_steps(kind: str, param: float, tol: float) -> int:
    """Smallest N with taylor_tail(N) <= tol."""
    N = 1
    while taylor_tail(kind, param, N) > tol:
        N += 1
    return N
