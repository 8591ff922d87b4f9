"""Error measures (oracle, test-only).

Paper passages:
  Def. 5   l1 error, l2 error and degree-normalized error
           max_u |y(u) - y^(u)| / d_u.
  Def. 3   pi_s is the fixed point of pi = alpha e_s + (1-alpha) P pi.
           Because ||P||_1 = 1, ||(I - (1-alpha) P)^{-1}||_1 = 1/alpha, so
           ||pi_s - pi^||_1 <= ||alpha e_s + (1-alpha) P pi^ - pi^||_1 / alpha,
           an a-posteriori bound that needs no reference vector.
"""

from __future__ import annotations

import numpy as np


def l1(y, y_hat) -> float:
    return float(np.sum(np.abs(np.asarray(y, np.float64) - np.asarray(y_hat, np.float64))))


def l2(y, y_hat) -> float:
    return float(np.sqrt(np.sum((np.asarray(y, np.float64) - np.asarray(y_hat, np.float64)) ** 2)))


def max_abs(y, y_hat) -> float:
    return float(np.max(np.abs(np.asarray(y, np.float64) - np.asarray(y_hat, np.float64))))


def degree_normalized(y, y_hat, degrees) -> float:
    d = np.asarray(degrees, np.float64)
    diff = np.abs(np.asarray(y, np.float64) - np.asarray(y_hat, np.float64))
    ok = d > 0
    return float(np.max(diff[ok] / d[ok])) if np.any(ok) else 0.0


def ppr_certificate(P, s: int, alpha: float, pi_hat) -> float:
    """Upper bound on ||pi_s - pi^||_1 from the fixed-point residual."""
    pi_hat = np.asarray(pi_hat, np.float64)
    res = (1.0 - alpha) * (P @ pi_hat) - pi_hat
    res[s] += alpha
    return float(np.sum(np.abs(res)) / alpha)
