"""Generalized graph propagation (oracle, test-only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages:
  Def. 8   Z = f(D^{-a} A D^{-b}) X for a feature matrix X (n x k), a + b = 1.
  Thm. 5   z = f(D^{-a} A D^{-b}) x = D^{-a} y with y = f(P) D^{a} x: the
           walk-matrix series applied to the rescaled start vector D^{a} x.
  Single-source form (appendix on generalized propagation): for x = e_s,
           z = d_s^{a} D^{-a} f(P) e_s.
  Alg. 3 / Alg. 1 with a general start vector: r_0 = x, r_1 = P x, then the
           recurrence of Eq. (6) (or r_{k+1} = P r_k); the estimate sums
           c_k r_k (zeta_k r_k).
  Clenshaw's backward recurrence (Clenshaw 1955, among the stability
           references of the related-work section) evaluates the same
           truncated series sum_{k<=K} c_k T_k(P) x without an estimate
           vector: b_{K+1} = b_{K+2} = 0, b_k = c_k x + 2 P b_{k+1} - b_{k+2}
           for k = K, ..., 1, and the sum is c_0 x + P b_1 - b_2.  It follows
           from T_{k+1} = 2 P T_k - T_{k-1} by summation by parts; the paper
           itself uses only the forward form.

Reading (not covered by the paper): a node of degree 0 is outside the
propagation.  D^{a} and D^{-a} are taken as 0 there, so its row of X is
ignored and its row of Z is 0.
"""

from __future__ import annotations

import numpy as np

from . import coefficients as C
from . import propagation as PR


def cheby_power_vector(P, x: np.ndarray, c: np.ndarray, K: int) -> np.ndarray:
    """Alg. 3 started from a dense vector x: y^ = sum_{k<=K} c_k T_k(P) x."""
    if K < 1:
        raise ValueError("ChebyPower needs K >= 1")
    c = np.asarray(c, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = c[0] * x
    r_prev = x
    r_cur = P @ x
    k = 1
    while k < K:
        y = y + c[k] * r_cur
        r_next = PR._chebyshev_step(P, r_cur, r_prev)
        r_prev, r_cur = r_cur, r_next
        k += 1
    return y + c[K] * r_cur


def _clenshaw_step(P, x: np.ndarray, b_next: np.ndarray, b_next2: np.ndarray, c_k: float) -> np.ndarray:
    """b_k = c_k x + 2 P b_{k+1} - b_{k+2}."""
    return c_k * x + 2.0 * (P @ b_next) - b_next2


def clenshaw_vector(P, x: np.ndarray, c: np.ndarray, K: int) -> np.ndarray:
    """Clenshaw's backward evaluation of sum_{k<=K} c_k T_k(P) x."""
    if K < 1:
        raise ValueError("the series needs K >= 1")
    c = np.asarray(c, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    b1 = np.zeros_like(x)  # b_{k+1}
    b2 = np.zeros_like(x)  # b_{k+2}
    for k in range(K, 0, -1):
        b1, b2 = _clenshaw_step(P, x, b1, b2, c[k]), b1
    return c[0] * x + P @ b1 - b2


def power_method_vector(P, x: np.ndarray, zeta: np.ndarray, N: int) -> np.ndarray:
    """Alg. 1 started from a dense vector x: y^ = sum_{k<N} zeta_k P^k x."""
    zeta = np.asarray(zeta, dtype=np.float64)
    y = np.zeros_like(np.asarray(x, dtype=np.float64))
    r = np.asarray(x, dtype=np.float64)
    for k in range(N):
        y = y + zeta[k] * r
        r = P @ r
    return y


def degree_powers(degrees: np.ndarray, a: float) -> tuple[np.ndarray, np.ndarray]:
    """(D^{a}, D^{-a}) as vectors, 0 at degree-0 nodes (see the reading above)."""
    d = np.asarray(degrees, dtype=np.float64)
    live = d > 0
    da = np.zeros_like(d)
    dma = np.zeros_like(d)
    da[live] = d[live] ** a
    dma[live] = d[live] ** (-a)
    return da, dma


def generalized_gp(row_ptr, col_idx, X: np.ndarray, a: float, kind: str, param: float, K: int,
                   method: str = "cheby") -> np.ndarray:
    """Def. 8 through Thm. 5, one column at a time: Z = D^{-a} y^ with y^ the
    K-term ChebyPower series (method="cheby"; "clenshaw": the same series by
    Clenshaw's backward recurrence; "power": the K-term PwMethod sum)
    applied to D^{a} x_j."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    P = PR.transition_matrix(row_ptr, col_idx)
    da, dma = degree_powers(np.diff(np.asarray(row_ptr, dtype=np.int64)), a)
    Z = np.zeros_like(X)
    for j in range(X.shape[1]):
        x = da * X[:, j]
        if method == "cheby":
            y = cheby_power_vector(P, x, C.chebyshev_coeffs(kind, param, K), K)
        elif method == "clenshaw":
            y = clenshaw_vector(P, x, C.chebyshev_coeffs(kind, param, K), K)
        else:
            y = power_method_vector(P, x, C.taylor_coeffs(kind, param, K), K)
        Z[:, j] = dma * y
    return Z


def single_source_generalized(row_ptr, col_idx, s: int, a: float, y: np.ndarray) -> np.ndarray:
    """The single-source form: z = d_s^{a} D^{-a} y for y = f(P) e_s."""
    d = np.diff(np.asarray(row_ptr, dtype=np.int64))
    _, dma = degree_powers(d, a)
    return float(d[s]) ** a * dma * np.asarray(y, dtype=np.float64)
