"""GP vectors by iteration on the random-walk matrix (oracle, test-only).

Paper passages:
  Sec. 2.1   P = A D^{-1} on an undirected graph; e_s the one-hot vector.
  Eq. (1)    y = f(P) e_s.
  Eq. (6)    r_0 = e_s, r_1 = P e_s, r_{k+1} = 2 P r_k - r_{k-1}, so that
             r_k = T_k(P) e_s.
  Alg. 3     ChebyPower: y^ = c_0 e_s, r_0, r_1 as above; while k < K:
             y^ += c_k r_k, r_{k+1} = 2 P r_k - r_{k-1}; finally
             y^ += c_K r_K.
  Alg. 1     PwMethod: y^ = 0, r_0 = e_s; while k < N: y^ += zeta_k r_k,
             r_{k+1} = P r_k.

P is formed as a scipy CSR matrix with entry 1/d_u at (v, u) for every arc
u -> v; the sparse matrix-vector product is the only library primitive.
Nodes with no edge have no column entries (their 1/d_u is never needed,
because nothing reaches them).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def transition_matrix(row_ptr: np.ndarray, col_idx: np.ndarray) -> sp.csr_matrix:
    """P = A D^{-1}.  Row v of the symmetric CSR lists N(v); entry (v, u)
    of P is A[v, u] / d_u."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    d = np.diff(row_ptr).astype(np.float64)
    inv_d = np.zeros(n, dtype=np.float64)
    inv_d[d > 0] = 1.0 / d[d > 0]
    data = inv_d[col_idx]
    return sp.csr_matrix((data, col_idx, row_ptr), shape=(n, n))


def one_hot(n: int, s: int) -> np.ndarray:
    e = np.zeros(n, dtype=np.float64)
    e[s] = 1.0
    return e


def _chebyshev_step(P, r_k: np.ndarray, r_km1: np.ndarray) -> np.ndarray:
    """r_{k+1} = 2 P r_k - r_{k-1}  (Eq. 6)."""
    return 2.0 * (P @ r_k) - r_km1


def chebyshev_vectors(P, s: int, K: int) -> list[np.ndarray]:
    """[T_0(P) e_s, ..., T_K(P) e_s] by the recurrence of Eq. (6)."""
    n = P.shape[0]
    r = [one_hot(n, s)]
    if K >= 1:
        r.append(P @ r[0])
    for k in range(1, K):
        r.append(_chebyshev_step(P, r[k], r[k - 1]))
    return r


def cheby_power(P, s: int, c: np.ndarray, K: int, stats: bool = False):
    """Algorithm 3 (ChebyPower).  ``c`` holds c_0..c_K; K >= 1.

    With ``stats``, also returns per-step lists of sum_u r_k(u) and
    ||r_k||_1 for k = 0..K.
    """
    if K < 1:
        raise ValueError("ChebyPower needs K >= 1 (with K = 0 its last line would add c_0 e_s twice)")
    c = np.asarray(c, dtype=np.float64)
    if c.shape[0] < K + 1:
        raise ValueError("need c_0..c_K")
    n = P.shape[0]
    e_s = one_hot(n, s)
    y = c[0] * e_s
    r_prev = e_s
    r_cur = P @ e_s
    sums, norms = [r_prev.sum(), r_cur.sum()], [np.abs(r_prev).sum(), np.abs(r_cur).sum()]
    k = 1
    while k < K:
        y = y + c[k] * r_cur
        r_next = _chebyshev_step(P, r_cur, r_prev)
        r_prev, r_cur = r_cur, r_next
        if stats:
            sums.append(r_cur.sum())
            norms.append(np.abs(r_cur).sum())
        k += 1
    y = y + c[K] * r_cur
    if stats:
        return y, {"sum_r": np.array(sums), "l1_r": np.array(norms)}
    return y


def power_method(P, s: int, zeta: np.ndarray, N: int) -> np.ndarray:
    """Algorithm 1 (PwMethod).  ``zeta`` holds zeta_0..zeta_{N-1}."""
    zeta = np.asarray(zeta, dtype=np.float64)
    n = P.shape[0]
    y = np.zeros(n, dtype=np.float64)
    r = one_hot(n, s)
    k = 0
    while k < N:
        y = y + zeta[k] * r
        r = P @ r
        k += 1
    return y


def ground_truth(P, s: int, kind: str, param: float, tol: float = 1e-15) -> np.ndarray:
    """f(P) e_s to l1 error ``tol`` plus FP64 rounding: PwMethod with N
    from the exact Taylor tail."""
    from .coefficients import taylor_coeffs
    from .truncation import pwmethod_steps

    N = pwmethod_steps(kind, param, tol)
    return power_method(P, s, taylor_coeffs(kind, param, N), N)


def cheby_power_query(row_ptr, col_idx, s: int, kind: str, param: float, K: int,
                      P=None) -> np.ndarray:
    """Convenience: coefficients of Lemma 2 / 3 and Algorithm 3 on (G, s)."""
    from .coefficients import chebyshev_coeffs

    if P is None:
        P = transition_matrix(row_ptr, col_idx)
    return cheby_power(P, s, chebyshev_coeffs(kind, param, K), K)
