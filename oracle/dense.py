"""Dense definitions for tiny graphs (oracle, test-only; n up to a few
hundred).

Paper passages:
  Def. 3   pi_s = alpha (I - (1-alpha) P)^{-1} e_s            (dense solve)
  Def. 4   rho_s = e^{-t (I - P)} e_s                          (expm)
  Lemma 1 (proof)  P = D^{1/2} A~ D^{-1/2},  A~ = D^{-1/2} A D^{-1/2}
           symmetric with eigen-decomposition U Lambda U^T, hence
           f(P) = D^{1/2} U f(Lambda) U^T D^{-1/2}               (eigen route)
  Def. 6   T_k(x) = cos(k arccos x) on [-1, 1]; used on the eigenvalues to
           form T_k(P) without the recurrence.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def adjacency(row_ptr, col_idx) -> np.ndarray:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    A = np.zeros((n, n), dtype=np.float64)
    for v in range(n):
        A[v, np.asarray(col_idx[row_ptr[v]:row_ptr[v + 1]], dtype=np.int64)] = 1.0
    return A


def random_walk_matrix(A: np.ndarray) -> np.ndarray:
    """P = A D^{-1} (column u scaled by 1/d_u)."""
    d = A.sum(axis=0)
    if np.any(d == 0):
        raise ValueError("dense routes need a graph without isolated nodes")
    return A / d[None, :]


def ppr_solve(A: np.ndarray, s: int, alpha: float) -> np.ndarray:
    n = A.shape[0]
    P = random_walk_matrix(A)
    e = np.zeros(n)
    e[s] = 1.0
    return alpha * np.linalg.solve(np.eye(n) - (1.0 - alpha) * P, e)


def hkpr_expm(A: np.ndarray, s: int, t: float) -> np.ndarray:
    n = A.shape[0]
    P = random_walk_matrix(A)
    return sla.expm(-t * (np.eye(n) - P))[:, s]


def _sym_eig(A: np.ndarray):
    d = A.sum(axis=0)
    if np.any(d == 0):
        raise ValueError("dense routes need a graph without isolated nodes")
    dh = np.sqrt(d)
    At = A / dh[:, None] / dh[None, :]
    lam, U = np.linalg.eigh(At)
    return np.clip(lam, -1.0, 1.0), U, dh


def matrix_function_eigen(A: np.ndarray, s: int, f) -> np.ndarray:
    """f(P) e_s = D^{1/2} U f(Lambda) U^T D^{-1/2} e_s."""
    lam, U, dh = _sym_eig(A)
    x = np.zeros(A.shape[0])
    x[s] = 1.0 / dh[s]
    return dh * (U @ (f(lam) * (U.T @ x)))


def chebyshev_matrix_eigen(A: np.ndarray, k: int) -> np.ndarray:
    """T_k(P) with T_k(lambda) = cos(k arccos lambda) on A~'s spectrum."""
    lam, U, dh = _sym_eig(A)
    Tk = np.cos(k * np.arccos(lam))
    return (dh[:, None] * (U * Tk[None, :]) @ U.T) / dh[None, :]


def generalized_definition(A: np.ndarray, X: np.ndarray, a: float, kind: str, param: float) -> np.ndarray:
    """Def. 8 written out: M = D^{-a} A D^{-(1-a)}, then f(M) X with f from
    Def. 3 (alpha (I - (1 - alpha) M)^{-1}) or Def. 4 (e^{-t (I - M)})."""
    n = A.shape[0]
    d = A.sum(axis=0)
    if np.any(d == 0):
        raise ValueError("dense routes need a graph without isolated nodes")
    M = (d ** (-a))[:, None] * A * (d ** (a - 1.0))[None, :]
    X = np.asarray(X, dtype=np.float64)
    if kind == "ppr":
        return param * np.linalg.solve(np.eye(n) - (1.0 - param) * M, X)
    return sla.expm(-param * (np.eye(n) - M)) @ X
