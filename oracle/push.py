"""ChebyPush and the subset Chebyshev recurrence (oracle, test-only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages (Sec. 4):
  Def. 7    subset Chebyshev recurrence: r^_0 = e_s, r^_1 = P e_s,
            r^_{k+1} = 2 P (r^_k|S_k) - r^_{k-1}|S_{k-1} + r^_{k-1}|(V - S_{k-1}).
  Sec. 4.2  the push form of that recurrence: r_cur = P e_s, r_new = -e_s;
            per iteration k: r_new += 2 P (r_cur|S_k), r_cur|S_k = -r_cur|S_k,
            then swap the two vectors (Lemma 6: r_cur is r^_{k+1} afterwards).
  Alg. 4    ChebyPush: y^ = c_0 e_s; for k = 1 .. K-1 the threshold
            eps_k = eps_a / (4 K sum_{l=k}^{K} |c_l|), S_k the nodes whose
            r_cur passes it; each u in S_k adds c_k r_cur(u) to y^(u), gives
            2 r_cur(u) / d_u to every neighbour in r_new and flips its sign.
  Lemma 5   r_k = r^_k + 2 sum_{l=1}^{k-1} T_{k-l}(P) delta_l with the
            deviations delta_l = r^_l|(V - S_l).
  Thm. 4    degree-normalised error of y^ below eps_a (under the stability
            assumption of Sec. 4.3).

Reading of the threshold (the paper is inconsistent): Alg. 4 tests
|r_cur(u)| > eps_k d_u, which is what Thm. 4's error argument needs; the
prose and the Lemma 7 proof write |r_cur(u)|^2 > eps_k d_u; the worked
example of Sec. 4.2 (eps_k = 1/3) is reproduced only by |r_cur(u)|^2 >=
eps_k d_u.  rule="linear" (the default, the GPU's rule) is Alg. 4's test;
rule="squared_inclusive" is the one the worked example follows.
"""

from __future__ import annotations

import numpy as np

from . import propagation as PR


def thresholds(c: np.ndarray, K: int, eps_a: float) -> np.ndarray:
    """eps_k for k = 0..K (entries 1..K-1 are used), Alg. 4."""
    c = np.abs(np.asarray(c, dtype=np.float64)[: K + 1])
    eps = np.zeros(K + 1)
    for k in range(1, K):
        eps[k] = eps_a / (4.0 * K * float(np.sum(c[k:K + 1])))
    return eps


def selected(r: np.ndarray, d: np.ndarray, eps: float, rule: str = "linear") -> np.ndarray:
    """Boolean mask of S_k for the vector r (degree-0 nodes never qualify)."""
    if rule == "linear":
        m = np.abs(r) > eps * d
    elif rule == "squared_inclusive":
        m = r * r >= eps * d
    else:
        raise ValueError(rule)
    return m & (d > 0) & (r != 0.0)


def cheby_push(row_ptr, col_idx, s: int, c: np.ndarray, K: int, eps, rule: str = "linear",
               trace: bool = False):
    """Alg. 4.  ``eps`` is eps_a (a float, thresholds from Alg. 4) or an array
    of eps_k indexed by k.  Returns y^ and, with ``trace``, a dict holding the
    per-iteration sets and the (r_cur, r_new) pair after each iteration's
    pushes and before the swap."""
    if K < 1:
        raise ValueError("K >= 1")
    P = PR.transition_matrix(row_ptr, col_idx)
    d = np.diff(np.asarray(row_ptr, dtype=np.int64)).astype(np.float64)
    n = d.shape[0]
    c = np.asarray(c, dtype=np.float64)
    eps_k = thresholds(c, K, eps) if np.isscalar(eps) else np.asarray(eps, dtype=np.float64)
    y = c[0] * PR.one_hot(n, s)
    r_cur = P @ PR.one_hot(n, s)
    r_new = -PR.one_hot(n, s)
    sets, states = [], []
    margin = np.inf  # smallest relative distance of a residual to its threshold (diagnostic)
    k = 1
    while k < K:
        S = selected(r_cur, d, eps_k[k], rule)
        if trace and eps_k[k] > 0:
            live = (r_cur != 0.0) & (d > 0)
            if np.any(live):
                t = eps_k[k] * d[live]
                margin = min(margin, float(np.min(np.abs(np.abs(r_cur[live]) - t) / t)))
        y = y + c[k] * np.where(S, r_cur, 0.0)
        r_new = r_new + 2.0 * (P @ np.where(S, r_cur, 0.0))
        r_cur = np.where(S, -r_cur, r_cur)
        if trace:
            sets.append(np.flatnonzero(S))
            states.append((r_cur.copy(), r_new.copy()))
        r_cur, r_new = r_new, r_cur
        k += 1
    if trace:
        return y, {"sets": sets, "states": states, "r_cur": r_cur, "eps": eps_k, "margin": margin}
    return y


def subset_recurrence(row_ptr, col_idx, s: int, sets) -> list[np.ndarray]:
    """Def. 7 written out for given node sets S_1, S_2, ... (index arrays);
    returns [r^_0, r^_1, ..., r^_{len(sets)+1}]."""
    P = PR.transition_matrix(row_ptr, col_idx)
    n = P.shape[0]
    r = [PR.one_hot(n, s), P @ PR.one_hot(n, s)]
    masks = [np.zeros(n, dtype=bool)]  # S_0 is never used with a weight (r^_{-1} does not exist)
    for S in sets:
        m = np.zeros(n, dtype=bool)
        m[np.asarray(S, dtype=np.int64)] = True
        masks.append(m)
    for k in range(1, len(sets) + 1):
        on = masks[k]
        prev_on = masks[k - 1] if k - 1 >= 1 else np.ones(n, dtype=bool)
        term = 2.0 * (P @ np.where(on, r[k], 0.0))
        term = term - np.where(prev_on, r[k - 1], 0.0) + np.where(prev_on, 0.0, r[k - 1])
        r.append(term)
    return r


def degree_normalized_error(y: np.ndarray, y_hat: np.ndarray, degrees) -> float:
    """max_u |y(u) - y^(u)| / d_u over nodes with edges (Thm. 4's measure)."""
    d = np.asarray(degrees, dtype=np.float64)
    live = d > 0
    return float(np.max(np.abs(y[live] - y_hat[live]) / d[live])) if np.any(live) else 0.0
