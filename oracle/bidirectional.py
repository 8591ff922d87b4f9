"""ChebyPush + random walks (Alg. 5, Sec. 5.2) for SSPPR (oracle, test-only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages (Sec. 5.2):
  W      = 2 (2 eps_r / 3 + 2) log n / (eps_r^2 delta)   (log read as natural)
  r_max  = sqrt(alpha) / W
  pi^    = ChebyPush(G, f = alpha (1 - (1 - alpha) x)^{-1}, s, K, r_max)
  r      = e_s - alpha^{-1} [I - (1 - alpha) P] pi^        (the residual)
  every v with r(v) != 0 starts W_v = ceil(|r(v)| W) alpha-random walks; a
  walk stops at its current node with probability alpha, else moves to a
  uniform neighbour; each walk that stops at u adds r(v) / W_v to pi^(u).
  Lemma 9: pi_s(u) = pi^(u) + sum_v r(v) pi_v(u), so the walk phase is an
  unbiased estimate of the remaining mass.

Random numbers (the method draws them; both implementations derive them
from one published counter-based generator, SplitMix64 of Steele, Lea &
Flood, 2014):
  out(seed, c) = mix(seed + (c + 1) * 0x9E3779B97F4A7C15), mix the
  variant-13 finalizer.  Walk j from node v (caller id) uses the stream
  key_v = out(seed, v) and draws out(key_v, j * 2^32 + 2 t) (stop test at
  step t: (x >> 11) * 2^-53 < alpha) and out(key_v, j * 2^32 + 2 t + 1)
  (neighbour index (x * d) >> 64 into the row of the current node in CSR
  order).  A walk is cut after 2^20 steps (probability (1 - alpha)^(2^20)).
"""

from __future__ import annotations

import math

import numpy as np

from . import coefficients as C
from . import propagation as PR
from . import push as PU

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
MAX_STEPS = 1 << 20


def splitmix64(seed: int, ctr: int) -> int:
    """Output number ``ctr`` (0-based) of the SplitMix64 stream of ``seed``."""
    z = (seed + (ctr + 1) * _GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def walk_budget(n: int, eps_r: float, delta: float) -> float:
    """W of Alg. 5."""
    return 2.0 * (2.0 * eps_r / 3.0 + 2.0) * math.log(n) / (eps_r * eps_r * delta)


def residual(row_ptr, col_idx, s: int, alpha: float, pi_hat: np.ndarray) -> np.ndarray:
    """r = e_s - alpha^{-1} [I - (1 - alpha) P] pi^."""
    P = PR.transition_matrix(row_ptr, col_idx)
    n = P.shape[0]
    return PR.one_hot(n, s) - (pi_hat - (1.0 - alpha) * (P @ pi_hat)) / alpha


def walk(row_ptr, col_idx, key: int, j: int, start: int, alpha: float) -> tuple[int, int]:
    """The alpha-random walk j of stream ``key`` from ``start``: (end node,
    number of moves)."""
    cur = int(start)
    base = j << 32
    for t in range(MAX_STEPS):
        x = splitmix64(key, base + 2 * t)
        if (x >> 11) * 2.0**-53 < alpha:
            return cur, t
        p0, p1 = int(row_ptr[cur]), int(row_ptr[cur + 1])
        x2 = splitmix64(key, base + 2 * t + 1)
        cur = int(col_idx[p0 + ((x2 * (p1 - p0)) >> 64)])
    return cur, MAX_STEPS


def walk_terminal(row_ptr, col_idx, key: int, j: int, start: int, alpha: float) -> int:
    return walk(row_ptr, col_idx, key, j, start, alpha)[0]


def push_rw(row_ptr, col_idx, s: int, alpha: float, K: int, eps_r: float, delta: float, seed: int,
            trace: bool = False, r_max: float | None = None):
    """Alg. 5.  Returns pi^ (and, with ``trace``, the push-phase estimate, the
    residual, the walk counts and the walk end nodes per start node).
    ``r_max`` overrides Alg. 5's sqrt(alpha) / W (a larger threshold leaves
    more of the mass to the walks)."""
    n = int(np.asarray(row_ptr).shape[0] - 1)
    W = walk_budget(n, eps_r, delta)
    if r_max is None:
        r_max = math.sqrt(alpha) / W
    c = C.ppr_chebyshev_coeffs(alpha, K)
    pi_push = PU.cheby_push(row_ptr, col_idx, s, c, K, r_max)
    r = residual(row_ptr, col_idx, s, alpha, pi_push)
    pi_hat = pi_push.copy()
    counts = np.zeros(n, dtype=np.int64)
    ends = {}
    steps = 0
    ceil_margin = np.inf  # distance of |r(v)| W to the integers (diagnostic)
    for v in np.flatnonzero(r != 0.0):
        x = abs(r[v]) * W
        ceil_margin = min(ceil_margin, x - math.floor(x) if x != math.floor(x) else 0.0,
                          math.ceil(x) - x if x != math.ceil(x) else 0.0)
        Wv = int(math.ceil(x))
        counts[v] = Wv
        key = splitmix64(seed, int(v))
        share = r[v] / Wv
        ends[int(v)] = []
        for j in range(Wv):
            u, t = walk(row_ptr, col_idx, key, j, v, alpha)
            steps += t
            pi_hat[u] += share
            ends[int(v)].append(u)
    if trace:
        return pi_hat, {"pi_push": pi_push, "residual": r, "walks": counts, "ends": ends, "W": W,
                        "r_max": r_max, "steps": steps, "ceil_margin": ceil_margin}
    return pi_hat
