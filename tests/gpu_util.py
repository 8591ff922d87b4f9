"""Helpers for the GPU tests: run the HIP library through its C ABI (via the
ctypes binding) and the oracle on the same seeded inputs."""

from __future__ import annotations

import numpy as np

from oracle import coefficients as C
from oracle import errors as E
from oracle import propagation as PR


def require_gpu():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a GPU")
    from paper_2412_10789_amd import chebyprop

    chebyprop.load()  # raises if the HIP library is missing
    return torch


def gpu_graph(g, **kw):
    from paper_2412_10789_amd.chebyprop import Graph

    return Graph(g.row_ptr, g.col_idx, **kw)


def oracle_yK(g, s, kind, param, K, P=None):
    """Alg. 3 in FP64 at the GPU's K."""
    if P is None:
        P = PR.transition_matrix(g.row_ptr, g.col_idx)
    return PR.cheby_power(P, int(s), C.chebyshev_coeffs(kind, param, K), K)


def compare(y_gpu, y_ref, degrees=None) -> dict:
    y = np.asarray(y_gpu, dtype=np.float64)
    out = {"l1": E.l1(y, y_ref), "max_abs": E.max_abs(y, y_ref), "l2": E.l2(y, y_ref)}
    if degrees is not None:
        out["deg_norm"] = E.degree_normalized(y, y_ref, degrees)
    return out


def oracle_yK_multi(g, metas, Ks):
    """Alg. 3 in FP64 at the GPU's K for several (kind, param, source)
    queries at once: the plain-C oracle's several-source form, [n][B]."""
    from oracle import native as NO

    cs = [C.chebyshev_coeffs(kind, param, K) for (kind, param, _), K in zip(metas, Ks)]
    return NO.cheby_power_multi(g.row_ptr, g.col_idx, [int(s) for _, _, s in metas], cs, list(Ks))


def oracle_exact_multi(g, metas, tail=1e-15):
    """The converged vectors f(P) e_s of several queries: the plain-C
    PwMethod with its exact l1 tail below `tail`, [n][B]."""
    from oracle import native as NO
    from oracle import truncation as T

    Ns = [T.pwmethod_steps(kind, param, tail) for kind, param, _ in metas]
    zs = [C.taylor_coeffs(kind, param, N) for (kind, param, _), N in zip(metas, Ns)]
    return NO.power_method_multi(g.row_ptr, g.col_idx, [int(s) for _, _, s in metas], zs, Ns)


# Rounding bars (l1 against Alg. 3 in FP64 at the same K).  FP32 storage with
# double sums measures about 6e-8 at 4M nodes and below that on smaller
# graphs; float sums measured 1.7e-7, which these bars reject.  BF16 storage
# (float sums) measures 1.5e-3 to 3.6e-3 on the benchmark graphs and up to
# 5.0e-3 for the longest recurrences (K near 50) of a 150K-node graph.
F32_L1 = 1.2e-7
BF16_L1 = 8e-3
# FP32 storage with float sums, float partials and a float estimate
# (CP_F32F) measures 1.7e-7 to 2.9e-7 at 150K and 4M nodes (HKPR t = 10 the
# largest); this bar is twice the largest, and it rejects BF16-level error.
F32F_L1 = 6e-7


def f32_bar(K: int, kind: str = "ppr", param: float = 0.0) -> float:
    """The FP32 rounding bar for a recurrence of K steps: the stored iterates'
    rounding accumulates over the steps, so F32_L1 holds up to K = 30 and
    grows in proportion beyond; HKPR with t above 5 weights the later,
    larger iterates more and gets twice that (measured 1.34e-7 for t = 10 at
    K = 22 on 4M nodes)."""
    bar = F32_L1 * max(1.0, K / 30.0)
    return 2.0 * bar if kind == "hkpr" and param > 5.0 else bar


def f32f_bar(K: int) -> float:
    """The CP_F32F rounding bar for a recurrence of K steps (grows in
    proportion beyond K = 30, as f32_bar)."""
    return F32F_L1 * max(1.0, K / 30.0)
