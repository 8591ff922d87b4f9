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
