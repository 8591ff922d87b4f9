"""ctypes access to the plain-C FP64 oracle (oracle/c/chebypower.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Same Alg. 3 / Alg. 1 as
oracle.propagation, for graphs where the scipy version is too slow; it is
pinned against the Python oracle by tests/test_oracle_native.py.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c", "chebypower.c")
_LIB = os.path.join(_HERE, "c", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        for fn in ("oracle_chebypower", "oracle_pwmethod"):
            f = getattr(lib, fn)
            f.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, P, ctypes.c_int32, P]
            f.restype = ctypes.c_int
        lib.oracle_chebypower_multi.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, P, ctypes.c_int32, P, P]
        lib.oracle_chebypower_multi.restype = ctypes.c_int
        lib.oracle_pwmethod_multi.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, P, ctypes.c_int32, P, P]
        lib.oracle_pwmethod_multi.restype = ctypes.c_int
        lib.oracle_ppr_residual_multi.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, P, P, P]
        lib.oracle_ppr_residual_multi.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_verbose.argtypes = [ctypes.c_int]
        lib.oracle_set_verbose.restype = None
        _lib = lib
    return _lib


def set_verbose(on: bool) -> None:
    """Print one line per step to stderr (long runs on large graphs)."""
    _load().oracle_set_verbose(1 if on else 0)


def threads() -> int:
    return int(_load().oracle_threads())


def set_threads(t: int) -> None:
    """Threads of the oracle's OpenMP loops from here on (0: the count the
    process started with)."""
    _load().oracle_set_threads(int(t))


def _call(name, row_ptr, col_idx, s, coeffs, K):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    n = rp.shape[0] - 1
    y = np.empty(n, dtype=np.float64)
    rc = getattr(_load(), name)(n, rp.ctypes.data, ci.ctypes.data, int(s), c.ctypes.data, int(K), y.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"{name} failed with {rc}")
    return y


def cheby_power(row_ptr, col_idx, s: int, c, K: int) -> np.ndarray:
    """Alg. 3 with coefficients c_0..c_K (FP64)."""
    if len(c) < K + 1:
        raise ValueError("need c_0..c_K")
    return _call("oracle_chebypower", row_ptr, col_idx, s, c, K)


def _multi(name, row_ptr, col_idx, sources, coeffs, Ks, extra: int) -> np.ndarray:
    """Shared marshalling of the several-source calls: coefficient row j
    holds Ks[j] + extra leading entries (extra = 1: c_0..c_K; extra = 0:
    zeta_0..zeta_{N-1})."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int64)
    Kv = np.ascontiguousarray(Ks, dtype=np.int32)
    B = src.shape[0]
    if Kv.shape[0] != B or len(coeffs) != B:
        raise ValueError("one truncation step and one coefficient row per source")
    ldc = int(Kv.max()) + extra
    c = np.zeros((B, ldc), dtype=np.float64)
    for j, cj in enumerate(coeffs):
        need = int(Kv[j]) + extra
        if len(cj) < need:
            raise ValueError("coefficient row too short")
        c[j, :need] = np.asarray(cj, dtype=np.float64)[:need]
    n = rp.shape[0] - 1
    Y = np.empty((n, B), dtype=np.float64)
    rc = getattr(_load(), name)(n, rp.ctypes.data, ci.ctypes.data, B, src.ctypes.data, c.ctypes.data, ldc,
                                Kv.ctypes.data, Y.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"{name} failed with {rc}")
    return Y


def cheby_power_multi(row_ptr, col_idx, sources, coeffs, Ks) -> np.ndarray:
    """Alg. 3 for several sources in one pass per step: column j of the
    [n][B] result is Alg. 3 from sources[j] with coefficients coeffs[j]
    (c_0..c_{K_j}) and truncation step Ks[j], summed exactly as
    cheby_power sums it."""
    return _multi("oracle_chebypower_multi", row_ptr, col_idx, sources, coeffs, Ks, 1)


def power_method_multi(row_ptr, col_idx, sources, zetas, Ns) -> np.ndarray:
    """Alg. 1 for several sources in one pass per step: column j is
    power_method from sources[j] with weights zetas[j] (zeta_0..zeta_{N_j-1})."""
    return _multi("oracle_pwmethod_multi", row_ptr, col_idx, sources, zetas, Ns, 0)


def ppr_residual_multi(row_ptr, col_idx, sources, alphas, Y) -> np.ndarray:
    """For each column y_j of Y [n][B]: ||alpha_j e_s + (1 - alpha_j) P y_j -
    y_j||_1, the residual of Def. 3's fixed-point equation.  Divided by
    alpha_j it bounds ||pi_s - y_j||_1 (see oracle.errors.ppr_certificate)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int64)
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    Yd = np.ascontiguousarray(Y, dtype=np.float64)
    n = rp.shape[0] - 1
    B = src.shape[0]
    if Yd.shape != (n, B) or al.shape[0] != B:
        raise ValueError("Y must be [n][B] with one alpha per column")
    res = np.empty(B, dtype=np.float64)
    rc = _load().oracle_ppr_residual_multi(n, rp.ctypes.data, ci.ctypes.data, B, src.ctypes.data, al.ctypes.data,
                                           Yd.ctypes.data, res.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_ppr_residual_multi failed with {rc}")
    return res


def power_method(row_ptr, col_idx, s: int, zeta, N: int) -> np.ndarray:
    """Alg. 1 with Taylor coefficients zeta_0..zeta_{N-1} (FP64)."""
    return _call("oracle_pwmethod", row_ptr, col_idx, s, zeta, N)
