"""Python binding of the C ABI in include/chebyprop.h (argument marshalling
only: every step of the computation runs in the HIP library).

The functions ``cp_*`` mirror the C calls one to one.  ``Graph`` is a thin
convenience wrapper that uses PyTorch for device memory and streams.  If
``libchebyprop.so`` has not been built the import fails loudly: there is no
CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libchebyprop.so")

# status codes
CP_OK = 0
CP_EINVAL = -1
CP_ESOURCE = -2
CP_EISOLATED = -3
CP_ENOMEM = -4
CP_EHIP = -5
CP_EKMAX = -6
CP_EBUSY = -7
CP_ECANCELLED = -8
CP_ENOTFOUND = -9
CP_EGRAPH = -10
CP_EPENDING = -11
CP_EWORKSPACE = -12

CP_PPR, CP_HKPR = 0, 1
CP_F64, CP_F32, CP_BF16, CP_F32F = 0, 1, 2, 3
CP_K_CERTIFIED, CP_K_TAIL, CP_K_PAPER, CP_K_FIXED = 0, 1, 2, 3
CP_GRAPH_BORROW, CP_GRAPH_VALIDATE, CP_GRAPH_REORDER, CP_GRAPH_HOST = 0x1, 0x2, 0x4, 0x8
CP_GRAPH_HOT_SPLIT = 0x20
CP_GRAPH_XCD_STRIPES = 0x10
CP_Q_STATS, CP_Q_TIMING, CP_Q_PWMETHOD, CP_Q_CLENSHAW = 0x1, 0x2, 0x4, 0x8
CP_NOALLOC_SCRATCH_BYTES = 64 << 20  # the static device array cp_power_noalloc works in

KINDS = {"ppr": CP_PPR, "hkpr": CP_HKPR}
PRECS = {"f64": CP_F64, "f32": CP_F32, "f32f": CP_F32F, "bf16": CP_BF16}
KMODES = {"certified": CP_K_CERTIFIED, "tail": CP_K_TAIL, "paper": CP_K_PAPER, "fixed": CP_K_FIXED}
# Alg. 3 (ChebyPower), Alg. 1 (PwMethod), Alg. 3's series by Clenshaw's
# recurrence (cp_propagate only)
METHODS = {"cheby": 0, "power": CP_Q_PWMETHOD, "clenshaw": CP_Q_CLENSHAW}

# every symbol the header declares
EXPORTED = [
    "cp_graph_create", "cp_graph_destroy", "cp_graph_get_stats", "cp_coeffs", "cp_choose_K",
    "cp_taylor", "cp_choose_N",
    "cp_workspace_bytes", "cp_power", "cp_power_noalloc", "cp_power_batch", "cp_propagate", "cp_push", "cp_push_workspace_bytes",
    "cp_push_rw", "cp_push_rw_workspace_bytes", "cp_autotune_batch", "cp_autotune_single", "cp_set_batch_width",
    "cp_status_str", "cp_last_hip_error", "cp_version",
    "cp_server_create", "cp_server_submit", "cp_server_poll", "cp_server_wait", "cp_server_cancel",
    "cp_server_get_stats", "cp_server_destroy",
]


class cp_query(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("kmode", ctypes.c_int32),
        ("param", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("source", ctypes.c_int64),
        ("K_fixed", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("a", ctypes.c_double),
    ]


class cp_info(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("tail", ctypes.c_double),
        ("tail_bound_l1", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("step_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
        ("wait_ms", ctypes.c_double),
        ("pushes", ctypes.c_int64),
        ("arcs", ctypes.c_int64),
        ("walks", ctypes.c_int64),
        ("walk_steps", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class cp_graph_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("d_max", ctypes.c_int64),
        ("blocks", ctypes.c_int64),
        ("long_rows", ctypes.c_int64),
        ("hub_rows", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("reordered", ctypes.c_int32),
        ("borrowed", ctypes.c_int32),
        ("stripe_tiles", ctypes.c_int64),
        ("stripe_packed", ctypes.c_int64),
        ("stripe_count", ctypes.c_int64),
        ("hot_nodes", ctypes.c_int64),
        ("hot_arcs", ctypes.c_int64),
        ("single_long_cut", ctypes.c_int64),
        ("single_hub_cut", ctypes.c_int64),
        ("single_hub_seg", ctypes.c_int64),
        ("batch_long_cut", ctypes.c_int64),
        ("batch_hub_cut", ctypes.c_int64),
        ("batch_hub_seg", ctypes.c_int64),
    ]


class cp_server_stats(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int64),
        ("active", ctypes.c_int64),
        ("queued", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("cancelled", ctypes.c_int64),
        ("ticks", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("tile_width", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("waiters", ctypes.c_int32),
        ("direct_limit", ctypes.c_int32),
        ("direct", ctypes.c_int64),
        ("narrow_ticks", ctypes.c_int64),
    ]


class ChebypropError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = cp_status_str(status)
        if status == CP_EHIP:
            msg += f" (hipError_t {cp_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")


_lib = None


def load() -> ctypes.CDLL:
    """Load libchebyprop.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2412_10789_amd.build` "
            "(there is no CPU fallback)"
        )
    # Bind to the HIP runtime PyTorch uses (torch ships its own libamdhip64
    # with the same soname as ROCm's): streams and device pointers handed
    # over from torch are only valid in that runtime, so torch is loaded
    # first and the library's libamdhip64 dependency resolves to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "cp_graph_create": (i32, [i64, i64, P, P, i32, P, ctypes.POINTER(P)]),
        "cp_graph_destroy": (i32, [P]),
        "cp_graph_get_stats": (i32, [P, ctypes.POINTER(cp_graph_stats)]),
        "cp_coeffs": (i32, [i32, f64, i32, ctypes.POINTER(f64)]),
        "cp_choose_K": (i32, [i32, f64, f64, i32, i32, f64, f64, i32, ctypes.POINTER(i32), ctypes.POINTER(f64)]),
        "cp_taylor": (i32, [i32, f64, i32, ctypes.POINTER(f64)]),
        "cp_choose_N": (i32, [i32, f64, f64, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(f64)]),
        "cp_workspace_bytes": (sz, [P, i32, i32]),
        "cp_power": (i32, [P, ctypes.POINTER(cp_query), i32, P, P, sz, P, ctypes.POINTER(cp_info)]),
        "cp_power_noalloc": (i32, [P, ctypes.POINTER(cp_query), i32, P, P, ctypes.POINTER(cp_info)]),
        "cp_power_batch": (i32, [P, i32, ctypes.POINTER(cp_query), i32, P, P, sz, P, ctypes.POINTER(cp_info)]),
        "cp_push": (i32, [P, ctypes.POINTER(cp_query), f64, P, P, sz, P, ctypes.POINTER(cp_info)]),
        "cp_push_workspace_bytes": (sz, [P]),
        "cp_push_rw": (i32, [P, ctypes.POINTER(cp_query), f64, f64, f64, ctypes.c_uint64, P, P, sz, P,
                             ctypes.POINTER(cp_info)]),
        "cp_push_rw_workspace_bytes": (sz, [P]),
        "cp_propagate": (i32, [P, ctypes.POINTER(cp_query), i32, i32, P, P, P, sz, P, ctypes.POINTER(cp_info)]),
        "cp_autotune_batch": (i32, [P, i32, ctypes.POINTER(cp_query), i32, P, P, sz, P, ctypes.POINTER(i32)]),
        "cp_set_batch_width": (i32, [P, i32, i32, i32]),
        "cp_autotune_single": (i32, [P, ctypes.POINTER(cp_query), i32, P, P, sz, P]),
        "cp_server_create": (i32, [P, sz, i32, i32, i32, ctypes.POINTER(P)]),
        "cp_server_submit": (i32, [P, ctypes.POINTER(cp_query), P, ctypes.POINTER(ctypes.c_uint64)]),
        "cp_server_poll": (i32, [P, ctypes.c_uint64, ctypes.POINTER(cp_info)]),
        "cp_server_wait": (i32, [P, ctypes.c_uint64, i64, ctypes.POINTER(cp_info)]),
        "cp_server_cancel": (i32, [P, ctypes.c_uint64]),
        "cp_server_get_stats": (i32, [P, ctypes.POINTER(cp_server_stats)]),
        "cp_server_destroy": (i32, [P]),
        "cp_status_str": (ctypes.c_char_p, [i32]),
        "cp_last_hip_error": (i32, []),
        "cp_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ---------------------------------------------------------------- raw calls


def cp_status_str(status: int) -> str:
    return load().cp_status_str(status).decode()


def cp_last_hip_error() -> int:
    return int(load().cp_last_hip_error())


def cp_version() -> str:
    return load().cp_version().decode()


def _check(status: int, where: str) -> None:
    if status != CP_OK:
        raise ChebypropError(status, where)


def cp_coeffs(kind: int, param: float, K: int) -> np.ndarray:
    c = np.zeros(K + 1, dtype=np.float64)
    _check(load().cp_coeffs(kind, param, K, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "cp_coeffs")
    return c


def cp_choose_K(kind: int, param: float, tol: float, kmode: int = CP_K_CERTIFIED, K_fixed: int = 0,
                vol: float = 1.0, d_s: float = 1.0, K_max: int = 0) -> tuple[int, float]:
    K = ctypes.c_int32(0)
    tail = ctypes.c_double(0.0)
    _check(load().cp_choose_K(kind, param, tol, kmode, K_fixed, vol, d_s, K_max,
                              ctypes.byref(K), ctypes.byref(tail)), "cp_choose_K")
    return int(K.value), float(tail.value)


def cp_taylor(kind: int, param: float, N: int) -> np.ndarray:
    z = np.zeros(N, dtype=np.float64)
    _check(load().cp_taylor(kind, param, N, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "cp_taylor")
    return z


def cp_choose_N(kind: int, param: float, tol: float, kmode: int = CP_K_CERTIFIED, N_fixed: int = 0,
                N_max: int = 0) -> tuple[int, float]:
    N = ctypes.c_int32(0)
    tail = ctypes.c_double(0.0)
    _check(load().cp_choose_N(kind, param, tol, kmode, N_fixed, N_max, ctypes.byref(N), ctypes.byref(tail)),
           "cp_choose_N")
    return int(N.value), float(tail.value)


def cp_graph_create(n: int, nnz: int, row_ptr_ptr: int, col_idx_ptr: int, flags: int, stream: int) -> int:
    out = ctypes.c_void_p()
    _check(load().cp_graph_create(n, nnz, row_ptr_ptr, col_idx_ptr, flags, stream, ctypes.byref(out)),
           "cp_graph_create")
    return out.value


def cp_graph_destroy(handle: int) -> None:
    _check(load().cp_graph_destroy(handle), "cp_graph_destroy")


def cp_graph_get_stats(handle: int) -> dict:
    st = cp_graph_stats()
    _check(load().cp_graph_get_stats(handle, ctypes.byref(st)), "cp_graph_get_stats")
    return {f: getattr(st, f) for f, _ in st._fields_}


def cp_workspace_bytes(handle: int, nq: int, prec: int) -> int:
    return int(load().cp_workspace_bytes(handle, nq, prec))


def cp_power(handle: int, query: cp_query, prec: int, y_ptr: int, ws_ptr: int, ws_bytes: int,
             stream: int) -> cp_info:
    info = cp_info()
    _check(load().cp_power(handle, ctypes.byref(query), prec, y_ptr, ws_ptr, ws_bytes, stream,
                           ctypes.byref(info)), "cp_power")
    return info


def cp_power_noalloc(handle: int, query: cp_query, prec: int, y_ptr: int, stream: int) -> cp_info:
    info = cp_info()
    _check(load().cp_power_noalloc(handle, ctypes.byref(query), prec, y_ptr, stream, ctypes.byref(info)),
           "cp_power_noalloc")
    return info


def cp_power_batch(handle: int, queries, prec: int, Y_ptr: int, ws_ptr: int, ws_bytes: int,
                   stream: int) -> list:
    nq = len(queries)
    arr = (cp_query * nq)(*queries)
    infos = (cp_info * nq)()
    _check(load().cp_power_batch(handle, nq, arr, prec, Y_ptr, ws_ptr, ws_bytes, stream, infos),
           "cp_power_batch")
    return list(infos)


def cp_push(handle: int, query: cp_query, eps_a: float, y_ptr: int, ws_ptr: int, ws_bytes: int,
            stream: int) -> cp_info:
    info = cp_info()
    _check(load().cp_push(handle, ctypes.byref(query), float(eps_a), y_ptr, ws_ptr, ws_bytes, stream,
                          ctypes.byref(info)), "cp_push")
    return info


def cp_push_workspace_bytes(handle: int) -> int:
    return int(load().cp_push_workspace_bytes(handle))


def cp_push_rw(handle: int, query: cp_query, eps_r: float, delta: float, r_max: float, seed: int, y_ptr: int,
               ws_ptr: int, ws_bytes: int, stream: int) -> cp_info:
    info = cp_info()
    _check(load().cp_push_rw(handle, ctypes.byref(query), float(eps_r), float(delta), float(r_max),
                             int(seed) & ((1 << 64) - 1), y_ptr, ws_ptr, ws_bytes, stream, ctypes.byref(info)),
           "cp_push_rw")
    return info


def cp_push_rw_workspace_bytes(handle: int) -> int:
    return int(load().cp_push_rw_workspace_bytes(handle))


def cp_propagate(handle: int, query: cp_query, k: int, prec: int, X_ptr: int, Z_ptr: int, ws_ptr: int,
                 ws_bytes: int, stream: int) -> cp_info:
    info = cp_info()
    _check(load().cp_propagate(handle, ctypes.byref(query), k, prec, X_ptr, Z_ptr, ws_ptr, ws_bytes, stream,
                               ctypes.byref(info)), "cp_propagate")
    return info


def cp_autotune_batch(handle: int, queries, prec: int, Y_ptr: int, ws_ptr: int, ws_bytes: int,
                      stream: int) -> int:
    nq = len(queries)
    arr = (cp_query * nq)(*queries)
    bw = ctypes.c_int32(0)
    _check(load().cp_autotune_batch(handle, nq, arr, prec, Y_ptr, ws_ptr, ws_bytes, stream, ctypes.byref(bw)),
           "cp_autotune_batch")
    return int(bw.value)


def cp_set_batch_width(handle: int, nq: int, prec: int, bw: int) -> None:
    _check(load().cp_set_batch_width(handle, nq, prec, bw), "cp_set_batch_width")


def make_query(kind: str, param: float, source: int, tol: float = 1e-6, kmode: str = "certified",
               K: int = 0, flags: int = 0, method: str = "cheby", a: float = 0.0) -> cp_query:
    return cp_query(KINDS[kind], KMODES[kmode], float(param), float(tol), int(source), int(K),
                    int(flags) | METHODS[method], float(a))


# ---------------------------------------------------------------- torch wrapper


@dataclass
class Result:
    y: "object"  # torch tensor on the GPU (caller ids)
    info: dict


class Graph:
    """A graph resident in HBM (owned by the library)."""

    def __init__(self, row_ptr, col_idx, reorder: bool = False, validate: bool = False, device=None,
                 stripes: bool = False, host_input: bool | None = None, hot_split: bool = False):
        """row_ptr / col_idx: host arrays (numpy), handed to the library as
        host pointers (CP_GRAPH_HOST), or device tensors (host_input=False
        uploads host arrays first and passes device pointers)."""
        import torch

        self.torch = torch
        dev = torch.device(device or "cuda")
        on_device = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
        if host_input is None:
            host_input = not on_device
        if host_input:
            rp = np.ascontiguousarray(row_ptr.cpu().numpy() if isinstance(row_ptr, torch.Tensor) else row_ptr,
                                      dtype=np.int64)
            ci = np.ascontiguousarray(col_idx.cpu().numpy() if isinstance(col_idx, torch.Tensor) else col_idx,
                                      dtype=np.int32)
            rp_ptr, ci_ptr = rp.ctypes.data, ci.ctypes.data
            n, nnz = rp.shape[0] - 1, ci.shape[0]
        else:
            rp = torch.as_tensor(row_ptr, dtype=torch.int64).to(dev).contiguous()
            ci = torch.as_tensor(col_idx, dtype=torch.int32).to(dev).contiguous()
            rp_ptr, ci_ptr = rp.data_ptr(), ci.data_ptr()
            n, nnz = int(rp.numel() - 1), int(ci.numel())
        self.n = int(n)
        self.nnz = int(nnz)
        self.device = dev
        flags = ((CP_GRAPH_REORDER if reorder else 0) | (CP_GRAPH_VALIDATE if validate else 0)
                 | (CP_GRAPH_XCD_STRIPES if stripes else 0) | (CP_GRAPH_HOST if host_input else 0)
                 | (CP_GRAPH_HOT_SPLIT if hot_split else 0))
        with torch.cuda.device(dev):
            stream = torch.cuda.current_stream().cuda_stream
            self.handle = cp_graph_create(self.n, self.nnz, rp_ptr, ci_ptr, flags, stream)
        self.stats = cp_graph_get_stats(self.handle)
        self._ws = {}
        self._push_ws = None

    def close(self) -> None:
        if getattr(self, "handle", None):
            cp_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def workspace(self, nq: int, prec: int):
        nbytes = cp_workspace_bytes(self.handle, nq, prec)
        key = (nq, prec)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
            self._ws = {key: ws}
        return ws, nbytes

    def out_dtype(self, prec: int):
        return self.torch.float64 if prec == CP_F64 else self.torch.float32

    def power(self, kind: str, param: float, source: int, tol: float = 1e-6, prec: str = "f32",
              kmode: str = "certified", K: int = 0, flags: int = 0, y=None, stream=None,
              method: str = "cheby", a: float = 0.0) -> Result:
        torch = self.torch
        p = PRECS[prec]
        if y is None:
            y = torch.empty(self.n, dtype=self.out_dtype(p), device=self.device)
        ws, nbytes = self.workspace(1, p)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        q = make_query(kind, param, source, tol, kmode, K, flags, method, a)
        info = cp_power(self.handle, q, p, y.data_ptr(), ws.data_ptr(), nbytes, st)
        return Result(y, info.as_dict())

    def power_noalloc(self, kind: str, param: float, source: int, y, tol: float = 1e-6, prec: str = "f32",
                      kmode: str = "certified", K: int = 0, flags: int = 0, stream=None, method: str = "cheby",
                      a: float = 0.0) -> dict:
        """cp_power_noalloc: the query into the caller's tensor y, with the
        library's static device array as workspace; returns the info dict."""
        st = stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        q = make_query(kind, param, source, tol, kmode, K, flags, method, a)
        return cp_power_noalloc(self.handle, q, PRECS[prec], y.data_ptr(), st).as_dict()

    def autotune_single(self, kind: str, param: float, source: int, tol: float = 1e-6, prec: str = "f32",
                        stream=None) -> dict:
        """cp_autotune_single: time the query under each candidate row split
        and keep the fastest plan; returns the graph's stats afterwards."""
        p = PRECS[prec]
        y = self.torch.empty(self.n, dtype=self.out_dtype(p), device=self.device)
        ws, nbytes = self.workspace(1, p)
        st = stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        q = make_query(kind, param, source, tol)
        _check(load().cp_autotune_single(self.handle, ctypes.byref(q), p, y.data_ptr(), ws.data_ptr(), nbytes, st),
               "cp_autotune_single")
        self.stats = cp_graph_get_stats(self.handle)
        return self.stats

    def set_batch_width(self, nq: int, prec: str, bw: int) -> None:
        cp_set_batch_width(self.handle, nq, PRECS[prec], bw)

    def autotune_batch(self, queries, prec: str = "f32", stream=None) -> int:
        torch = self.torch
        p = PRECS[prec]
        nq = len(queries)
        Y = torch.empty((self.n, nq), dtype=self.out_dtype(p), device=self.device)
        ws, nbytes = self.workspace(nq, p)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        bw = cp_autotune_batch(self.handle, queries, p, Y.data_ptr(), ws.data_ptr(), nbytes, st)
        self.stats = cp_graph_get_stats(self.handle)
        return bw

    def power_batch(self, queries, prec: str = "f32", Y=None, stream=None):
        torch = self.torch
        p = PRECS[prec]
        nq = len(queries)
        if Y is None:
            Y = torch.empty((self.n, nq), dtype=self.out_dtype(p), device=self.device)
        ws, nbytes = self.workspace(nq, p)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        infos = cp_power_batch(self.handle, queries, p, Y.data_ptr(), ws.data_ptr(), nbytes, st)
        return Y, [i.as_dict() for i in infos]

    def push(self, kind: str, param: float, source: int, eps_a: float, tol: float = 1e-6,
             kmode: str = "certified", K: int = 0, a: float = 0.0, flags: int = 0, y=None, stream=None) -> Result:
        """ChebyPush (Alg. 4): FP64 result in caller ids."""
        torch = self.torch
        if y is None:
            y = torch.empty(self.n, dtype=torch.float64, device=self.device)
        nbytes = cp_push_workspace_bytes(self.handle)
        ws = self._push_ws
        if ws is None or ws.numel() < nbytes:
            ws = self._push_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        q = make_query(kind, param, source, tol, kmode, K, flags, "cheby", a)
        info = cp_push(self.handle, q, eps_a, y.data_ptr(), ws.data_ptr(), nbytes, st)
        return Result(y, info.as_dict())

    def push_rw(self, alpha: float, source: int, eps_r: float, delta: float, seed: int, r_max: float = 0.0,
                kmode: str = "paper", K: int = 0, a: float = 0.0, flags: int = 0, y=None, stream=None) -> Result:
        """ChebyPush + random walks for SSPPR (Alg. 5): FP64 result in caller ids."""
        torch = self.torch
        if y is None:
            y = torch.empty(self.n, dtype=torch.float64, device=self.device)
        nbytes = cp_push_rw_workspace_bytes(self.handle)
        ws = self._push_ws
        if ws is None or ws.numel() < nbytes:
            ws = self._push_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        q = make_query("ppr", alpha, source, 0.5, kmode, K, flags, "cheby", a)
        info = cp_push_rw(self.handle, q, eps_r, delta, r_max, seed, y.data_ptr(), ws.data_ptr(), nbytes, st)
        return Result(y, info.as_dict())

    def propagate(self, X, kind: str, param: float, a: float = 0.0, tol: float = 1e-6, kmode: str = "tail",
                  K: int = 0, prec: str = "f32", method: str = "cheby", flags: int = 0, Z=None, stream=None):
        """Z = f(D^{-a} A D^{-b}) X (b = 1 - a) for a device matrix X [n][k]
        (float64 for f64, float32 otherwise; caller ids)."""
        torch = self.torch
        p = PRECS[prec]
        if X.dim() != 2 or X.shape[0] != self.n or X.dtype != self.out_dtype(p) or not X.is_contiguous():
            raise ValueError("X must be a contiguous [n, k] tensor of the precision's output type")
        k = int(X.shape[1])
        if Z is None:
            Z = torch.empty_like(X)
        ws, nbytes = self.workspace(k, p)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        q = make_query(kind, param, 0, tol, kmode, K, flags, method, a)
        info = cp_propagate(self.handle, q, k, p, X.data_ptr(), Z.data_ptr(), ws.data_ptr(), nbytes, st)
        return Z, info.as_dict()


# ---------------------------------------------------------------- server


class Server:
    """Query server over a Graph (see cp_server_* in include/chebyprop.h).

    Results land in caller-provided torch tensors; ``submit`` returns a
    ticket, ``wait``/``poll`` return (status, info dict)."""

    def __init__(self, graph: Graph, hbm_budget_bytes: int, max_slots: int = 0, max_queue: int = 4096,
                 prec: str = "f32"):
        self.graph = graph
        self.prec = PRECS[prec]
        out = ctypes.c_void_p()
        _check(load().cp_server_create(graph.handle, int(hbm_budget_bytes), int(max_slots), int(max_queue),
                                       self.prec, ctypes.byref(out)), "cp_server_create")
        self.handle = out.value

    def submit(self, query: cp_query, y) -> int:
        t = ctypes.c_uint64(0)
        _check(load().cp_server_submit(self.handle, ctypes.byref(query), y.data_ptr(), ctypes.byref(t)),
               "cp_server_submit")
        return int(t.value)

    def poll(self, ticket: int):
        info = cp_info()
        st = load().cp_server_poll(self.handle, ticket, ctypes.byref(info))
        return st, (info.as_dict() if st == CP_OK else None)

    def wait(self, ticket: int, timeout_ms: int = -1):
        info = cp_info()
        st = load().cp_server_wait(self.handle, ticket, int(timeout_ms), ctypes.byref(info))
        return st, (info.as_dict() if st == CP_OK else None)

    def cancel(self, ticket: int) -> int:
        return int(load().cp_server_cancel(self.handle, ticket))

    def stats(self) -> dict:
        st = cp_server_stats()
        _check(load().cp_server_get_stats(self.handle, ctypes.byref(st)), "cp_server_get_stats")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check(load().cp_server_destroy(self.handle), "cp_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
