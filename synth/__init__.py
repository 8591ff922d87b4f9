"""Seeded synthetic inputs for the ChebyPower workloads.

Holds no propagation arithmetic: graphs (Chung-Lu power-law graphs and small
textbook graphs, all as symmetric CSR with int64 offsets and int32 columns),
source-node draws and tolerance draws.  Both the CPU reference and the GPU
library's tests and benchmark take their inputs from here.

Every random draw is a pure function of (seed, counter) through SplitMix64
(Steele, Lea & Flood 2014), the same generator the C++ part uses.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chunglu.cpp")
_LIB = os.path.join(_HERE, "libsynth.so")
_MASK = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def build(force: bool = True) -> str:
    """Compile the C++ generator into ``synth/libsynth.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("n_target", ctypes.c_int64),
        ("m_target", ctypes.c_int64),
        ("gamma", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("relabel", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("tune_passes", ctypes.c_int32),
        ("verbose", ctypes.c_int32),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("d_max", ctypes.c_int64),
        ("n_dropped", ctypes.c_int64),
        ("pairs_drawn", ctypes.c_int64),
        ("i0", ctypes.c_double),
    ]


class _Graph(ctypes.Structure):
    _fields_ = [
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col_idx", ctypes.POINTER(ctypes.c_int32)),
        ("info", _Info),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.synth_chunglu.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.POINTER(_Graph))]
        lib.synth_chunglu.restype = ctypes.c_int
        lib.synth_graph_free.argtypes = [ctypes.POINTER(_Graph)]
        lib.synth_graph_free.restype = None
        lib.synth_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_splitmix64_at.restype = ctypes.c_uint64
        _lib = lib
    return _lib


@dataclass
class CSRGraph:
    """Undirected simple graph as symmetric CSR (rows sorted by column)."""

    row_ptr: np.ndarray  # int64 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    name: str = ""
    meta: dict | None = None

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


# --------------------------------------------------------------------------
# counter-based random numbers


def splitmix64_at(seed: int, ctr: int) -> int:
    """Output ``ctr`` (0-based) of the SplitMix64 stream started at ``seed``."""
    z = (seed + (ctr + 1) * _GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def uniform_ints(seed: int, count: int, high: int, offset: int = 0) -> np.ndarray:
    """``count`` draws, uniform over ``[0, high)`` (multiply-high mapping)."""
    return np.array(
        [(splitmix64_at(seed, offset + i) * high) >> 64 for i in range(count)], dtype=np.int64
    )


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    return np.array(
        [(splitmix64_at(seed, offset + i) >> 11) * 2.0**-53 for i in range(count)], dtype=np.float64
    )


def sources(g: CSRGraph, count: int, seed: int) -> np.ndarray:
    """Source nodes uniform over the nodes that have at least one edge."""
    deg = g.degrees
    ok = np.flatnonzero(deg > 0)
    idx = uniform_ints(seed ^ 0x51ED5EED, count, len(ok))
    return ok[idx].astype(np.int64)


def top_degree_sources(g: CSRGraph, count: int) -> np.ndarray:
    deg = g.degrees
    order = np.argsort(-deg, kind="stable")
    return order[:count].astype(np.int64)


def tolerance_choice(seed: int, count: int, choices) -> np.ndarray:
    choices = np.asarray(choices, dtype=np.float64)
    return choices[uniform_ints(seed ^ 0x70715EED, count, len(choices))]


def tolerance_loguniform(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    u = uniform01(seed ^ 0x10C0A11F, count)
    return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))


# --------------------------------------------------------------------------
# graphs


def chung_lu(
    n: int,
    m: int,
    gamma: float,
    seed: int,
    relabel: str = "random",
    threads: int = 0,
    tune_passes: int = 3,
    verbose: bool = False,
) -> CSRGraph:
    """Seeded Chung-Lu power-law graph with about ``m`` undirected edges."""
    lib = _load()
    p = _Params(n, m, gamma, seed & _MASK, {"none": 0, "random": 1}[relabel], threads, tune_passes, int(verbose))
    out = ctypes.POINTER(_Graph)()
    rc = lib.synth_chunglu(ctypes.byref(p), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"synth_chunglu failed with code {rc}")
    try:
        info = out.contents.info
        nn, nnz = int(info.n), int(info.nnz)
        rp = np.ctypeslib.as_array(out.contents.row_ptr, shape=(nn + 1,)).copy()
        ci = (
            np.ctypeslib.as_array(out.contents.col_idx, shape=(nnz,)).copy()
            if nnz
            else np.zeros(0, np.int32)
        )
        meta = dict(
            n_target=n, m_target=m, gamma=gamma, seed=seed, relabel=relabel,
            d_max=int(info.d_max), n_dropped=int(info.n_dropped),
            pairs_drawn=int(info.pairs_drawn), i0=float(info.i0),
        )
    finally:
        lib.synth_graph_free(out)
    return CSRGraph(rp, ci, name=f"chunglu(n={n},m={m},gamma={gamma},seed={seed})", meta=meta)


def from_edges(n: int, edges, name: str = "") -> CSRGraph:
    """Symmetric simple CSR from an undirected edge list (self-loops and
    duplicates removed)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]], axis=0)
    if both.size:
        key = np.unique(both[:, 0] * n + both[:, 1])
        src, dst = key // n, key % n
    else:
        src = dst = np.zeros(0, np.int64)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    return CSRGraph(rp.astype(np.int64), dst.astype(np.int32), name=name)


def star(leaves: int) -> CSRGraph:
    """Centre 0 joined to nodes 1..leaves."""
    return from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)], name=f"star({leaves})")


def cycle(n: int) -> CSRGraph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name=f"cycle({n})")


def path(n: int) -> CSRGraph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name=f"path({n})")


def complete(n: int) -> CSRGraph:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name=f"complete({n})")


def erdos_renyi(n: int, p: float, seed: int) -> CSRGraph:
    """G(n, p) with one counter-based coin per unordered pair."""
    iu, ju = np.triu_indices(n, k=1)
    u = uniform01(seed ^ 0xE5D05E11, len(iu))
    keep = u < p
    return from_edges(n, zip(iu[keep].tolist(), ju[keep].tolist()), name=f"er({n},{p},{seed})")


def barbell_with_tail(clique: int, tail: int) -> CSRGraph:
    """Two cliques joined by a path: irregular degrees, long diameter."""
    n = 2 * clique + tail
    edges = [(i, j) for i in range(clique) for j in range(i + 1, clique)]
    off = clique + tail
    edges += [(off + i, off + j) for i in range(clique) for j in range(i + 1, clique)]
    chain = [clique - 1] + list(range(clique, clique + tail)) + [off]
    edges += list(zip(chain[:-1], chain[1:]))
    return from_edges(n, edges, name=f"barbell({clique},{tail})")
