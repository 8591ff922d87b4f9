"""Closed forms on circulant graphs (oracle, test-only): any size, O(n log n).

A circulant graph on n nodes with a symmetric offset set O (o in O implies
-o in O, 0 not in O) joins v to (v + o) mod n.  It is |O|-regular, so
P = A D^{-1} = A / |O| is a symmetric circulant matrix.  The discrete
Fourier transform diagonalises every circulant matrix: if p is P's first
column, P = F^{-1} diag(lambda) F with lambda = DFT(p), real here because p
is symmetric.  For any function g applied to P (Lemma 1 applies f to P
through its eigenvalues),

    g(P) e_s = shift by s of IDFT(g(lambda)).

With g = f this is the exact PPR vector (Def. 3) or HKPR vector (Def. 4);
with g(x) = sum_{k<=K} c_k T_k(x) (Def. 6, Eq. 6 applied to each eigenvalue)
it is ChebyPower's output at truncation step K (Algorithm 3), without any
sparse product.  The tests pin these forms against the dense definitions
and against Algorithm 3 on small circulant graphs; the GPU tests use them
where the graph is too large for a sparse oracle (more than 2^31 arcs).
"""

from __future__ import annotations

import numpy as np


def offsets_band(h: int) -> np.ndarray:
    """O = {-h, ..., -1, 1, ..., h}, ascending."""
    return np.concatenate([np.arange(-h, 0), np.arange(1, h + 1)]).astype(np.int64)


def eigenvalues(n: int, offsets) -> np.ndarray:
    """Eigenvalues of P, indexed by frequency: DFT of P's first column."""
    offsets = np.asarray(offsets, dtype=np.int64)
    p = np.zeros(n, dtype=np.float64)
    np.add.at(p, offsets % n, 1.0 / offsets.shape[0])
    lam = np.fft.fft(p)
    if np.abs(lam.imag).max() > 1e-12:
        raise ValueError("offset set is not symmetric")
    return np.clip(lam.real, -1.0, 1.0)


def apply_spectral(n: int, offsets, s: int, g_lam: np.ndarray) -> np.ndarray:
    """g(P) e_s given g evaluated on the eigenvalues of P."""
    col0 = np.fft.ifft(g_lam).real
    return np.roll(col0, s)


def exact(n: int, offsets, s: int, kind: str, param: float) -> np.ndarray:
    """f(P) e_s: PPR (Def. 3) or HKPR (Def. 4) through the eigenvalues."""
    lam = eigenvalues(n, offsets)
    if kind == "ppr":
        g = param / (1.0 - (1.0 - param) * lam)
    elif kind == "hkpr":
        g = np.exp(-param * (1.0 - lam))
    else:
        raise ValueError(kind)
    return apply_spectral(n, offsets, s, g)


def cheby_truncated(n: int, offsets, s: int, c) -> np.ndarray:
    """sum_{k=0..K} c_k T_k(P) e_s with K = len(c) - 1: the three-term
    recurrence (Eq. 6) run on each eigenvalue, then one inverse DFT."""
    c = np.asarray(c, dtype=np.float64)
    lam = eigenvalues(n, offsets)
    t_prev = np.ones(n)
    g = c[0] * t_prev
    if c.shape[0] > 1:
        t_cur = lam.copy()
        g = g + c[1] * t_cur
        for k in range(2, c.shape[0]):
            t_prev, t_cur = t_cur, 2.0 * lam * t_cur - t_prev
            g = g + c[k] * t_cur
    return apply_spectral(n, offsets, s, g)


def csr(n: int, offsets, chunk_rows: int = 1 << 18):
    """CSR of the circulant graph: row v lists (v + o) mod n for o in the
    given order (rows that wrap around are not sorted).  Offsets are int64,
    columns int32; built in row chunks to bound temporary memory."""
    offsets = np.asarray(offsets, dtype=np.int64)
    d = offsets.shape[0]
    if n >= 1 << 31:
        raise ValueError("int32 columns")
    row_ptr = np.arange(n + 1, dtype=np.int64) * d
    col = np.empty(n * d, dtype=np.int32).reshape(n, d)
    off32 = offsets.astype(np.int32)
    for b in range(0, n, chunk_rows):
        e = min(n, b + chunk_rows)
        blk = col[b:e]
        np.add(np.arange(b, e, dtype=np.int32)[:, None], off32[None, :], out=blk)
        np.remainder(blk, np.int32(n), out=blk)
    return row_ptr, col.reshape(-1)
