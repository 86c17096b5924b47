"""CPU oracle for the exact local-alignment search.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU search path (``paper_1208_0274_amd``) and never imports it.

Contents
--------
* :func:`sw_hits` -- plain Smith-Waterman-Gotoh over the whole m x n matrix
  in C (``sw_oracle.c``), returning every (query end, text end, A) with
  A >= H, sorted by (query end, text end).  Definition: Section 2.1 (local
  alignment problem) and Algorithm 1 (initialise to 0, keep the max, return
  the entries that reach H).
* :func:`sw_matrix` -- the full A matrix for small inputs.
* :func:`lmax` -- Equation 1 (Theorem 1), used by the chunked oracle.
* :mod:`oracle.brute` -- exhaustive transcript enumeration, sim(), the
  literal M_X/G_a/G_b recurrences of Section 2.2 and Algorithm 1 BASIC.
* :func:`scoring_table` -- the scoring scheme of Section 2.1 as a table.

Pins (all in ``tests/test_oracle.py``): exhaustive search on strings of at
most 8 characters, Algorithm 1 over the Section 2.2 recurrences, Figure 1,
sim(AAACG, AACCG) = 1, the Section 3.1.2 example, and invariants
(reversal, transposition, H-monotonicity, planted copies, m = 1, the
ungapped closed form, chunked == unchunked).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

DNA = "ACGT"
PROTEIN = "ARNDCQEGHILKMFPSTWYV"


class _Hits(ctypes.Structure):
    _fields_ = [
        ("qend", ctypes.POINTER(ctypes.c_int64)),
        ("tend", ctypes.POINTER(ctypes.c_int64)),
        ("score", ctypes.POINTER(ctypes.c_int64)),
        ("count", ctypes.c_int64),
        ("cap", ctypes.c_int64),
        ("cells", ctypes.c_int64),
    ]


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_sw_hits.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, i32p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_Hits)]
        lib.oracle_sw_hits.restype = ctypes.c_int
        lib.oracle_sw_matrix.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, i32p, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_sw_matrix.restype = ctypes.c_int
        lib.oracle_lmax.argtypes = [ctypes.c_int64] * 5
        lib.oracle_lmax.restype = ctypes.c_int64
        lib.oracle_global_suffix.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, i32p, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_global_suffix.restype = ctypes.c_int
        lib.oracle_hits_free.argtypes = [ctypes.POINTER(_Hits)]
        lib.oracle_hits_free.restype = None
        _LIB = lib
    return _LIB


def scoring_table(sigma: int, sa: int, sb: int) -> np.ndarray:
    """Section 2.1: an identical pair scores sa, any other pair sb."""
    tab = np.full((sigma, sigma), sb, dtype=np.int32)
    np.fill_diagonal(tab, sa)
    return tab


def encode(s: str, alphabet: str = DNA) -> np.ndarray:
    lut = {c: i for i, c in enumerate(alphabet)}
    return np.array([lut[c] for c in s.upper()], dtype=np.uint8)


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def lmax(m: int, smax: int, sg: int, ss: int, H: int) -> int:
    """Equation 1: L_max = max(m, m + floor((H - (smax*m + sg)) / ss))."""
    return int(_lib().oracle_lmax(m, smax, sg, ss, H))


def sw_hits(T, P, sub, sg: int, ss: int, H: int, t_lo: int = 0, t_hi: int | None = None,
            threads: int = 1, return_cells: bool = False):
    """All (j, i, A(i,j)) with A >= H and text end i in [t_lo, t_hi).

    T and P are code arrays (uint8), sub a sigma x sigma table indexed
    [text char][query char].  Indices are 0-based inclusive ends.  The
    result is three int64 arrays sorted by (query end j, text end i).
    """
    lib = _lib()
    T, Tp = _u8(T)
    P, Pp = _u8(P)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    n = int(T.shape[0])
    if t_hi is None:
        t_hi = n
    out = _Hits()
    rc = lib.oracle_sw_hits(Tp, n, Pp, int(P.shape[0]), sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            int(sub.shape[0]), int(sg), int(ss), int(H), int(t_lo), int(t_hi),
                            int(threads), ctypes.byref(out))
    if rc != 0:
        lib.oracle_hits_free(ctypes.byref(out))
        raise RuntimeError(f"oracle_sw_hits failed with code {rc}")
    cnt = int(out.count)
    if cnt:
        j = np.ctypeslib.as_array(out.qend, shape=(cnt,)).copy()
        i = np.ctypeslib.as_array(out.tend, shape=(cnt,)).copy()
        s = np.ctypeslib.as_array(out.score, shape=(cnt,)).copy()
    else:
        j = np.zeros(0, np.int64)
        i = np.zeros(0, np.int64)
        s = np.zeros(0, np.int64)
    cells = int(out.cells)
    lib.oracle_hits_free(ctypes.byref(out))
    order = np.lexsort((i, j))
    res = (j[order], i[order], s[order])
    if return_cells:
        return res, cells
    return res


def global_suffix(T, P, sub, sg: int, ss: int) -> np.ndarray:
    """G[a, b] = sim(T[-a:], P[-b:]) (the empty suffix for a or b = 0): the best global
    alignment score of the last a text and last b query characters (Section 2.1)."""
    lib = _lib()
    T, Tp = _u8(T)
    P, Pp = _u8(P)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    a, b = int(T.shape[0]), int(P.shape[0])
    out = np.zeros((a + 1) * (b + 1), dtype=np.int64)
    rc = lib.oracle_global_suffix(Tp, a, Pp, b, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(sub.shape[0]),
                                  int(sg), int(ss), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError(f"oracle_global_suffix failed with code {rc}")
    return out.reshape(a + 1, b + 1)


def alignment_start(T, P, sub, sg: int, ss: int, t: int, j: int):
    """The start (x, y) of the optimal local alignment ending at text end t and query end j
    with the largest x, and among those the largest y (the paper's A(i,j).pos, one reading of
    it made unique), and its score A(t, j).  Every alignment scoring A(t, j) >= 1 spans at
    most L_max text characters (Equation 1 with the j + 1 query characters available), so
    only that many text characters before t are looked at (with threshold 1, which bounds
    every alignment of positive score).  Returns None when A(t, j) = 0."""
    P = np.asarray(P)
    T = np.asarray(T)
    smax = int(np.max(sub))
    L = lmax(j + 1, smax, sg, ss, 1)
    lo = max(0, t - L + 1)
    G = global_suffix(T[lo:t + 1], P[:j + 1], sub, sg, ss)
    S = int(G.max())
    if S <= 0:
        return None
    cand = np.argwhere(G == S)
    cand = cand[(cand[:, 0] > 0) & (cand[:, 1] > 0)]
    a = int(cand[:, 0].min())
    b = int(cand[cand[:, 0] == a][:, 1].min())
    return t - a + 1, j - b + 1, S


def sw_matrix(T, P, sub, sg: int, ss: int) -> np.ndarray:
    """The (n+1) x (m+1) matrix A of the Smith-Waterman-Gotoh recurrence."""
    lib = _lib()
    T, Tp = _u8(T)
    P, Pp = _u8(P)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    n, m = int(T.shape[0]), int(P.shape[0])
    out = np.zeros((n + 1) * (m + 1), dtype=np.int64)
    rc = lib.oracle_sw_matrix(Tp, n, Pp, m, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              int(sub.shape[0]), int(sg), int(ss),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError(f"oracle_sw_matrix failed with code {rc}")
    return out.reshape(n + 1, m + 1)
