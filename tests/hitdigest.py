"""Digests of hit sets by text-end bin, for parity at sizes where storing
every expected hit is impractical.

A hit is the triple (query end j, text end t, score s).  Each hit gets two
64-bit hashes (splitmix64 finalisers of the packed record); a bin of text
ends is summarised by (count, sum of the first hashes, sum of the second
hashes), sums taken modulo 2^64.  Hit sets hold one record per (j, t), so
equal digests mean equal sets except with probability about 2^-128 per bin;
the digest does not depend on the order of the records.

Test infrastructure: used by ``tests/golden/make_digests.py`` (on oracle
output) and by the GPU tests (on device output).  It holds none of the
search method's arithmetic.
"""
from __future__ import annotations

import numpy as np

_C1 = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_K2 = np.uint64(0xD6E8FEB86659FD93)


def mix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014), elementwise on uint64."""
    z = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z += _C1
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def record_hashes(j, t, s):
    """Two 64-bit hashes per hit; j < 2^24, t < 2^40, |s| < 2^31."""
    j = np.asarray(j, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    key = (j.astype(np.uint64) << np.uint64(40)) | t.astype(np.uint64)
    h1 = mix64(mix64(key) ^ (s.astype(np.uint64) & np.uint64(0xFFFFFFFF)))
    h2 = mix64(h1 ^ _K2)
    return h1, h2


def _binned_sum_mod64(vals: np.ndarray, bins: np.ndarray, nbins: int) -> list:
    """Exact per-bin sums of uint64 values modulo 2^64: four 16-bit limbs, each
    summed in float64 (exact while count * 2^16 < 2^53)."""
    out = [0] * nbins
    for k in range(4):
        limb = ((vals >> np.uint64(16 * k)) & np.uint64(0xFFFF)).astype(np.float64)
        sums = np.bincount(bins, weights=limb, minlength=nbins)
        for b in range(nbins):
            out[b] += int(sums[b]) << (16 * k)
    return [v & ((1 << 64) - 1) for v in out]


def digest_by_bins(j, t, s, edges):
    """Digests of the hits whose text end t lies in [edges[b], edges[b+1]) for
    every b; hits outside [edges[0], edges[-1]) are ignored.  Returns a list of
    (count, sum1, sum2)."""
    edges = np.asarray(edges, dtype=np.int64)
    nb = edges.shape[0] - 1
    t = np.asarray(t, dtype=np.int64)
    sel = (t >= edges[0]) & (t < edges[-1])
    j, t, s = np.asarray(j)[sel], t[sel], np.asarray(s)[sel]
    if t.shape[0] == 0:
        return [(0, 0, 0)] * nb
    bins = (np.searchsorted(edges, t, side="right") - 1).astype(np.int64)
    h1, h2 = record_hashes(j, t, s)
    cnt = np.bincount(bins, minlength=nb)
    s1 = _binned_sum_mod64(h1, bins, nb)
    s2 = _binned_sum_mod64(h2, bins, nb)
    return [(int(cnt[b]), s1[b], s2[b]) for b in range(nb)]


def digest(j, t, s):
    """Digest of a whole hit set."""
    h1, h2 = record_hashes(j, t, s)
    with np.errstate(over="ignore"):
        return (int(np.asarray(j).shape[0]), int(np.sum(h1, dtype=np.uint64)), int(np.sum(h2, dtype=np.uint64)))


def read_digest_file(path):
    """Lines 'key... count sum1 sum2' (integers) after '#' comments; returns a
    list of integer tuples."""
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(tuple(int(x) for x in line.split()))
    return rows


# The same hashes with torch int64 tensors (two's complement, products taken
# modulo 2^64; logical right shifts by masking the sign extension), so that a
# test can digest a result where it lies, on the GPU.
def _signed(v: int) -> int:
    return v - (1 << 64) if v >= (1 << 63) else v


def _mix64_torch(z):
    z = z + _signed(0x9E3779B97F4A7C15)
    z = z ^ ((z >> 30) & ((1 << 34) - 1))
    z = z * _signed(0xBF58476D1CE4E5B9)
    z = z ^ ((z >> 27) & ((1 << 37) - 1))
    z = z * _signed(0x94D049BB133111EB)
    z = z ^ ((z >> 31) & ((1 << 33) - 1))
    return z


def record_hashes_torch(j, t, s):
    """record_hashes for int64 torch tensors; returns int64 tensors holding the same bits."""
    key = (j << 40) | t
    h1 = _mix64_torch(_mix64_torch(key) ^ (s & 0xFFFFFFFF))
    h2 = _mix64_torch(h1 ^ _signed(0xD6E8FEB86659FD93))
    return h1, h2


def unsigned(v: int) -> int:
    return v & ((1 << 64) - 1)
