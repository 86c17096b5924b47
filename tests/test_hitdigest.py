"""The hit digest used for full-size parity: its numpy form (which writes the
stored oracle digests) and its torch form (which digests device results) give
the same bits, per-bin sums are exact modulo 2^64, and the digest tells sets
apart that differ in one field of one record."""
import numpy as np
import torch

from hitdigest import digest, digest_by_bins, record_hashes, record_hashes_torch, unsigned

M64 = (1 << 64) - 1


def _records(n, seed):
    rng = np.random.default_rng(seed)
    j = rng.integers(0, 1 << 24, n, dtype=np.int64)
    t = rng.integers(0, 1 << 40, n, dtype=np.int64)
    s = rng.integers(1, 1 << 31, n, dtype=np.int64)
    return j, t, s


def test_torch_hashes_equal_numpy_hashes():
    j, t, s = _records(5000, 1)
    h1, h2 = record_hashes(j, t, s)
    g1, g2 = record_hashes_torch(torch.from_numpy(j), torch.from_numpy(t), torch.from_numpy(s))
    assert [unsigned(int(v)) for v in g1] == [int(v) for v in h1]
    assert [unsigned(int(v)) for v in g2] == [int(v) for v in h2]


def test_binned_sums_are_exact():
    j, t, s = _records(20000, 2)
    t = t % 1000
    edges = [0, 100, 250, 251, 700, 1000]
    got = digest_by_bins(j, t, s, edges)
    h1, h2 = record_hashes(j, t, s)
    for b in range(len(edges) - 1):
        sel = (t >= edges[b]) & (t < edges[b + 1])
        want = (int(sel.sum()), sum(int(v) for v in h1[sel]) & M64, sum(int(v) for v in h2[sel]) & M64)
        assert got[b] == want


def test_digest_sees_one_changed_field():
    j, t, s = _records(1000, 3)
    base = digest(j, t, s)
    for arr in (j, t, s):
        arr[17] += 1
        assert digest(j, t, s) != base
        arr[17] -= 1
    assert digest(j, t, s) == base
    order = np.random.default_rng(0).permutation(1000)
    assert digest(j[order], t[order], s[order]) == base
