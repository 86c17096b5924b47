"""Databases of several records (Section 2.2 joins a database's sequences into
one text): no alignment may cross from one record into the next, so the hit
set of a search equals the oracle's hits of every record searched alone, with
text positions shifted by the record's start (the separators count as text
positions).  Homologs are planted across record boundaries so that an
alignment crossing one would show up as an extra or a wrong hit; long ones
drive the wave walkers and the gapped domination window against a separator."""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae

pytestmark = pytest.mark.gpu


def per_record_oracle(recs, P, sub, sg, ss, H):
    js, ts, ss_ = [], [], []
    start = 0
    for rec in recs:
        j, t, s = oracle.sw_hits(rec, P, sub, sg, ss, H, threads=1)
        js.append(j)
        ts.append(t + start)
        ss_.append(s)
        start += rec.shape[0] + 1
    j, t, s = np.concatenate(js), np.concatenate(ts), np.concatenate(ss_)
    order = np.lexsort((t, j))
    return j[order], t[order], s[order]


def boundary_database(seed, sigma, k=24, lo=40, hi=2500, m=900, long_copy=0):
    """k random records and a query; query segments are copied (with a few substitutions) so
    that they run across record boundaries, and inside records."""
    rng = np.random.default_rng(seed)
    m = max(m, long_copy + 100)
    recs = [rng.integers(0, sigma, int(rng.integers(lo, hi)), dtype=np.uint8) for _ in range(k)]
    recs.insert(3, rng.integers(0, sigma, 1, dtype=np.uint8))      # one-character records
    recs.insert(9, rng.integers(0, sigma, 2, dtype=np.uint8))
    P = rng.integers(0, sigma, m, dtype=np.uint8)
    for r in range(0, len(recs) - 1, 2):
        a, b = recs[r], recs[r + 1]
        L = int(rng.integers(30, 120))
        y = int(rng.integers(0, m - 2 * L))
        cut = min(L, a.shape[0], b.shape[0])
        if cut < 4:
            continue
        a[-cut:] = P[y:y + cut]                 # the end of record r ...
        b[:cut] = P[y + cut:y + 2 * cut]        # ... continues the query at the start of record r+1
        b[cut // 2] = (b[cut // 2] + 1) % sigma
    for r in range(1, len(recs), 3):            # copies inside records
        rec = recs[r]
        L = int(min(rec.shape[0] // 2, rng.integers(40, 200)))
        if L < 10:
            continue
        x = int(rng.integers(0, rec.shape[0] - L + 1))
        y = int(rng.integers(0, m - L))
        rec[x:x + L] = P[y:y + L]
    if long_copy:
        # a long homolog split by a boundary in its middle
        a, b = recs[-2], recs[-1]
        h = long_copy // 2
        if a.shape[0] < h:
            recs[-2] = a = np.concatenate([a, rng.integers(0, sigma, h, dtype=np.uint8)])
        if b.shape[0] < h:
            recs[-1] = b = np.concatenate([rng.integers(0, sigma, h, dtype=np.uint8), b])
        y = int(rng.integers(0, m - long_copy))
        a[-h:] = P[y:y + h]
        b[:h] = P[y + h:y + 2 * h]
        for q in range(0, 2 * h, 37):
            (a if q < h else b)[q % h] ^= 1
    return recs, P


def assert_same(got, exp, what=""):
    assert got[0].shape == exp[0].shape, (what, got[0].shape, exp[0].shape)
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e, err_msg=what)


@pytest.mark.parametrize("seed,scheme,H", [(1, (1, -3, -5, -2), 14), (2, (1, -1, -5, -2), 16),
                                           (3, (2, -3, -4, -1), 26)])
def test_dna_records_match_per_record_oracle(seed, scheme, H):
    recs, P = boundary_database(seed, 4, long_copy=1200)
    sa, sb, sg, ss = scheme
    exp = per_record_oracle(recs, P, oracle.scoring_table(4, sa, sb), sg, ss, H)
    assert exp[0].shape[0] > 0
    idx = alae.Index.build_records(recs, "dna")
    print(f"records dna seed={seed} k={len(recs)} n={idx.info()['n']} scheme={scheme} H={H}", flush=True)
    st = alae.Stats()
    got = alae.search(idx, P, H, alae.make_scoring(*scheme), stats=st)
    assert_same(got, exp, f"seed {seed}")
    for opt in (dict(use_domination=False), dict(tail_split=False), dict(level_graph=8),
                dict(level_graph=3, tail_split=False)):
        assert_same(alae.search(idx, P, H, alae.make_scoring(*scheme), **opt), exp, str(opt))
    # every hit maps inside one record
    for t in got[1][:: max(1, got[1].shape[0] // 50)]:
        r, o = idx.record_of(int(t))
        assert o < recs[r].shape[0]


def test_protein_records_and_matrix_scoring():
    recs, P = boundary_database(4, 20, k=16, lo=30, hi=900, m=500, long_copy=600)
    exp = per_record_oracle(recs, P, oracle.scoring_table(20, 1, -3), -11, -1, 20)
    idx = alae.Index.build_records(recs, "protein")
    print(f"records protein k={len(recs)} n={idx.info()['n']}", flush=True)
    assert exp[0].shape[0] > 0
    assert_same(alae.search(idx, P, 20, alae.make_scoring(1, -3, -11, -1)), exp, "protein")
    rng = np.random.default_rng(5)
    B = rng.integers(-4, 2, (20, 20))
    B = np.triu(B) + np.triu(B, 1).T
    np.fill_diagonal(B, rng.integers(4, 9, 20))
    expm = per_record_oracle(recs, P, B.astype(np.int32), -11, -1, 30)
    assert_same(alae.search(idx, P, 30, alae.make_scoring(sg=-11, ss=-1, matrix=B)), expm, "matrix")


def test_records_batch_and_builders():
    recs, P = boundary_database(6, 4, k=30, m=1500)
    idx = alae.Index.build_records(recs, "dna", builder="gpu")
    host = alae.Index.build_records(recs, "dna", builder="host")
    assert idx.info()["C"] == host.info()["C"] and idx.info()["dollar_row"] == host.info()["dollar_row"]
    np.testing.assert_array_equal(idx.sa_end(), host.sa_end())
    np.testing.assert_array_equal(idx.bwt(), host.bwt())
    qs = [P[:400], P[400:1100], P[1100:]]
    res = alae.search_batch(idx, qs, 14)
    for i, q in enumerate(qs):
        assert_same(res[i], per_record_oracle(recs, q, oracle.scoring_table(4, 1, -3), -5, -2, 14), f"query {i}")
