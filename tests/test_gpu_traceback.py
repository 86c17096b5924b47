"""Alignment starts (A(i,j).pos) and transcripts of reported hits on the GPU
against the oracle: the start must equal the oracle's (largest text start,
then largest query start, among the optimal alignments ending at the cell);
the transcript must consume exactly T[x..t] and P[y..j] and score A(t, j)
(several optimal transcripts may exist, so it is checked for validity)."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def sample_hits(res, k, seed):
    j, t, s = res
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(j.shape[0], size=min(k, j.shape[0]), replace=False).tolist())
    pick |= set(np.argsort(-s)[:20].tolist())  # the best cells: the longest alignments
    pick = sorted(pick)
    return j[pick], t[pick], s[pick]


def check(idx, T, P, sub, sg, ss, j, t, s, scoring):
    out = alae.traceback(idx, P, j, t, s, scoring)
    subl = np.asarray(sub).tolist()
    for a, jj, tt, S in zip(out, j.tolist(), t.tolist(), s.tolist()):
        assert a["status"] == 0, (jj, tt, S, a)
        exp = oracle.alignment_start(T, P, sub, sg, ss, tt, jj)
        assert exp is not None and exp[2] == S
        assert (a["text_start"], a["query_start"]) == exp[:2], (jj, tt, S, a, exp)
        ops = a["ops"]
        x, y = a["text_start"], a["query_start"]
        assert ops.count("M") + ops.count("D") == tt - x + 1
        assert ops.count("M") + ops.count("I") == jj - y + 1
        assert brute.score_transcript(list(T[x:tt + 1]), list(P[y:jj + 1]), ops, subl, sg, ss) == S
    return out


@pytest.mark.parametrize("scheme,H", [((1, -3, -5, -2), 12), ((1, -1, -5, -2), 16), ((2, -3, -4, -1), 24)])
def test_traceback_planted_dna(scheme, H):
    w = synth.small_dna(planted=True, H=12)
    T, P = w["text"], w["queries"][0]
    rng = np.random.default_rng(3)
    T = T.copy()
    T[60_000:60_700] = P[200:900]  # a long homolog: windows must grow
    for q in range(60_000, 60_700, 29):
        T[q] = (T[q] + 1) % 4
    sa, sb, sg, ss = scheme
    sc = alae.make_scoring(*scheme)
    idx = alae.Index.build(T, "dna")
    res = alae.search(idx, P, H, sc)
    assert res[0].shape[0] > 0
    j, t, s = sample_hits(res, 120, 1)
    print(f"traceback dna {scheme} H={H}: {j.shape[0]} of {res[0].shape[0]} hits", flush=True)
    check(idx, T, P, oracle.scoring_table(4, sa, sb), sg, ss, j, t, s, sc)
    # a score that is not A(t, j), and a cell outside the text, are refused per cell
    bad = alae.traceback(idx, P, [int(j[0]), 0], [int(t[0]), T.shape[0] + 5], [int(s[0]) + 1, 30], sc)
    assert [b["status"] for b in bad] == [1, 1]
    del rng


def test_traceback_protein_matrix_and_records():
    rng = np.random.default_rng(8)
    B = rng.integers(-4, 2, (20, 20))
    B = np.triu(B) + np.triu(B, 1).T
    np.fill_diagonal(B, rng.integers(4, 9, 20))
    recs = [rng.integers(0, 20, int(rng.integers(200, 3000)), dtype=np.uint8) for _ in range(8)]
    P = rng.integers(0, 20, 400, dtype=np.uint8)
    recs[2][:150] = P[100:250]          # a homolog at the very start of a record
    recs[5][-200:] = P[150:350]
    recs[6][500:560] = P[0:60]
    idx = alae.Index.build_records(recs, "protein")
    sc = alae.make_scoring(sg=-11, ss=-1, matrix=B)
    res = alae.search(idx, P, 40, sc)
    assert res[0].shape[0] > 0
    j, t, s = sample_hits(res, 80, 2)
    # the oracle on the concatenated text with separators is the oracle record by record
    starts = np.cumsum([0] + [r.shape[0] + 1 for r in recs[:-1]])
    out = alae.traceback(idx, P, j, t, s, sc)
    subl = B.tolist()
    for a, jj, tt, S in zip(out, j.tolist(), t.tolist(), s.tolist()):
        r = int(np.searchsorted(starts, tt, side="right") - 1)
        exp = oracle.alignment_start(recs[r], P, B.astype(np.int32), -11, -1, tt - int(starts[r]), jj)
        assert a["status"] == 0 and exp[2] == S
        assert (a["text_start"] - int(starts[r]), a["query_start"]) == exp[:2]
        x = a["text_start"] - int(starts[r])
        assert brute.score_transcript(list(recs[r][x:tt - int(starts[r]) + 1]), list(P[a["query_start"]:jj + 1]),
                                      a["ops"], subl, -11, -1) == S
