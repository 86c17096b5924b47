"""Parity of the HIP search path against the CPU oracle (bit-exact hit sets).

Scores are integers, so every case compares the full sorted arrays
(query end, text end, score) element by element.
"""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu

PAPER_SCHEMES = [(1, -3, -5, -2), (1, -4, -5, -2), (1, -1, -5, -2), (1, -3, -2, -2)]


def _sub(sigma, sa, sb, matrix):
    return np.asarray(matrix, dtype=np.int32) if matrix is not None else oracle.scoring_table(sigma, sa, sb)


def run_pair(T, P, scheme, H, sigma=4, matrix=None, index=None, **opt):
    sa, sb, sg, ss = scheme
    idx = index if index is not None else alae.Index.build(T, "dna" if sigma == 4 else "protein")
    st = alae.Stats()
    got = alae.search(idx, P, H, alae.make_scoring(sa, sb, sg, ss, matrix), stats=st, **opt)
    exp = oracle.sw_hits(T, P, _sub(sigma, sa, sb, matrix), sg, ss, H, threads=8)
    return got, exp, st


def assert_same(got, exp):
    assert got[0].shape == exp[0].shape, (got[0].shape, exp[0].shape)
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e)


def planted_case(seed, n, m, sigma=4, n_plants=3, p_sub=0.1, p_indel=0.02):
    rng = np.random.default_rng(seed)
    T = rng.integers(0, sigma, size=n).astype(np.uint8)
    P = rng.integers(0, sigma, size=m).astype(np.uint8)
    srcs = []
    for _ in range(n_plants):
        L = int(rng.integers(min(m, 20), min(m, 120) + 1))
        y = int(rng.integers(0, m - L + 1))
        srcs.append(P[y:y + L])
    if n > 4 * sum(s.shape[0] for s in srcs) + 10:
        synth.plant_segments(rng, T, srcs, sigma, p_sub, p_indel)
    return T, P


@pytest.mark.parametrize("seed", range(12))
def test_random_small(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(200, 20000))
    m = int(rng.integers(5, 400))
    scheme = PAPER_SCHEMES[seed % 4]
    T, P = planted_case(seed, n, m)
    H = int(rng.integers(6, 20))
    got, exp, st = run_pair(T, P, scheme, H)
    print(f"seed={seed} n={n} m={m} scheme={scheme} H={H} hits={exp[0].shape[0]} stats={st.as_dict()}", flush=True)
    assert_same(got, exp)


@pytest.mark.parametrize("H", [4, 5, 8])
def test_low_threshold_many_hits(H):
    """H at or below q: hits already at the seed depth and from multi-occurrence nodes."""
    T, P = planted_case(7, 5000, 150)
    got, exp, _ = run_pair(T, P, (1, -3, -5, -2), H)
    assert exp[0].shape[0] > 100
    assert_same(got, exp)


@pytest.mark.parametrize("kind", ["periodic", "two_letters", "one_letter"])
def test_repetitive_texts(kind):
    """Highly repetitive texts: wide BWT ranges, hits spread over many occurrences."""
    rng = np.random.default_rng(3)
    if kind == "periodic":
        T = np.tile(np.array([0, 1, 2, 3, 3, 1], dtype=np.uint8), 500)
        P = np.concatenate([T[7:47], rng.integers(0, 4, 30).astype(np.uint8)])
    elif kind == "two_letters":
        T = rng.integers(0, 2, size=3000).astype(np.uint8)
        P = rng.integers(0, 2, size=80).astype(np.uint8)
    else:
        T = np.zeros(400, dtype=np.uint8)
        P = np.zeros(40, dtype=np.uint8)
    got, exp, _ = run_pair(T, P, (1, -3, -5, -2), 10)
    assert_same(got, exp)


def test_matrix_mode_dna():
    rng = np.random.default_rng(11)
    a = rng.integers(-4, 2, size=(4, 4))
    a = np.triu(a) + np.triu(a, 1).T
    np.fill_diagonal(a, [2, 3, 2, 4])
    T, P = planted_case(11, 8000, 200)
    got, exp, _ = run_pair(T, P, (0, 0, -4, -1), 12, matrix=a)
    assert exp[0].shape[0] > 0
    assert_same(got, exp)


def test_protein_match_mismatch():
    """The paper's protein scheme <1,-3,-11,-1> (Section 7.5) over 20 letters."""
    T, P = planted_case(12, 20000, 300, sigma=20, p_sub=0.2, p_indel=0.03)
    got, exp, _ = run_pair(T, P, (1, -3, -11, -1), 15, sigma=20)
    assert exp[0].shape[0] > 0
    assert_same(got, exp)


def test_protein_matrix_mode():
    rng = np.random.default_rng(13)
    a = rng.integers(-4, 3, size=(20, 20))
    a = np.triu(a) + np.triu(a, 1).T
    np.fill_diagonal(a, rng.integers(4, 12, size=20))
    T, P = planted_case(13, 6000, 150, sigma=20, p_sub=0.3, p_indel=0.03)
    got, exp, _ = run_pair(T, P, (0, 0, -11, -1), 40, sigma=20, matrix=a)
    assert exp[0].shape[0] > 0
    assert_same(got, exp)


@pytest.mark.parametrize("case", ["m1", "n1", "query_longer", "no_hits", "H1"])
def test_edge_cases(case):
    rng = np.random.default_rng(21)
    if case == "m1":
        T = rng.integers(0, 4, size=1000).astype(np.uint8)
        P = np.array([2], dtype=np.uint8)
        scheme, H = (3, -3, -5, -2), 3
    elif case == "n1":
        T = np.array([1], dtype=np.uint8)
        P = rng.integers(0, 4, size=50).astype(np.uint8)
        scheme, H = (1, -3, -5, -2), 1
    elif case == "query_longer":
        T = rng.integers(0, 4, size=300).astype(np.uint8)
        P = np.concatenate([rng.integers(0, 4, 200), T[50:250], rng.integers(0, 4, 300)]).astype(np.uint8)
        scheme, H = (1, -3, -5, -2), 20
    elif case == "no_hits":
        T = rng.integers(0, 4, size=2000).astype(np.uint8)
        P = rng.integers(0, 4, size=100).astype(np.uint8)
        scheme, H = (1, -3, -5, -2), 60
    else:
        T = rng.integers(0, 4, size=300).astype(np.uint8)
        P = rng.integers(0, 4, size=30).astype(np.uint8)
        scheme, H = (1, -3, -5, -2), 1
    got, exp, _ = run_pair(T, P, scheme, H)
    assert_same(got, exp)


@pytest.mark.parametrize("toggle", ["use_domination", "use_score_filter", "use_qprefix"])
def test_filter_ablation_identity(toggle):
    """Every filter can be switched off without changing the hits (exactness)."""
    T, P = planted_case(31, 15000, 300, n_plants=4)
    idx = alae.Index.build(T, "dna")
    got_on, exp, st_on = run_pair(T, P, (1, -3, -5, -2), 14, index=idx)
    st_off = alae.Stats()
    got_off = alae.search(idx, P, 14, alae.make_scoring(), stats=st_off, **{toggle: False})
    assert_same(got_on, exp)
    assert_same(got_off, exp)
    assert st_off.entries >= st_on.entries


def test_forced_capacity_retries():
    """Tiny frontier and hit buffers force overflow and re-runs; the hits stay the same."""
    T, P = planted_case(41, 12000, 250, n_plants=4)
    got, exp, st = run_pair(T, P, (1, -3, -5, -2), 12, entry_capacity=64, hit_capacity=16)
    assert st.retries > 0
    assert_same(got, exp)


def test_small_dna_and_planted():
    """The small DNA workload (text 1e5, query 1e3, <1,-3,-5,-2>, H=18) and its planted variant at lower H."""
    for planted, H in ((False, 18), (True, 18), (True, 12), (True, 10), (True, 8)):
        w = synth.small_dna(planted=planted, H=H)
        got, exp, st = run_pair(w["text"], w["queries"][0], (1, -3, -5, -2), H)
        print(f"small DNA planted={planted} H={H} hits={exp[0].shape[0]} entries={st.entries}", flush=True)
        assert_same(got, exp)


def test_batch_matches_single():
    T, P = planted_case(51, 10000, 200)
    idx = alae.Index.build(T, "dna")
    rng = np.random.default_rng(52)
    qs = [P, rng.integers(0, 4, 50).astype(np.uint8), P[30:150].copy()]
    res = alae.search_batch(idx, qs, 12)
    for q, r in zip(qs, res):
        assert_same(r, alae.search(idx, q, 12))
        assert_same(r, oracle.sw_hits(T, q, oracle.scoring_table(4, 1, -3), -5, -2, 12, threads=8))


def test_device_resident_path():
    import torch

    T, P = planted_case(61, 10000, 200)
    idx = alae.Index.build(T, "dna")
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    cnt = ws.search_device(dq, 12)
    keys, scores = ws.result_torch()
    torch.cuda.synchronize()
    keys = keys.cpu().numpy()
    got = ((keys >> 32).astype(np.int64), (keys & 0xFFFFFFFF).astype(np.int64), scores.cpu().numpy().astype(np.int64))
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, 1, -3), -5, -2, 12, threads=8)
    assert cnt == exp[0].shape[0]
    assert_same(got, exp)
    # a second search on the same workspace, smaller query
    cnt2 = ws.search_device(dq[20:120].contiguous(), 10)
    exp2 = oracle.sw_hits(T, P[20:120], oracle.scoring_table(4, 1, -3), -5, -2, 10, threads=8)
    assert cnt2 == exp2[0].shape[0]
    ws.free()


@pytest.mark.parametrize("scheme", [(1, -3, -5, -2), (1, -1, -5, -2), (2, -3, -4, -1)])
def test_long_homolog_wide_rows(scheme):
    """A long mutated copy makes gap wedges hundreds of columns wide: rows are
    walked by whole waves over several 64-entry rounds."""
    rng = np.random.default_rng(71)
    m = 4000
    P = rng.integers(0, 4, size=m).astype(np.uint8)
    T = rng.integers(0, 4, size=30000).astype(np.uint8)
    synth.plant_segments(rng, T, [P[200:3200], P[3300:3900]], 4, 0.10, 0.02)
    H = 30 if scheme[0] == 1 else 60
    got, exp, st = run_pair(T, P, scheme, H)
    print(f"scheme={scheme} hits={exp[0].shape[0]} stats={st.as_dict()}", flush=True)
    assert st.promoted > 0 and st.wide_steps > 0
    assert_same(got, exp)


def test_domination_switch_same_hits_on_homologs():
    """The gapped domination test removes interior starts inside homologs without changing hits."""
    rng = np.random.default_rng(72)
    m = 2000
    P = rng.integers(0, 4, size=m).astype(np.uint8)
    T = rng.integers(0, 4, size=40000).astype(np.uint8)
    synth.plant_segments(rng, T, [P[100:1100], P[1200:1900], P[300:800]], 4, 0.15, 0.02)
    idx = alae.Index.build(T, "dna")
    on, exp, st_on = run_pair(T, P, (1, -3, -5, -2), 30, index=idx)
    st_off = alae.Stats()
    off = alae.search(idx, P, 30, alae.make_scoring(), stats=st_off, use_domination=False)
    assert_same(on, exp)
    assert_same(off, exp)
    assert st_on.dominated + st_on.dominated_gapped > 0
    assert st_on.entries < st_off.entries


@pytest.mark.parametrize("case", ["planted", "repeats", "batch"])
def test_tail_split_identity(case):
    """The frontier's tail walked as one chain per occurrence gives the same hits as
    taking every level through the FM-index (and as the oracle)."""
    rng = np.random.default_rng(77)
    if case == "repeats":
        unit = rng.integers(0, 4, size=150).astype(np.uint8)
        T = np.concatenate([unit, rng.integers(0, 4, size=40).astype(np.uint8)] * 40)
        mut = rng.random(T.shape[0]) < 0.05
        T[mut] = rng.integers(0, 4, size=int(mut.sum())).astype(np.uint8)
        P = np.concatenate([unit[30:130], rng.integers(0, 4, size=200).astype(np.uint8)])
    else:
        T, P = planted_case(78, 200000, 500, n_plants=5)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(1, -3, -5, -2)
    H = 16
    if case == "batch":
        qs = [P, P[100:400].copy(), rng.integers(0, 4, size=80).astype(np.uint8)]
        on = alae.search_batch(idx, qs, H, sc)
        off = alae.search_batch(idx, qs, H, sc, tail_split=False)
        for q, a, b in zip(qs, on, off):
            assert_same(a, b)
            assert_same(a, oracle.sw_hits(T, q, oracle.scoring_table(4, 1, -3), -5, -2, H, threads=8))
        return
    st_on, st_off = alae.Stats(), alae.Stats()
    got_on = alae.search(idx, P, H, sc, stats=st_on)
    got_off = alae.search(idx, P, H, sc, stats=st_off, tail_split=False)
    print(f"{case}: tail chains {st_on.tail_chains} at depth {st_on.tail_depth}, levels {st_on.levels} "
          f"against {st_off.levels}; hit records {st_on.emitted} against {st_off.emitted}", flush=True)
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, 1, -3), -5, -2, H, threads=8)
    assert_same(got_on, exp)
    assert_same(got_off, exp)
    assert st_off.tail_chains == 0
    if case == "planted":
        assert st_on.tail_chains > 0 and st_on.levels < st_off.levels
