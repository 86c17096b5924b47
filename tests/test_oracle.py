"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own recurrence: exhaustive
search, the literal recurrences of Section 2.2 run through Algorithm 1,
values printed in the paper, closed forms and invariants.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))

# The four scoring schemes of Section 7.4 (<s_a, s_b, s_g, s_s>).
PAPER_SCHEMES = [(1, -3, -5, -2), (1, -4, -5, -2), (1, -1, -5, -2), (1, -3, -2, -2)]


def table(sigma, sa, sb):
    return oracle.scoring_table(sigma, sa, sb)


def sym_random_matrix(rng, sigma):
    a = rng.integers(-4, 3, size=(sigma, sigma))
    a = np.triu(a) + np.triu(a, 1).T
    np.fill_diagonal(a, rng.integers(1, 6, size=sigma))
    return a.astype(np.int32)


def load_fig1():
    rows = []
    with open(os.path.join(HERE, "golden", "fig1_gcta_gctag.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows.append(parts)
    return rows


def _val(tok):
    if tok == "-inf":
        return float("-inf")
    if tok == ".":
        return None
    return int(tok)


def test_figure1_mx_recurrences():
    """Figure 1 (Section 2.2): every printed M value; every printed G_a and G_b
    except the one typo cell G_b(2,5)."""
    X = oracle.encode("GCTA")
    P = oracle.encode("GCTAG")
    M, Ga, Gb = brute.mx_matrix(X, P, table(4, 1, -3), -5, -2)
    rows = load_fig1()
    assert len(rows) == 30
    for parts in rows:
        i, j = int(parts[0]), int(parts[1])
        m_v, ga_v, gb_v = _val(parts[2]), _val(parts[3]), _val(parts[4])
        typo = len(parts) > 5 and parts[5] == "typo"
        assert M[i][j] == m_v, (i, j)
        if ga_v is not None:
            assert Ga[i][j] == ga_v, (i, j)
        if gb_v is not None:
            if typo:
                assert Gb[i][j] == -9 and gb_v == -7
            else:
                assert Gb[i][j] == gb_v, (i, j)
    # the worked example under Figure 1: G_a(4,3) = -4, G_b(4,3) = -14, M = -4
    assert (Ga[4][3], Gb[4][3], M[4][3]) == (-4, -14, -4)


def test_sim_example_section21():
    """Section 2.1: sim(AAACG, AACCG) = 1 under <1,-3,-5,-2>."""
    assert brute.sim(oracle.encode("AAACG"), oracle.encode("AACCG"), table(4, 1, -3), -5, -2) == 1


def test_score_filter_example_section312():
    """Section 3.1.2: aligning GCTA against GCTAG, only the diagonal entries are
    meaningful, and with H = 3 the cells reaching H are (3,3) with 3 and (4,4)
    with 4 (1-based)."""
    j, i, s = oracle.sw_hits(oracle.encode("GCTA"), oracle.encode("GCTAG"), table(4, 1, -3), -5, -2, 3)
    assert list(zip(j.tolist(), i.tolist(), s.tolist())) == [(2, 2, 3), (3, 3, 4)]


def test_lmax_equation1():
    """Equation 1.  Section 8 of the survey's reading: m=1000, <1,-3,-5,-2>, H=18 -> 1488;
    m=1e5, H=30 -> 149982; protein m=5000, smax=11, <-11,-1>, H=45 -> 59944."""
    assert oracle.lmax(1000, 1, -5, -2, 18) == 1000 + (1000 - 5 - 18) // 2
    assert oracle.lmax(1000, 1, -5, -2, 18) == 1488
    assert oracle.lmax(100000, 1, -5, -2, 30) == 149982
    assert oracle.lmax(5000, 11, -11, -1, 45) == 59944
    # H above the best possible score: the bound falls back to m
    assert oracle.lmax(10, 1, -5, -2, 100) == 10


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_small(seed):
    """Exhaustive transcript enumeration (Section 2.1 definition) on random
    strings of at most 6 characters, full A matrix, several schemes."""
    rng = np.random.default_rng(1000 + seed)
    sigma = [4, 4, 3, 2, 4, 20][seed]
    n = int(rng.integers(1, 7))
    m = int(rng.integers(1, 7))
    T = rng.integers(0, sigma, size=n).astype(np.uint8)
    P = rng.integers(0, sigma, size=m).astype(np.uint8)
    if seed == 4:
        sub = sym_random_matrix(rng, sigma)
        sg, ss = -2, -1
    else:
        sa, sb, sg, ss = PAPER_SCHEMES[seed % 4]
        sub = table(sigma, sa, sb)
    A_or = oracle.sw_matrix(T, P, sub, sg, ss)
    A_bf = np.array(brute.brute_A(T, P, sub.tolist(), sg, ss))
    np.testing.assert_array_equal(A_or, A_bf)


def test_exhaustive_eight_chars():
    """Exhaustive search at the size limit: 8 x 8 with a gap-friendly scheme (the
    corner cell by per-substring enumeration, the full matrix by prefix enumeration)."""
    T = oracle.encode("GATTACAG")
    P = oracle.encode("GATACCAG")
    sub = table(4, 2, -1)
    A_or = oracle.sw_matrix(T, P, sub, -1, -1)
    best = 0
    for x in range(1, 9):
        for y in range(1, 9):
            best = max(best, brute.sim(T[x - 1:], P[y - 1:], sub.tolist(), -1, -1))
    assert A_or[8, 8] == best
    np.testing.assert_array_equal(A_or, np.array(brute.brute_A_prefixes(T, P, sub.tolist(), -1, -1)))


@pytest.mark.parametrize("seed", range(4))
def test_prefix_enumeration_equals_substring_enumeration(seed):
    """The prefix enumeration visits every alignment once; on small strings its A equals
    the per-substring enumeration's cell for cell."""
    rng = np.random.default_rng(2000 + seed)
    sigma = [4, 3, 2, 20][seed]
    T = rng.integers(0, sigma, size=int(rng.integers(1, 6))).astype(np.uint8)
    P = rng.integers(0, sigma, size=int(rng.integers(1, 6))).astype(np.uint8)
    sa, sb, sg, ss = PAPER_SCHEMES[seed % 4]
    sub = table(sigma, sa, sb).tolist()
    assert brute.brute_A_prefixes(T, P, sub, sg, ss) == brute.brute_A(T, P, sub, sg, ss)


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_full_matrix_up_to_eight(seed):
    """Every alignment of every substring pair enumerated, strings of 7 and 8 characters,
    the full A matrix against the oracle, under the paper's schemes and a random matrix."""
    rng = np.random.default_rng(3000 + seed)
    sigma = [4, 4, 2, 3, 4, 20][seed]
    n = int(rng.integers(7, 9))
    m = int(rng.integers(7, 9))
    T = rng.integers(0, sigma, size=n).astype(np.uint8)
    P = rng.integers(0, sigma, size=m).astype(np.uint8)
    if seed == 4:
        sub = sym_random_matrix(rng, sigma)
        sg, ss = -2, -1
    else:
        sa, sb, sg, ss = PAPER_SCHEMES[seed % 4]
        sub = table(sigma, sa, sb)
    np.testing.assert_array_equal(oracle.sw_matrix(T, P, sub, sg, ss),
                                  np.array(brute.brute_A_prefixes(T, P, sub.tolist(), sg, ss)))


@pytest.mark.parametrize("seed", range(8))
def test_algorithm1_basic(seed):
    """Algorithm 1 (BASIC) over the literal Section 2.2 recurrences gives the
    same A as the oracle, on strings long enough to hold gaps."""
    rng = np.random.default_rng(2000 + seed)
    sigma = 4 if seed < 6 else 20
    n = int(rng.integers(5, 25))
    m = int(rng.integers(5, 25))
    T = rng.integers(0, sigma, size=n).astype(np.uint8)
    P = rng.integers(0, sigma, size=m).astype(np.uint8)
    if seed % 3 == 2 and n > 8 and m > 8:
        T[2:8] = P[1:7]
    if seed == 7:
        sub = sym_random_matrix(rng, sigma)
        sg, ss = -3, -1
    else:
        sa, sb, sg, ss = PAPER_SCHEMES[seed % 4]
        sub = table(sigma, sa, sb)
    A_or = oracle.sw_matrix(T, P, sub, sg, ss)
    A_basic = np.array(brute.basic_A(T, P, sub.tolist(), sg, ss))
    np.testing.assert_array_equal(A_or, A_basic)


def _hitset(res):
    j, i, s = res
    return set(zip(j.tolist(), i.tolist(), s.tolist()))


@pytest.mark.parametrize("seed", range(4))
def test_reversal_invariant(seed):
    """The best score over all cells is unchanged when both strings are reversed."""
    rng = np.random.default_rng(3000 + seed)
    T = rng.integers(0, 4, size=300).astype(np.uint8)
    P = rng.integers(0, 4, size=80).astype(np.uint8)
    T[100:160] = P[10:70]
    sa, sb, sg, ss = PAPER_SCHEMES[seed]
    sub = table(4, sa, sb)
    a = oracle.sw_matrix(T, P, sub, sg, ss).max()
    b = oracle.sw_matrix(T[::-1].copy(), P[::-1].copy(), sub, sg, ss).max()
    assert a == b and a >= 20


@pytest.mark.parametrize("seed", range(3))
def test_transposition_invariant(seed):
    """For symmetric scoring, hits(T, P) equals hits(P, T) with the ends swapped."""
    rng = np.random.default_rng(4000 + seed)
    T = rng.integers(0, 4, size=400).astype(np.uint8)
    P = rng.integers(0, 4, size=150).astype(np.uint8)
    T[50:120] = P[20:90]
    T[200:230] = P[100:130]
    sa, sb, sg, ss = PAPER_SCHEMES[seed]
    sub = table(4, sa, sb)
    h1 = _hitset(oracle.sw_hits(T, P, sub, sg, ss, 8))
    j, i, s = oracle.sw_hits(P, T, sub, sg, ss, 8)
    h2 = set(zip(i.tolist(), j.tolist(), s.tolist()))
    assert h1 == h2 and len(h1) > 0


def test_h_monotone():
    """hits(H2) is exactly the subset of hits(H1) scoring >= H2 (H1 <= H2)."""
    rng = np.random.default_rng(5)
    T = rng.integers(0, 4, size=2000).astype(np.uint8)
    P = rng.integers(0, 4, size=200).astype(np.uint8)
    T[500:600] = P[50:150]
    sub = table(4, 1, -3)
    lo = oracle.sw_hits(T, P, sub, -5, -2, 6)
    for H2 in (7, 10, 25, 60):
        hi = oracle.sw_hits(T, P, sub, -5, -2, H2)
        assert _hitset(hi) == {h for h in _hitset(lo) if h[2] >= H2}


def test_planted_exact_copy():
    """An exact copy of P[y..y+L-1] at T[t..] gives A(t+L-1, y+L-1) >= L*s_a."""
    rng = np.random.default_rng(6)
    T = rng.integers(0, 4, size=1000).astype(np.uint8)
    P = rng.integers(0, 4, size=300).astype(np.uint8)
    L, y, t = 120, 77, 400
    T[t:t + L] = P[y:y + L]
    A = oracle.sw_matrix(T, P, table(4, 1, -3), -5, -2)
    assert A[t + L, y + L] >= L


def test_single_query_char():
    """m = 1: the hits are exactly the matching text positions, each with s_a."""
    rng = np.random.default_rng(7)
    T = rng.integers(0, 4, size=500).astype(np.uint8)
    P = np.array([2], dtype=np.uint8)
    j, i, s = oracle.sw_hits(T, P, table(4, 3, -3), -5, -2, 3)
    assert i.tolist() == np.nonzero(T == 2)[0].tolist()
    assert set(s.tolist()) == {3} and set(j.tolist()) == {0}


def test_ungapped_closed_form():
    """With a prohibitive gap-open cost, A(i,j) is the best suffix sum along the
    diagonal through (i,j): max(0, S(i) - min over k<i of S(k)) where S is the
    prefix sum of substitution scores on that diagonal."""
    rng = np.random.default_rng(8)
    n, m = 60, 45
    T = rng.integers(0, 4, size=n).astype(np.uint8)
    P = rng.integers(0, 4, size=m).astype(np.uint8)
    T[10:30] = P[5:25]
    sub = table(4, 1, -1)
    A = oracle.sw_matrix(T, P, sub, -1_000_000, -1)
    expect = np.zeros((n + 1, m + 1), dtype=np.int64)
    for d in range(-(n - 1), m):  # diagonal j - i = d (0-based)
        i0 = max(0, -d)
        i1 = min(n, m - d)
        ii = np.arange(i0, i1)
        s = sub[T[ii], P[ii + d]].astype(np.int64)
        S = np.concatenate(([0], np.cumsum(s)))
        prefmin = np.minimum.accumulate(S)[:-1]
        vals = np.maximum(0, S[1:] - prefmin)
        expect[ii + 1, ii + d + 1] = vals
    np.testing.assert_array_equal(A, expect)


def test_chunked_equals_unchunked():
    """The chunked (multi-threaded) oracle, exact by Theorem 1, equals one plain pass."""
    rng = np.random.default_rng(9)
    T = rng.integers(0, 4, size=20000).astype(np.uint8)
    P = rng.integers(0, 4, size=300).astype(np.uint8)
    for st in (1000, 5000, 12000, 19800):
        T[st:st + 150] = P[100:250]
    T[7000:7300] = P[0:300]
    sub = table(4, 1, -3)
    a = oracle.sw_hits(T, P, sub, -5, -2, 12, threads=1)
    for th in (2, 3, 8, 64):
        b = oracle.sw_hits(T, P, sub, -5, -2, 12, threads=th)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    # a window restricted to text ends in [t_lo, t_hi)
    w = oracle.sw_hits(T, P, sub, -5, -2, 12, t_lo=6900, t_hi=7400, threads=4)
    sel = (a[1] >= 6900) & (a[1] < 7400)
    for x, y in zip(w, a):
        np.testing.assert_array_equal(x, y[sel])
