"""Exhaustive and literal reference computations for tiny inputs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Nothing here uses a
dynamic-programming shortcut except :func:`mx_matrix`, which writes out the
recurrences of Section 2.2 exactly as printed so that Figure 1 can be checked.

* :func:`sim` and :func:`brute_A` enumerate every alignment transcript, score
  it by the scheme of Section 2.1 (a maximal run of r gap characters of one
  kind costs ``sg + r*ss``) and take the maximum.  They are the definition of
  the local alignment problem (Section 2.1) written out as search.
* :func:`basic_A` follows Algorithm 1 (BASIC): every suffix of the text is a
  path of the suffix trie; for each prefix X[1..i] of that path the score
  against every query end j is M_X(i, j) of Section 2.2, and A keeps the
  maximum over all paths, starting from 0.
"""
from __future__ import annotations

import itertools

NEG_INF = float("-inf")


def transcripts(a: int, b: int):
    """Every global alignment transcript of two strings of lengths a and b.

    'M' pairs one character of each string, 'D' aligns a character of the
    first string (the text) with a gap, 'I' a character of the second string
    (the query) with a gap.
    """
    if a == 0 and b == 0:
        yield ""
        return
    if a > 0 and b > 0:
        for t in transcripts(a - 1, b - 1):
            yield "M" + t
    if a > 0:
        for t in transcripts(a - 1, b):
            yield "D" + t
    if b > 0:
        for t in transcripts(a, b - 1):
            yield "I" + t


def score_transcript(s1, s2, ops: str, sub, sg: int, ss: int) -> int:
    """Score of one transcript: substitution scores plus sg + r*ss per maximal gap run."""
    total = 0
    i1 = i2 = 0
    for op, run in itertools.groupby(ops):
        r = len(list(run))
        if op == "M":
            for _ in range(r):
                total += sub[s1[i1]][s2[i2]]
                i1 += 1
                i2 += 1
        elif op == "D":
            total += sg + r * ss
            i1 += r
        else:
            total += sg + r * ss
            i2 += r
    return total


def sim(s1, s2, sub, sg: int, ss: int) -> int:
    """sim(S1, S2) of Section 2.1: the best global alignment score."""
    return max(score_transcript(s1, s2, t, sub, sg, ss) for t in transcripts(len(s1), len(s2)))


def brute_A(T, P, sub, sg: int, ss: int):
    """A(i, j) for 1 <= i <= n, 1 <= j <= m by exhaustive search (Section 2.1).

    Returns an (n+1) x (m+1) list of lists; row/column 0 are 0.
    A(i,j) = max(0, max over x <= i, y <= j of sim(T[x..i], P[y..j])).
    """
    n, m = len(T), len(P)
    A = [[0] * (m + 1) for _ in range(n + 1)]
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            best = 0
            for x in range(1, i + 1):
                for y in range(1, j + 1):
                    v = sim(T[x - 1:i], P[y - 1:j], sub, sg, ss)
                    if v > best:
                        best = v
            A[i][j] = best
    return A


def mx_matrix(X, P, sub, sg: int, ss: int):
    """M_X, G_a, G_b of Section 2.2 for a substring X against the query P.

    Initial conditions as printed: M(0,j)=0, M(i,0)=sg+i*ss, G_a(0,j)=-inf,
    G_b(i,0)=-inf.  The recurrences are applied for every i >= 1 and j >= 1
    (Figure 1 applies them in row 1 and column 1 too).  There is no zero
    floor: M_X(i,j) is the best score of X[1..i] against any P[y..j].
    Returns three (d+1) x (m+1) lists of lists.
    """
    d, m = len(X), len(P)
    M = [[0] * (m + 1) for _ in range(d + 1)]
    Ga = [[NEG_INF] * (m + 1) for _ in range(d + 1)]
    Gb = [[NEG_INF] * (m + 1) for _ in range(d + 1)]
    for i in range(1, d + 1):
        M[i][0] = sg + i * ss
    for i in range(1, d + 1):
        for j in range(1, m + 1):
            Ga[i][j] = max(Ga[i - 1][j] + ss, M[i - 1][j] + (sg + ss))
            Gb[i][j] = max(Gb[i][j - 1] + ss, M[i][j - 1] + (sg + ss))
            M[i][j] = max(M[i - 1][j - 1] + sub[X[i - 1]][P[j - 1]], Ga[i][j], Gb[i][j])
    return M, Ga, Gb


def basic_A(T, P, sub, sg: int, ss: int):
    """A(i, j) by Algorithm 1 (BASIC) with M_X from Section 2.2.

    Every suffix T[x..n] is one suffix-trie path X; its prefix X[1..k] ends
    at text position x+k-1 and scores M_X(k, j) against query ends j.
    A starts at 0 everywhere and keeps the maximum.
    """
    n, m = len(T), len(P)
    A = [[0] * (m + 1) for _ in range(n + 1)]
    for x in range(1, n + 1):
        X = T[x - 1:]
        M, _, _ = mx_matrix(X, P, sub, sg, ss)
        for k in range(1, len(X) + 1):
            i = x + k - 1
            for j in range(1, m + 1):
                if M[k][j] > A[i][j]:
                    A[i][j] = M[k][j]
    return A


def brute_A_prefixes(T, P, sub, sg: int, ss: int):
    """The same A as :func:`brute_A`, enumerating each alignment once as a prefix.

    Every alignment of T[x..i] against P[y..j] is a prefix of the transcripts
    that start at (x, y); a depth-first walk over all transcripts from each
    start keeps the running score of the prefix walked so far (a substitution
    score per pair; sg + ss for the first character of a gap run, ss for each
    further one: the Section 2.1 cost of the run cut where the prefix ends) and
    records it at the prefix's end cell.  No dynamic programming: the number of
    prefixes walked is the number of alignments, which makes 8 x 8 feasible.
    """
    n, m = len(T), len(P)
    A = [[0] * (m + 1) for _ in range(n + 1)]
    for x in range(n):
        for y in range(m):
            # (i, j, score, last op): i, j characters of T and P consumed from (x, y)
            stack = [(x, y, 0, "")]
            while stack:
                i, j, v, last = stack.pop()
                if i < n and j < m:
                    w = v + sub[T[i]][P[j]]
                    if w > A[i + 1][j + 1]:
                        A[i + 1][j + 1] = w
                    stack.append((i + 1, j + 1, w, "M"))
                if i < n:
                    w = v + ss + (sg if last != "D" else 0)
                    if w > A[i + 1][j]:
                        A[i + 1][j] = w
                    stack.append((i + 1, j, w, "D"))
                if j < m:
                    w = v + ss + (sg if last != "I" else 0)
                    if w > A[i][j + 1]:
                        A[i][j + 1] = w
                    stack.append((i, j + 1, w, "I"))
    # an alignment ends where its last pair or gap character ends; A is at least 0 and
    # row/column 0 hold no local alignment of a non-empty text and query prefix
    for i in range(n + 1):
        A[i][0] = 0
    for j in range(m + 1):
        A[0][j] = 0
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            A[i][j] = max(0, A[i][j])
    return A
