"""Karlin-Altschul statistics of ungapped local alignment scores, in plain
float64 Python, and the threshold H the paper derives from an E-value.

TEST INFRASTRUCTURE ONLY (tests/ may import it; the library never does).

* :func:`pair_score_distribution` -- the distribution of the score of one
  aligned pair of independent residues drawn from the background.
* :func:`karlin_lambda` -- the positive root of sum p(s) exp(lambda s) = 1,
  by bisection.
* :func:`karlin_K` -- K = lambda d exp(-2 sigma) / (H (1 - exp(-lambda d)))
  with sigma = sum_k (1/k) (E[exp(lambda S_k); S_k < 0] + P(S_k >= 0))
  (Karlin and Altschul, PNAS 87, 1990), S_k summed over the exact
  distribution of k pair scores.
* :func:`evalue_threshold` -- Section 7: H = ceil((ln(K m n) - ln E) / lambda).

Pins (tests/test_karlin.py): for scores +1/-1 the closed forms
lambda = ln(q/p) and K = (q - p)^2 / q; for +1/-3 on uniform DNA the root
from factoring the defining polynomial; and a Monte Carlo estimate of K from
maxima of simulated local alignments (the plain SW oracle with gaps off).
"""
from __future__ import annotations

import math
from functools import reduce


def pair_score_distribution(sub, background):
    dist = {}
    sigma = len(background)
    for a in range(sigma):
        for b in range(sigma):
            w = background[a] * background[b]
            if w > 0:
                s = int(sub[a][b])
                dist[s] = dist.get(s, 0.0) + w
    return dist


def karlin_lambda(dist) -> float:
    def f(x):
        return sum(p * math.exp(x * s) for s, p in dist.items()) - 1.0

    lo, hi = 1e-12, 1.0
    while f(hi) <= 0.0:
        hi *= 2.0
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def entropy(dist, lam: float) -> float:
    return lam * sum(p * s * math.exp(lam * s) for s, p in dist.items())


def karlin_K(dist, lam: float, kmax: int = 20000) -> float:
    d = reduce(math.gcd, [abs(s) for s in dist])
    H = entropy(dist, lam)
    cur = {0: 1.0}
    sig = 0.0
    for k in range(1, kmax + 1):
        nxt = {}
        for v, pv in cur.items():
            for s, ps in dist.items():
                nxt[v + s] = nxt.get(v + s, 0.0) + pv * ps
        cur = {v: p for v, p in nxt.items() if p >= 1e-300}
        term = sum((p * math.exp(lam * v)) if v < 0 else p for v, p in cur.items())
        sig += term / k
        if term / k < 1e-15 and k > 8:
            break
    return lam * d * math.exp(-2.0 * sig) / (H * (1.0 - math.exp(-lam * d)))


def statistics(sub, background):
    dist = pair_score_distribution(sub, background)
    lam = karlin_lambda(dist)
    return lam, karlin_K(dist, lam), entropy(dist, lam)


def evalue_threshold(lam: float, K: float, m: int, n: int, evalue: float) -> int:
    h = math.ceil((math.log(K * m * n) - math.log(evalue)) / lam)
    return max(1, h)
