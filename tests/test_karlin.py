"""E-value -> H (Section 7) with Karlin-Altschul lambda and K.

The float64 oracle (oracle/karlin.py) is pinned by closed forms and by a
Monte Carlo estimate of K from simulated local alignments; the library's
statistics and thresholds are compared with the oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import karlin
from paper_1208_0274_amd import alae


def _tab(sigma, sa, sb):
    return [[sa if a == b else sb for b in range(sigma)] for a in range(sigma)]


@pytest.mark.parametrize("bg", [[0.25] * 4, [0.4, 0.2, 0.2, 0.2], [0.1, 0.2, 0.3, 0.4]])
def test_oracle_plus_minus_one_closed_forms(bg):
    """Scores +1 (match, probability p = sum of squared frequencies) and -1: the walk
    has lambda = ln(q/p) and K = (q - p)^2 / q."""
    lam, K, H = karlin.statistics(_tab(4, 1, -1), bg)
    p = sum(x * x for x in bg)
    q = 1.0 - p
    assert lam == pytest.approx(math.log(q / p), rel=1e-10)
    assert K == pytest.approx((q - p) ** 2 / q, rel=1e-9)
    assert H == pytest.approx(lam * (q - p), rel=1e-10)


def test_oracle_plus_one_minus_three_root():
    """Uniform DNA, +1/-3: y = exp(lambda) solves y/4 + 3/(4 y^3) = 1, i.e.
    (y - 1)(y^3 - 3y^2 - 3y - 3) = 0; lambda is the log of the cubic's real root."""
    lam, K, _ = karlin.statistics(_tab(4, 1, -3), [0.25] * 4)
    roots = np.roots([1.0, -3.0, -3.0, -3.0])
    y = max(r.real for r in roots if abs(r.imag) < 1e-9)
    assert lam == pytest.approx(math.log(y), rel=1e-10)


def test_oracle_K_against_simulated_maxima():
    """P(max ungapped local score >= x) ~ 1 - exp(-K m n e^{-lambda x}) for random sequences:
    K estimated from maxima of the plain SW oracle (gaps switched off) at the two most
    likely x, 600 pairs of length 400, within 15% of the series value (edge effects of
    finite lengths lower the estimate slightly)."""
    lam, K, _ = karlin.statistics(_tab(4, 1, -3), [0.25] * 4)
    rng = np.random.default_rng(12)
    m = n = 400
    sub = oracle.scoring_table(4, 1, -3)
    Ms = np.array([oracle.sw_matrix(rng.integers(0, 4, n, dtype=np.uint8), rng.integers(0, 4, m, dtype=np.uint8),
                                    sub, -10 ** 6, -10 ** 6).max() for _ in range(600)])
    med = int(np.median(Ms))
    est = []
    for x in (med, med + 1):
        F = float((Ms >= x).mean())
        est.append(-math.log(1.0 - F) * math.exp(lam * x) / (m * n))
    assert abs(np.mean(est) / K - 1.0) < 0.15, (est, K)


SCHEMES = [
    ("dna", (1, -3), None), ("dna", (1, -1), None), ("dna", (1, -2), [0.3, 0.2, 0.2, 0.3]),
    ("dna", (2, -3), None), ("dna", (1, -4), None), ("protein", (1, -3), None),
]


@pytest.mark.parametrize("alpha,ab,bg", SCHEMES)
def test_library_statistics_equal_oracle(alpha, ab, bg):
    sigma = 4 if alpha == "dna" else 20
    got = alae.karlin_altschul(alae.make_scoring(ab[0], ab[1], -5, -2), alpha, bg)
    lam, K, H = karlin.statistics(_tab(sigma, *ab), bg if bg else [1.0 / sigma] * sigma)
    assert got["lambda"] == pytest.approx(lam, rel=1e-9)
    assert got["K"] == pytest.approx(K, rel=1e-7)
    assert got["H"] == pytest.approx(H, rel=1e-9)


def test_library_matrix_scoring_and_threshold():
    rng = np.random.default_rng(3)
    B = rng.integers(-4, 3, (20, 20))
    B = np.triu(B) + np.triu(B, 1).T
    np.fill_diagonal(B, rng.integers(4, 9, 20))
    bg = rng.random(20) + 0.2
    got = alae.karlin_altschul(alae.make_scoring(sg=-11, ss=-1, matrix=B), "protein", bg)
    lam, K, H = karlin.statistics(B.tolist(), list(bg / bg.sum()))
    assert got["lambda"] == pytest.approx(lam, rel=1e-9)
    assert got["K"] == pytest.approx(K, rel=1e-7)
    for m, n, E in ((10_000, 1_000_000_000, 10.0), (100_000, 100_000_000, 1e-5), (1000, 100_000, 1e-15)):
        h = alae.evalue_threshold(got, m, n, E)
        assert h == karlin.evalue_threshold(lam, K, m, n, E)
        # the threshold's E-value is at most E, one point lower it is above E
        assert K * m * n * math.exp(-lam * h) <= E * (1 + 1e-9)
        assert K * m * n * math.exp(-lam * (h - 1)) > E * (1 - 1e-9) or h == 1


def test_threshold_monotone_and_errors():
    st = alae.karlin_altschul(alae.make_scoring(1, -3, -5, -2), "dna")
    hs = [alae.evalue_threshold(st, 100_000, 100_000_000, E) for E in (1e-15, 1e-5, 1.0, 10.0)]
    assert hs == sorted(hs, reverse=True)
    with pytest.raises(alae.AlaeError):
        alae.karlin_altschul(alae.make_scoring(3, -1, -5, -2), "dna")  # positive expected score
    with pytest.raises(alae.AlaeError):
        alae.evalue_threshold(st, 100, 100, 0.0)
