"""Pins of the oracle's alignment start (the paper's A(i,j).pos made unique: the
optimal alignment ending at (t, j) with the largest text start, then the
largest query start) against exhaustive enumeration of transcripts."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute


def _sub(sigma, sa, sb):
    return [[sa if a == b else sb for b in range(sigma)] for a in range(sigma)]


@pytest.mark.parametrize("seed", range(6))
def test_global_suffix_is_sim_of_suffixes(seed):
    rng = np.random.default_rng(seed)
    T = rng.integers(0, 3, 5, dtype=np.uint8)
    P = rng.integers(0, 3, 4, dtype=np.uint8)
    sub = _sub(3, 2, -1)
    G = oracle.global_suffix(T, P, np.array(sub, dtype=np.int32), -3, -1)
    for a in range(1, 6):
        for b in range(1, 5):
            assert G[a, b] == brute.sim(list(T[5 - a:]), list(P[4 - b:]), sub, -3, -1)


@pytest.mark.parametrize("seed", range(8))
def test_alignment_start_by_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    T = rng.integers(0, 2, 7, dtype=np.uint8)
    P = rng.integers(0, 2, 5, dtype=np.uint8)
    sub = _sub(2, 1, -1)
    sg, ss = -2, -1
    subn = np.array(sub, dtype=np.int32)
    for t, j in itertools.product(range(7), range(5)):
        best, starts = 0, []
        for x in range(t + 1):
            for y in range(j + 1):
                v = brute.sim(list(T[x:t + 1]), list(P[y:j + 1]), sub, sg, ss)
                if v > best:
                    best, starts = v, [(x, y)]
                elif v == best and best > 0:
                    starts.append((x, y))
        got = oracle.alignment_start(T, P, subn, sg, ss, t, j)
        if best == 0:
            assert got is None
        else:
            assert got == (*max(starts), best)
