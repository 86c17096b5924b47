"""The index built on the GPU (prefix doubling) against the host build (SA-IS):
the same suffix array of text ends, BWT, C and terminator row, the same
backward-search ranges (which read the occ blocks), and searches on the
GPU-built index equal to the oracle.  The host build itself is pinned by the
paper's examples and naive suffix sorting in test_index.py."""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae

pytestmark = pytest.mark.gpu


def _texts():
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 7, 192, 193, 1000, 50_000):
        out.append((f"dna{n}", rng.integers(0, 4, n, dtype=np.uint8), "dna"))
        out.append((f"prot{n}", rng.integers(0, 20, n, dtype=np.uint8), "protein"))
    out.append(("allA", np.zeros(5000, dtype=np.uint8), "dna"))
    out.append(("period3", np.tile(np.array([0, 1, 2], dtype=np.uint8), 3000), "dna"))
    out.append(("period2prot", np.tile(np.array([7, 19], dtype=np.uint8), 2000), "protein"))
    x = rng.integers(0, 4, 777, dtype=np.uint8)
    out.append(("repeats", np.concatenate([x, x, rng.integers(0, 4, 50, dtype=np.uint8), x, x[:300]]), "dna"))
    return out


def _compare(T, alpha, patterns=200, seed=0):
    h = alae.Index.build(T, alpha, builder="host")
    g = alae.Index.build(T, alpha, builder="gpu")
    hi, gi = h.info(), g.info()
    assert hi["C"] == gi["C"]
    assert hi["dollar_row"] == gi["dollar_row"]
    np.testing.assert_array_equal(h.sa_end(), g.sa_end())
    np.testing.assert_array_equal(h.bwt(), g.bwt())
    rng = np.random.default_rng(seed)
    sigma = 4 if alpha == "dna" else 20
    n = T.shape[0]
    for _ in range(patterns):
        L = int(rng.integers(1, 12))
        if n >= L and rng.random() < 0.7:
            a = int(rng.integers(0, n - L + 1))
            pat = T[a:a + L]
        else:
            pat = rng.integers(0, sigma, L, dtype=np.uint8)
        assert h.range(pat) == g.range(pat)
    return h, g


@pytest.mark.parametrize("name,T,alpha", _texts(), ids=[t[0] for t in _texts()])
def test_gpu_build_equals_host_build(name, T, alpha):
    print(f"index build compare: {name} n={T.shape[0]} {alpha}", flush=True)
    h, g = _compare(T, alpha)
    h.free()
    g.free()


def test_gpu_build_large_with_repeats():
    rng = np.random.default_rng(3)
    n = (1 << 22) + 3
    T = rng.integers(0, 4, n, dtype=np.uint8)
    for _ in range(200):  # exact and mutated copies: long shared prefixes, many doubling rounds
        L = int(rng.integers(100, 5000))
        a, b = (int(v) for v in rng.integers(0, n - L, 2))
        T[b:b + L] = T[a:a + L]
        if rng.random() < 0.5:
            T[b + L // 2] = (T[b + L // 2] + 1) % 4
    print(f"index build compare: n={n} with 200 copies", flush=True)
    h, g = _compare(T, "dna", patterns=500)
    h.free()
    g.free()


def test_search_on_gpu_built_index():
    rng = np.random.default_rng(4)
    T = rng.integers(0, 4, 60_000, dtype=np.uint8)
    P = rng.integers(0, 4, 700, dtype=np.uint8)
    for a, y, L in ((1000, 10, 300), (30_000, 350, 200), (50_000, 100, 400)):
        T[a:a + L] = P[y:y + L]
        T[a + L // 3] = (T[a + L // 3] + 2) % 4
    idx = alae.Index.build(T, "dna", builder="gpu")
    got = alae.search(idx, P, 20, alae.make_scoring(1, -3, -5, -2))
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, 1, -3), -5, -2, 20, threads=8)
    assert exp[0].shape[0] > 0
    for x, y in zip(got, exp):
        np.testing.assert_array_equal(x, y)
    idx.free()
