"""Text-sharded index: shards own disjoint ranges of text ends and index
L_max - 1 characters before them (Theorem 1), so the union of their owned hits
is the whole text's hit set.  Homologs are planted across shard boundaries;
the result must equal the oracle's on the unsharded text, also when shards
stream through device memory one at a time."""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def sharded_case(seed, n=300_000, m=800, shard=40_000, sigma=4):
    rng = np.random.default_rng(seed)
    T = rng.integers(0, sigma, n, dtype=np.uint8)
    P = rng.integers(0, sigma, m, dtype=np.uint8)
    srcs = []
    for b in range(shard, n, shard):  # a copy of a query segment over every shard boundary
        L = int(rng.integers(min(150, m // 3), min(500, m - 20)))
        y = int(rng.integers(0, m - L))
        st = b - L // 2
        T[st:st + L] = P[y:y + L]
        T[st + L // 3] = (T[st + L // 3] + 1) % sigma
    for _ in range(6):
        L = int(rng.integers(50, min(300, m - 20)))
        y = int(rng.integers(0, m - L))
        srcs.append(P[y:y + L])
    synth.plant_segments(rng, T, srcs, sigma, 0.12, 0.02)
    return T, P


@pytest.mark.parametrize("max_resident", [0, 1])
def test_sharded_equals_oracle(max_resident):
    T, P = sharded_case(1)
    H = 18
    lmax = oracle.lmax(P.shape[0], 1, -5, -2, H)
    sh = alae.ShardedIndex(T, "dna", shard_len=40_000, overlap=lmax - 1, max_resident=max_resident)
    print(f"sharded n={T.shape[0]} shards of 40000, overlap {lmax - 1}, max_resident {max_resident}", flush=True)
    got = sh.search(P, H, alae.make_scoring(1, -3, -5, -2))
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, 1, -3), -5, -2, H, threads=8)
    assert exp[0].shape[0] > 0
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e)
    # the same hits as one index over the whole text
    one = alae.search(alae.Index.build(T, "dna"), P, H, alae.make_scoring(1, -3, -5, -2))
    for g, e in zip(got, one):
        np.testing.assert_array_equal(g, e)
    sh.free()


def test_sharded_protein_and_limits():
    T, P = sharded_case(2, n=120_000, m=300, shard=25_000, sigma=20)
    lmax = oracle.lmax(P.shape[0], 1, -11, -1, 25)
    sh = alae.ShardedIndex(T, "protein", shard_len=25_000, overlap=lmax - 1)
    got = sh.search(P, 25, alae.make_scoring(1, -3, -11, -1))
    exp = oracle.sw_hits(T, P, oracle.scoring_table(20, 1, -3), -11, -1, 25, threads=8)
    assert exp[0].shape[0] > 0
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e)
    # a query whose L_max exceeds the overlap is refused
    with pytest.raises(alae.AlaeError) as ei:
        sh.search(np.concatenate([P, P, P]), 25, alae.make_scoring(1, -3, -11, -1))
    assert ei.value.status == 4
    sh.free()
