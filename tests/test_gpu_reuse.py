"""Reuse of duplicate forks (Section 4): queries holding repeated segments.

With reuse on, a chain row made of identical forks is walked as one fork and
its hits are emitted once per copy; the hit set must stay identical to the
oracle's and to the search without reuse, and the reusing ratio (Equation 6)
must be positive on these queries.
"""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def assert_same(got, exp):
    assert got[0].shape == exp[0].shape, (got[0].shape, exp[0].shape)
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e)


def repeat_query(rng, unit_len, copies, flank=48, gap_lo=50, gap_hi=400):
    """Random query holding `copies` copies of one segment (with a shared left flank)."""
    F = rng.integers(0, 4, size=flank).astype(np.uint8)
    S = rng.integers(0, 4, size=unit_len).astype(np.uint8)
    parts = [rng.integers(0, 4, size=int(rng.integers(gap_lo, gap_hi))).astype(np.uint8)]
    for _ in range(copies):
        parts += [F, S, rng.integers(0, 4, size=int(rng.integers(gap_lo, gap_hi))).astype(np.uint8)]
    return np.concatenate(parts), np.concatenate([F, S])


@pytest.mark.parametrize("scheme,copies,seed", [((1, -3, -5, -2), 2, 1), ((1, -3, -5, -2), 3, 2),
                                                 ((1, -1, -5, -2), 2, 3), ((2, -3, -4, -1), 2, 4)])
def test_reuse_identical_hits(scheme, copies, seed):
    rng = np.random.default_rng(900 + seed)
    P, seg = repeat_query(rng, 700, copies)
    T = rng.integers(0, 4, size=40000).astype(np.uint8)
    synth.plant_segments(rng, T, [seg, seg[100:600]], 4, 0.08, 0.02)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(*scheme)
    H = 30 if scheme[0] == 1 else 60
    st_on, st_off = alae.Stats(), alae.Stats()
    on = alae.search(idx, P, H, sc, stats=st_on, use_reuse=True)
    off = alae.search(idx, P, H, sc, stats=st_off)
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, scheme[0], scheme[1]), scheme[2], scheme[3], H, threads=8)
    print(f"scheme={scheme} copies={copies} hits={exp[0].shape[0]} reused={st_on.reused} "
          f"computed={st_on.entries} (off: {st_off.entries}) ratio={st_on.reusing_ratio():.3f} "
          f"chains={st_on.replay_chains}", flush=True)
    assert_same(off, exp)
    assert_same(on, exp)
    assert st_on.reused > 0
    assert st_off.reused == 0


def test_reuse_inert_on_random_query():
    """An i.i.d. query has no repeated forks: reuse finds nothing and changes nothing."""
    rng = np.random.default_rng(950)
    P = rng.integers(0, 4, size=2000).astype(np.uint8)
    T = rng.integers(0, 4, size=30000).astype(np.uint8)
    synth.plant_segments(rng, T, [P[100:900]], 4, 0.1, 0.02)
    idx = alae.Index.build(T, "dna")
    st = alae.Stats()
    on = alae.search(idx, P, 30, stats=st, use_reuse=True)
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, 1, -3), -5, -2, 30, threads=8)
    assert_same(on, exp)
    print(f"reused={st.reused} chains={st.replay_chains}", flush=True)
