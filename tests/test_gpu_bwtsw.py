"""BWT-SW's rule alone (Section 2.4): trie rows are expanded while they hold a
positive entry, with none of ALAE's filters (length, score, q-prefix,
domination).  The hit set must not change (both are exact), while the
computed entries give the denominator of the filtering ratio (Equation 5)."""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def _cases():
    w = synth.small_dna(planted=True, H=12)
    yield "small-planted-H12", w["text"], w["queries"][0], (1, -3, -5, -2), 12, 4
    rng = np.random.default_rng(9)
    T = rng.integers(0, 4, 40_000, dtype=np.uint8)
    P = rng.integers(0, 4, 600, dtype=np.uint8)
    for a, y, L in ((3000, 20, 250), (22_000, 300, 280)):
        T[a:a + L] = P[y:y + L]
        T[a + 50] = (T[a + 50] + 1) % 4
    yield "planted-<1,-4,-5,-2>", T, P, (1, -4, -5, -2), 16, 4
    yield "planted-<1,-3,-2,-2>", T, P, (1, -3, -2, -2), 16, 4
    Tp = rng.integers(0, 20, 30_000, dtype=np.uint8)
    Pp = rng.integers(0, 20, 300, dtype=np.uint8)
    Tp[9000:9150] = Pp[100:250]
    yield "protein-<1,-3,-11,-1>", Tp, Pp, (1, -3, -11, -1), 20, 20


@pytest.mark.parametrize("name,T,P,scheme,H,sigma", list(_cases()), ids=[c[0] for c in _cases()])
def test_zero_floor_only_same_hits(name, T, P, scheme, H, sigma):
    idx = alae.Index.build(T, "dna" if sigma == 4 else "protein")
    sc = alae.make_scoring(*scheme)
    st_alae, st_bwtsw = alae.Stats(), alae.Stats()
    got = alae.search(idx, P, H, sc, stats=st_alae)
    base = alae.search(idx, P, H, sc, stats=st_bwtsw, zero_floor_only=True)
    exp = oracle.sw_hits(T, P, oracle.scoring_table(sigma, scheme[0], scheme[1]), scheme[2], scheme[3], H, threads=8)
    assert exp[0].shape[0] > 0
    for g, b, e in zip(got, base, exp):
        np.testing.assert_array_equal(b, e)
        np.testing.assert_array_equal(g, e)
    ratio = (st_bwtsw.entries - st_alae.entries) / st_bwtsw.entries
    print(f"{name}: entries ALAE {st_alae.entries}, BWT-SW rule {st_bwtsw.entries}, filtering ratio {ratio:.3f}",
          flush=True)
    assert st_bwtsw.entries >= st_alae.entries
