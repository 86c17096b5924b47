"""Device-driven levels (alae_search_opts.level_graph): the level loop runs in
batches of K level slots with no host round trip between levels, replayed
from a captured HIP graph (K > 0) or enqueued kernel by kernel (K < 0).

Every case compares the full sorted hit arrays with the CPU oracle and with
the host-driven loop, bit for bit; graphs are replayed across searches with
the rest of each search (eager kernels and copies) in between.
"""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def assert_same(got, exp, what=""):
    assert got[0].shape == exp[0].shape, (what, got[0].shape, exp[0].shape)
    for g, e in zip(got, exp):
        np.testing.assert_array_equal(g, e, err_msg=what)


def oracle_hits(T, P, scheme, H, sigma=4):
    sa, sb, sg, ss = scheme
    return oracle.sw_hits(T, P, oracle.scoring_table(sigma, sa, sb), sg, ss, H, threads=8)


def planted(seed, n, m, n_plants=6):
    rng = np.random.default_rng(seed)
    T = rng.integers(0, 4, size=n).astype(np.uint8)
    P = rng.integers(0, 4, size=m).astype(np.uint8)
    srcs = []
    for _ in range(n_plants):
        L = int(rng.integers(40, 200))
        y = int(rng.integers(0, m - L + 1))
        srcs.append(P[y:y + L])
    synth.plant_segments(rng, T, srcs, 4, 0.1, 0.02)
    return T, P


SCHEME = (1, -3, -5, -2)


@pytest.mark.parametrize("K", [1, 3, 8, -4])
@pytest.mark.parametrize("tail_split", [True, False])
def test_level_graph_matches_oracle(K, tail_split):
    T, P = planted(5, 200_000, 700)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(*SCHEME)
    exp = oracle_hits(T, P, SCHEME, 16)
    st0, st = alae.Stats(), alae.Stats()
    host = alae.search(idx, P, 16, sc, stats=st0, tail_split=tail_split)
    got = alae.search(idx, P, 16, sc, stats=st, tail_split=tail_split, level_graph=K)
    print(f"K={K} tail_split={tail_split} hits={exp[0].shape[0]} levels host {st0.levels} device {st.levels} "
          f"(device-driven {st.device_levels}, captures {st.graph_captures}, retries {st.retries})", flush=True)
    assert exp[0].shape[0] > 0
    assert_same(host, exp, "host-driven")
    assert_same(got, exp, "device-driven")
    assert st.device_levels > 0
    assert st.levels == st0.levels
    assert st.max_depth == st0.max_depth
    assert (st.graph_captures > 0) == (K > 0)


def test_level_graph_replayed_across_searches():
    """One workspace, the same query four times: the last searches replay the
    graphs captured before (no capture), each result equal to the oracle."""
    T, P = planted(6, 150_000, 500)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(*SCHEME)
    exp = oracle_hits(T, P, SCHEME, 15)
    import torch

    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).cuda()
    want = ((exp[0].astype(np.int64) << 32) | exp[1].astype(np.int64), exp[2].astype(np.int64))
    captures = []
    for r in range(4):
        st = alae.Stats()
        n = ws.search_device(dq, 15, sc, stats=st, tail_split=False, level_graph=6)
        k, s = ws.result_torch()
        torch.cuda.synchronize()
        captures.append(st.graph_captures)
        print(f"search {r}: {n} hits, levels {st.levels} device-driven {st.device_levels} "
              f"captures {st.graph_captures}", flush=True)
        assert st.device_levels > 0
        assert_same((k.cpu().numpy().astype(np.int64), s.cpu().numpy().astype(np.int64)), want, f"search {r}")
    assert captures[0] > 0
    assert captures[-1] == 0


def test_level_graph_overflow_reruns():
    """Buffers far too small: levels of a batch overflow, the host grows the
    buffers and runs the level again, and the batches go on."""
    T, P = planted(7, 120_000, 400)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(*SCHEME)
    exp = oracle_hits(T, P, SCHEME, 14)
    st = alae.Stats()
    got = alae.search(idx, P, 14, sc, stats=st, entry_capacity=256, hit_capacity=64, tail_split=False,
                      level_graph=5)
    print(f"retries {st.retries} device-driven {st.device_levels} captures {st.graph_captures}", flush=True)
    assert st.retries > 0
    assert st.device_levels > 0
    assert_same(got, exp)


def test_level_graph_batch():
    rng = np.random.default_rng(9)
    T = rng.integers(0, 4, size=80_000).astype(np.uint8)
    qs = [rng.integers(0, 4, size=int(rng.integers(30, 400))).astype(np.uint8) for _ in range(7)]
    synth.plant_segments(rng, T, [q[: max(20, q.shape[0] // 2)] for q in qs], 4, 0.1, 0.02)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(*SCHEME)
    st = alae.Stats()
    res = alae.search_batch(idx, qs, 14, sc, stats=st, level_graph=4)
    print(f"device-driven {st.device_levels} captures {st.graph_captures}", flush=True)
    assert st.device_levels > 0
    for i, q in enumerate(qs):
        assert_same(res[i], oracle_hits(T, q, SCHEME, 14), f"query {i}")


def test_level_graph_option_range():
    T, P = planted(10, 5_000, 100, n_plants=1)
    idx = alae.Index.build(T, "dna")
    with pytest.raises(alae.AlaeError):
        alae.search(idx, P, 14, alae.make_scoring(*SCHEME), level_graph=65)


def test_level_graph_protein_matrix_mode():
    """20 letters, a substitution matrix (seeds at depth 1): device-driven levels
    against the oracle."""
    rng = np.random.default_rng(14)
    a = rng.integers(-4, 3, size=(20, 20))
    a = np.triu(a) + np.triu(a, 1).T
    np.fill_diagonal(a, rng.integers(4, 12, size=20))
    T = rng.integers(0, 20, size=40_000).astype(np.uint8)
    P = rng.integers(0, 20, size=250).astype(np.uint8)
    synth.plant_segments(rng, T, [P[20:140], P[100:220]], 20, 0.3, 0.03)
    idx = alae.Index.build(T, "protein")
    sc = alae.make_scoring(0, 0, -11, -1, a)
    exp = oracle.sw_hits(T, P, np.asarray(a, dtype=np.int32), -11, -1, 40, threads=8)
    st = alae.Stats()
    got = alae.search(idx, P, 40, sc, stats=st, level_graph=4)
    print(f"hits {exp[0].shape[0]} levels {st.levels} device-driven {st.device_levels} "
          f"captures {st.graph_captures}", flush=True)
    assert exp[0].shape[0] > 0
    assert st.device_levels > 0
    assert_same(got, exp)


def test_level_graph_ignored_without_allocation():
    """The entry point that allocates nothing runs the host-driven loop whatever
    level_graph says (its buffers are cut from a fixed array): same hits."""
    import torch

    T, P = planted(15, 30_000, 200, n_plants=3)
    idx = alae.Index.build(T, "dna")
    idx.upload()
    sc = alae.make_scoring(*SCHEME)
    exp = oracle_hits(T, P, SCHEME, 14)
    dq = torch.from_numpy(P).cuda()
    cap = exp[0].shape[0] + 4096
    keys = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    scores = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    st = alae.Stats()
    n = alae.search_device_noalloc(idx, dq, 14, keys, scores, sc, stats=st, level_graph=8)
    torch.cuda.synchronize()
    k = keys[:n].cpu().numpy().view(np.uint64)
    got = ((k >> np.uint64(32)).astype(np.int64), (k & np.uint64(0xFFFFFFFF)).astype(np.int64),
           scores[:n].cpu().numpy().astype(np.int64))
    print(f"noalloc with level_graph=8: {n} hits, device-driven levels {st.device_levels}", flush=True)
    assert st.device_levels == 0
    assert_same(got, exp)


def test_level_graph_modes_alternate_on_one_workspace():
    """One workspace, queries of two lengths and the three modes in turn (graph,
    host-driven, enqueued, graph again): graphs captured for one query are not
    replayed for another, and every result equals the oracle's."""
    import torch

    T, P = planted(16, 100_000, 600)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(*SCHEME)
    ws = alae.Workspace(idx)
    cases = [(P, 8), (P[:350], 8), (P, 0), (P[:350], -4), (P, 8), (P[:350], 8)]
    want = {}
    for q, K in cases:
        m = q.shape[0]
        if m not in want:
            e = oracle_hits(T, q, SCHEME, 15)
            want[m] = ((e[0].astype(np.int64) << 32) | e[1].astype(np.int64), e[2].astype(np.int64))
        st = alae.Stats()
        n = ws.search_device(torch.from_numpy(np.ascontiguousarray(q)).cuda(), 15, sc, stats=st, tail_split=False,
                             level_graph=K)
        k, s = ws.result_torch()
        torch.cuda.synchronize()
        print(f"m={m} K={K}: {n} hits, device-driven {st.device_levels}, captures {st.graph_captures}", flush=True)
        assert (st.device_levels > 0) == (K != 0)
        assert_same((k.cpu().numpy().astype(np.int64), s.cpu().numpy().astype(np.int64)), want[m], f"m={m} K={K}")
