"""The search entry point that allocates nothing (alae_search_device_noalloc),
called through the C ABI, against the allocating entry point
(alae_search_device) and the oracle: two calls in a row on one device, the
second with a smaller input, then the error paths."""
import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def _split(keys, scores):
    k = keys.cpu().numpy().view(np.uint64)
    return (k >> np.uint64(32)).astype(np.int64), (k & np.uint64(0xFFFFFFFF)).astype(np.int64), \
        scores.cpu().numpy().astype(np.int64)


def _allocating(ws, dq, H, sc):
    ws.search_device(dq, H, sc)
    keys, scores = ws.result_torch()
    return _split(keys, scores)


def _noalloc(idx, dq, H, sc, cap):
    import torch

    keys = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    scores = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    cnt = alae.search_device_noalloc(idx, dq, H, keys, scores, sc)
    torch.cuda.synchronize()
    return _split(keys[:cnt], scores[:cnt])


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_noalloc_matches_allocating_search_twice():
    import torch

    w = synth.small_dna(planted=True, H=12)
    T, P, H = w["text"], w["queries"][0], 12
    sc = alae.make_scoring(1, -3, -5, -2)
    idx = alae.Index.build(T, "dna")
    idx.upload()
    ws = alae.Workspace(idx)
    sub = oracle.scoring_table(4, 1, -3)
    # first call: the whole query; second call: a shorter one (smaller input)
    for q in (P, P[100:500]):
        print(f"noalloc search: n={T.shape[0]} m={q.shape[0]} H={H}", flush=True)
        dq = torch.from_numpy(np.ascontiguousarray(q)).to("cuda")
        ref = _allocating(ws, dq, H, sc)
        got = _noalloc(idx, dq, H, sc, cap=ref[0].shape[0] + 1000)
        assert ref[0].shape[0] > 0
        _same(got, ref)
        _same(got, oracle.sw_hits(T, q, sub, -5, -2, H, threads=8))
    ws.free()
    idx.free()


def test_noalloc_protein_after_dna():
    """A different index and alphabet on the same device's array."""
    import torch

    rng = np.random.default_rng(7)
    T = rng.integers(0, 20, 30000, dtype=np.uint8)
    P = rng.integers(0, 20, 300, dtype=np.uint8)
    T[5000:5200] = P[50:250]
    T[20000:20150] = P[100:250]
    idx = alae.Index.build(T, "protein")
    idx.upload()
    sc = alae.make_scoring(1, -3, -11, -1)
    dq = torch.from_numpy(P).to("cuda")
    print("noalloc search: protein n=30000 m=300 H=20", flush=True)
    got = _noalloc(idx, dq, 20, sc, cap=1 << 16)
    exp = oracle.sw_hits(T, P, oracle.scoring_table(20, 1, -3), -11, -1, 20, threads=8)
    assert exp[0].shape[0] > 0
    _same(got, exp)
    idx.free()


def test_noalloc_errors():
    import torch

    w = synth.small_dna(planted=True, H=12)
    T, P = w["text"], w["queries"][0]
    sc = alae.make_scoring(1, -3, -5, -2)
    dq = torch.from_numpy(P).to("cuda")
    keys = torch.empty(4, dtype=torch.int64, device="cuda")
    scores = torch.empty(4, dtype=torch.int32, device="cuda")
    fresh = alae.Index.build(T, "dna")
    print("noalloc errors: index not on the device", flush=True)
    with pytest.raises(alae.AlaeError) as ei:
        alae.search_device_noalloc(fresh, dq, 12, keys, scores, sc)
    assert ei.value.status == 1
    fresh.upload()
    print("noalloc errors: output capacity too small", flush=True)
    with pytest.raises(alae.AlaeError) as ei:
        alae.search_device_noalloc(fresh, dq, 12, keys, scores, sc)
    assert ei.value.status == 5 and "capacity" in str(ei.value)
    print("noalloc errors: buffers beyond the fixed array", flush=True)
    with pytest.raises(alae.AlaeError) as ei:
        alae.search_device_noalloc(fresh, dq, 12, keys, scores, sc, entry_capacity=1 << 26)
    assert ei.value.status == 5 and "fixed scratch" in str(ei.value)
    print("noalloc errors: a model is refused", flush=True)
    net = alae.MLP(seed=0)
    with pytest.raises(alae.AlaeError) as ei:
        alae.search_device_noalloc(fresh, dq, 12, keys, scores, sc, order_model=net)
    assert ei.value.status == 1
    net.free()
    # the device's array still serves a normal call afterwards
    big_k = torch.empty(1 << 16, dtype=torch.int64, device="cuda")
    big_s = torch.empty(1 << 16, dtype=torch.int32, device="cuda")
    cnt = alae.search_device_noalloc(fresh, dq, 12, big_k, big_s, sc)
    exp = oracle.sw_hits(T, P, oracle.scoring_table(4, 1, -3), -5, -2, 12, threads=8)
    assert cnt == exp[0].shape[0]
    fresh.free()
