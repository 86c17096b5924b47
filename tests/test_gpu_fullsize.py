"""Parity at the full workload sizes, in the launch configuration bench.py times
(device-resident query and result, one workspace).

DNA long query (text 1e8, query 1e5): the hits whose text end falls in a window are
exactly the oracle's hits on T[window start - L_max .. window end] (Theorem 1
bounds the text span of any alignment scoring >= H), so planted-copy windows
and random background windows are checked exactly, many in parallel.
The protein stand-in (text 5e7, query 5e3) is checked in full.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def device_search(w):
    import torch

    T, P = w["text"], w["queries"][0]
    idx = alae.Index.build(T, w["alphabet"])
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    st = alae.Stats()
    cnt = ws.search_device(dq, w["H"], alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"]), stats=st)
    keys, scores = ws.result_torch()
    torch.cuda.synchronize()
    keys = keys.cpu().numpy().view(np.uint64)
    scores = scores.cpu().numpy().astype(np.int64)
    ws.free()
    assert keys.shape[0] == cnt
    return (keys >> np.uint64(32)).astype(np.int64), (keys & np.uint64(0xFFFFFFFF)).astype(np.int64), scores, st


def check_global_properties(j, t, s, w):
    """Properties that hold at any size: sorted unique (j, t), scores >= H, ends in range."""
    assert np.all(s >= w["H"])
    assert np.all((j >= 0) & (j < w["queries"][0].shape[0]))
    assert np.all((t >= 0) & (t < w["text"].shape[0]))
    key = j * (1 << 32) + t
    assert np.all(np.diff(key) > 0)


def test_dna_long_query_windows():
    w = synth.dna_long_query()
    T, P, H = w["text"], w["queries"][0], w["H"]
    j, t, s, st = device_search(w)
    print(f"DNA 1e8 x 1e5: {j.shape[0]} hits, {st.entries} entries, {st.device_ms:.1f} ms", flush=True)
    check_global_properties(j, t, s, w)
    sub = oracle.scoring_table(4, 1, -3)
    lmax = oracle.lmax(P.shape[0], 1, w["sg"], w["ss"], H)
    rng = np.random.default_rng(2024)
    plants = w["plants"]
    pick = list(rng.choice(len(plants), size=10, replace=False))
    pick.append(int(np.argmin([p[1] for p in plants])))
    pick.append(int(np.argmax([p[1] for p in plants])))
    windows = [(plants[k][0], plants[k][0] + plants[k][1] + 50) for k in pick]
    for _ in range(4):  # background windows
        a = int(rng.integers(lmax, T.shape[0] - 3000))
        windows.append((a, a + 2000))

    def one(win):
        a, b = win
        lo = max(0, a - lmax)
        ej, et, es = oracle.sw_hits(T[lo:b], P, sub, w["sg"], w["ss"], H, t_lo=a - lo, t_hi=b - lo, threads=1)
        return a, b, ej, et + lo, es

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        results = list(ex.map(one, windows))
    checked = 0
    for a, b, ej, et, es in results:
        sel = (t >= a) & (t < b)
        gj, gt, gs = j[sel], t[sel], s[sel]
        order = np.lexsort((gt, gj))
        np.testing.assert_array_equal(gj[order], ej)
        np.testing.assert_array_equal(gt[order], et)
        np.testing.assert_array_equal(gs[order], es)
        checked += ej.shape[0]
    print(f"DNA 1e8 x 1e5 windows: {len(windows)} windows, {checked} hits checked exactly", flush=True)
    assert checked > 0


def test_protein_standin_full():
    w = synth.protein_standin()
    T, P, H = w["text"], w["queries"][0], w["H"]
    j, t, s, st = device_search(w)
    print(f"protein 5e7 x 5e3: {j.shape[0]} hits, {st.entries} entries, {st.device_ms:.1f} ms", flush=True)
    check_global_properties(j, t, s, w)
    ej, et, es = oracle.sw_hits(T, P, oracle.scoring_table(20, 1, -3), w["sg"], w["ss"], H,
                                threads=min(64, os.cpu_count() or 1))
    np.testing.assert_array_equal(j, ej)
    np.testing.assert_array_equal(t, et)
    np.testing.assert_array_equal(s, es)


def _device_digest_check(keys, scores, golden_rows, edges):
    """Digest the device result per bin of text ends on the GPU and compare with the
    oracle's stored digests."""
    import torch

    from hitdigest import record_hashes, record_hashes_torch, unsigned

    # the GPU form of the hash agrees with the numpy form that wrote the golden file
    rng = np.random.default_rng(1)
    jj, tt, ss = (rng.integers(0, 1 << 20, 1000), rng.integers(0, 1 << 31, 1000), rng.integers(30, 1 << 20, 1000))
    g1, _ = record_hashes_torch(*(torch.from_numpy(x.astype(np.int64)).cuda() for x in (jj, tt, ss)))
    n1, _ = record_hashes(jj, tt, ss)
    assert [unsigned(int(v)) for v in g1.cpu()] == [int(v) for v in n1]
    j = keys >> 32
    t = keys & 0xFFFFFFFF
    h1, h2 = record_hashes_torch(j, t, scores.to(torch.int64))
    e = torch.tensor(edges, dtype=torch.int64, device=keys.device)
    b = torch.searchsorted(e, t, right=True) - 1
    nb = len(edges) - 1
    inside = (b >= 0) & (b < nb)
    b = torch.where(inside, b, torch.full_like(b, nb))
    cnt = torch.bincount(b, minlength=nb + 1).cpu().tolist()
    s1 = torch.zeros(nb + 1, dtype=torch.int64, device=keys.device).index_add_(0, b, h1).cpu().tolist()
    s2 = torch.zeros(nb + 1, dtype=torch.int64, device=keys.device).index_add_(0, b, h2).cpu().tolist()
    bad = []
    for k, row in enumerate(golden_rows):
        got = (cnt[k], unsigned(s1[k]), unsigned(s2[k]))
        if got != tuple(row[-3:]):
            bad.append((row[0], row[1], got, tuple(row[-3:])))
    return bad, cnt[nb]


def test_dna_long_query_all_hits():
    """Every hit of the DNA long query (2.1e8) against the oracle: digests of 1,000 bins of
    100,000 text ends, written by tests/golden/make_digests.py from the oracle alone."""
    import torch

    from hitdigest import read_digest_file

    rows = read_digest_file(os.path.join(os.path.dirname(__file__), "golden", "dna_long_query_digests.txt"))
    rows = sorted({r[0]: r for r in rows}.values())
    edges = [r[0] for r in rows] + [rows[-1][1]]
    assert len(rows) == 1000 and edges[0] == 0 and edges[-1] == 100_000_000
    assert all(rows[k][1] == rows[k + 1][0] for k in range(len(rows) - 1))
    w = synth.dna_long_query()
    T, P, H = w["text"], w["queries"][0], w["H"]
    idx = alae.Index.build(T, w["alphabet"])
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    cnt = ws.search_device(dq, H, alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"]))
    keys, scores = ws.result_torch()
    bad, outside = _device_digest_check(keys, scores, rows, edges)
    total = sum(r[2] for r in rows)
    print(f"DNA 1e8 x 1e5: {cnt} device hits, oracle {total}; {len(rows) - len(bad)}/{len(rows)} bins equal",
          flush=True)
    assert outside == 0
    assert not bad, bad[:5]
    assert cnt == total
    ws.free()
    idx.free()
