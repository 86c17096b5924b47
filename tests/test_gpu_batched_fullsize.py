"""Parity of the batched workload at its full size: 256 DNA queries (log-uniform
500-50,000, 20 planted mutated segments of each) against a 1e9-base text, run as
one batched device search in the configuration bench.py times.

The oracle cannot cover 2.6e15 cells, so its hits are checked by windows of text
ends (Theorem 1: an alignment scoring at least H spans at most L_max text
characters, so a window's hits are the oracle's hits on the window plus L_max
characters before it): for every query one window per planted copy of it and one
seeded random window of 1e6 text ends.  tests/golden/make_digests.py wrote the
oracle's digests of those windows.  Every device hit of a query that lies in none
of its windows is counted as unchecked; on this workload there are none (hits
arise only at the planted copies)."""
import os

import numpy as np
import pytest

from paper_1208_0274_amd import alae, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batched_dna_window_digests.txt")


@pytest.mark.timeout(600)
def test_batched_dna_windows():
    import torch

    from hitdigest import read_digest_file, record_hashes_torch, unsigned

    rows = read_digest_file(GOLDEN)
    w = synth.batched_dna()
    T, qs, H = w["text"], w["queries"], w["H"]
    n_windows = len(w["plants"]) + len(qs)
    wins = {}
    for (q, lo, hi, c, s1, s2) in rows:
        wins.setdefault(q, {})[(lo, hi)] = (c, s1, s2)
    assert sum(len(v) for v in wins.values()) == n_windows, "golden digests incomplete"
    idx = alae.Index.build(T, "dna")
    ws = alae.Workspace(idx)
    lens = [q.shape[0] for q in qs]
    cat = torch.from_numpy(np.concatenate(qs)).to("cuda")
    print(f"batched search: 256 queries, sum m={sum(lens)}, n={T.shape[0]}", flush=True)
    cnt = ws.search_device_batch(cat, lens, H, alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"]))
    off = ws.batch_offsets()
    keys, scores = ws.result_torch()
    checked = unchecked = 0
    bad = []
    for q in range(len(qs)):
        k = keys[off[q]:off[q + 1]]
        j = k >> 32
        t = k & 0xFFFFFFFF
        h1, h2 = record_hashes_torch(j, t, scores[off[q]:off[q + 1]].to(torch.int64))
        t, order = torch.sort(t)
        c1 = torch.cumsum(torch.cat([torch.zeros(1, dtype=torch.int64, device=t.device), h1[order]]), 0)
        c2 = torch.cumsum(torch.cat([torch.zeros(1, dtype=torch.int64, device=t.device), h2[order]]), 0)
        spans = sorted(wins[q])
        bounds = torch.tensor([x for sp in spans for x in sp], dtype=torch.int64, device=t.device)
        pos_t = torch.searchsorted(t, bounds)
        pos = pos_t.cpu().tolist()
        v1 = c1[pos_t].cpu().tolist()
        v2 = c2[pos_t].cpu().tolist()
        for i, sp in enumerate(spans):
            a, b = pos[2 * i], pos[2 * i + 1]
            got = (b - a, unsigned(v1[2 * i + 1] - v1[2 * i]), unsigned(v2[2 * i + 1] - v2[2 * i]))
            if got != wins[q][sp]:
                bad.append((q, sp, got, wins[q][sp]))
        # hits of this query outside the union of its windows
        cur_lo = cur_hi = None
        merged = []
        for lo, hi in spans:
            if cur_hi is not None and lo <= cur_hi:
                cur_hi = max(cur_hi, hi)
            else:
                if cur_hi is not None:
                    merged.append((cur_lo, cur_hi))
                cur_lo, cur_hi = lo, hi
        merged.append((cur_lo, cur_hi))
        mb = torch.tensor([x for sp in merged for x in sp], dtype=torch.int64, device=t.device)
        mp = torch.searchsorted(t, mb).cpu().tolist()
        covered = sum(mp[2 * i + 1] - mp[2 * i] for i in range(len(merged)))
        checked += covered
        unchecked += t.shape[0] - covered
    print(f"batched 256 x 1e9: {cnt} device hits; {checked} in the {n_windows} oracle windows, "
          f"{unchecked} outside them; {len(bad)} windows differ", flush=True)
    assert not bad, bad[:5]
    assert unchecked == 0
    assert checked == cnt
    ws.free()
    idx.free()
