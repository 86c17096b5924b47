"""Serving with continuous batching: results in the mix equal results alone."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1208_0274_amd import alae, synth

pytestmark = pytest.mark.gpu


def _same(a, b, what=""):
    assert a[0].shape == b[0].shape, (what, a[0].shape, b[0].shape)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y, err_msg=what)


@pytest.fixture(scope="module")
def planted():
    rng = np.random.default_rng(77)
    T = rng.integers(0, 4, size=300000).astype(np.uint8)
    qs = []
    for i in range(30):
        L = int(np.exp(rng.uniform(np.log(50), np.log(4000))))
        q = rng.integers(0, 4, size=L).astype(np.uint8)
        if i % 2 == 0 and L >= 60:  # half carry a mutated text segment
            hl = min(L, int(rng.integers(60, 600)))
            st = int(rng.integers(0, T.shape[0] - hl))
            seg = synth.mutate(rng, T[st:st + hl], 4, 0.1, 0.02)[:L]
            off = int(rng.integers(0, L - seg.shape[0] + 1))
            q[off:off + seg.shape[0]] = seg
        qs.append(q)
    qs.append(qs[3].copy())  # identical requests
    qs.append(qs[3].copy())
    return T, alae.Index.build(T, "dna"), qs


def test_alone_vs_mix(planted):
    T, idx, qs = planted
    schemes = [(alae.make_scoring(1, -3, -5, -2), 20), (alae.make_scoring(1, -3, -5, -2), 26),
               (alae.make_scoring(1, -1, -5, -2), 24)]
    plan = [(q, schemes[i % 3 if i < 20 else 0]) for i, q in enumerate(qs)]
    alone = [alae.search(idx, q, H, sc) for q, (sc, H) in plan]
    srv = alae.Server(idx, slots=3, max_batch=6)
    ids = [srv.submit(q, H, sc) for q, (sc, H) in plan]
    mix = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    print(st, flush=True)
    assert st["completed"] == len(plan) and st["batches"] < len(plan)
    for k, (a, b) in enumerate(zip(alone, mix)):
        _same(a, b, f"request {k}")
    # pin a few against the oracle as well
    for k in (0, 1, 2, 5, 30):
        q, (sc, H) = plan[k]
        sa, sb, sg, ss = sc.sa, sc.sb, sc.sg, sc.ss
        _same(mix[k], oracle.sw_hits(T, q, oracle.scoring_table(4, sa, sb), sg, ss, H, threads=8), f"oracle {k}")


def test_poisson_arrivals_identical_and_latency(planted):
    """Requests arrive while others run (Poisson, 300/s); each result equals
    the result alone; latency percentiles are reported."""
    T, idx, qs = planted
    sc = alae.make_scoring()
    alone = [alae.search(idx, q, 22, sc) for q in qs]
    srv = alae.Server(idx, slots=4, max_batch=8)
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1 / 300.0, size=len(qs)))
    ids = [None] * len(qs)

    def client():
        t0 = time.perf_counter()
        for k, t in enumerate(arrivals):
            d = t - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            ids[k] = srv.submit(qs[k], 22, sc)

    th = threading.Thread(target=client)
    th.start()
    th.join()
    res = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    print(st, flush=True)
    assert st["completed"] == len(qs)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    for k, (a, b) in enumerate(zip(alone, res)):
        _same(a, b, f"request {k}")


def test_admission_and_errors(planted):
    T, idx, qs = planted
    srv = alae.Server(idx, memory_budget=64 * 1000 * 20 + 30 * 1000, slots=2)
    with pytest.raises(alae.AlaeError) as e:
        srv.submit(qs[0] if qs[0].shape[0] > 2000 else np.zeros(3000, np.uint8), 20)
    assert alae.STATUS[e.value.status] == "ALAE_E_ADMISSION"
    rid = srv.submit(qs[1][:500], 20)
    r = srv.poll(rid, wait=True)
    _same(r, alae.search(idx, qs[1][:500], 20))
    with pytest.raises(alae.AlaeError):
        srv.poll(rid)  # already collected
    srv.close()


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_serving_on_1e9_index():
    """Serving at full size: the 1e9-base index of the batched workload stays resident;
    40 requests shaped like the serving workload (log-uniform 100-100,000, half carrying a
    mutated text segment) arrive at once.  Every result equals the same query searched
    alone; for the shorter requests with hits, the oracle on a text window around all of
    their hits (2,000 text ends on either side, plus L_max of context) gives exactly the
    served hits."""
    w = synth.batched_dna()
    T = w["text"]
    qs = synth.serving_queries(T, 40)
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(1, -3, -5, -2)
    H = 30
    print(f"serving on n={T.shape[0]}: {len(qs)} requests, sum m={sum(q.shape[0] for q in qs)}", flush=True)
    srv = alae.Server(idx, max_batch=16)
    ids = [srv.submit(q, H, sc) for q in qs]
    mix = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    print(st, flush=True)
    assert st["completed"] == len(qs)
    ws = alae.Workspace(idx)
    for k, q in enumerate(qs):
        _same(mix[k], alae.search(idx, q, H, sc), f"request {k} alone")
    ws.free()
    sub = oracle.scoring_table(4, 1, -3)
    checked = 0
    for k, q in enumerate(qs):
        j, t, s = mix[k]
        if t.shape[0] == 0 or q.shape[0] > 4000:
            continue
        a = max(0, int(t.min()) - 2000)
        b = min(T.shape[0], int(t.max()) + 2001)
        lo = max(0, a - oracle.lmax(q.shape[0], 1, -5, -2, H))
        oj, ot, os_ = oracle.sw_hits(T[lo:b], q, sub, -5, -2, H, t_lo=a - lo, t_hi=b - lo, threads=8)
        _same(mix[k], (oj, ot + lo, os_), f"request {k} oracle window [{a}, {b})")
        checked += 1
    print(f"{checked} requests checked against oracle windows", flush=True)
    assert checked >= 3
    idx.free()
