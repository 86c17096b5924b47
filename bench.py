"""Benchmark of the exact local-alignment search on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload dna|small|protein] [--no-cpu]

A step is one complete search of the workload's query against the resident
index: seeding, every trie level, hit emission, sort and max-merge, with the
sorted hit set left in device memory.  The query is already in HBM when the
timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective m*n cell-updates/s + DP entries/s at exact hits; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1208_0274_amd import synth

    if name == "dna":
        w = synth.dna_long_query()
        desc = ("DNA long query: text 1e8 i.i.d. ACGT + 1,000 planted mutated query segments "
                "(200-2,000, 15% subs, 2% indels); query 1e5; <1,-3,-5,-2>; H=30")
    elif name == "small":
        w = synth.small_dna()
        desc = "plain method, single query: text 1e5 i.i.d. ACGT; query 1e3; <1,-3,-5,-2>; H=18"
    elif name == "protein":
        w = synth.protein_standin()
        desc = ("protein stand-in: text 5e7 uniform residues + 500 planted segments (50-500, 30% subs, "
                "3% indels); query 5,000; <1,-3,-11,-1>; H=45")
    else:
        raise SystemExit(f"unknown workload {name}")
    return w, desc


def cpu_baseline(w, budget_s: float):
    """The oracle as it stands, on a bounded slice of the same text.

    The chunked oracle recomputes L_max text rows in front of every thread's
    chunk (that overlap makes it exact), so the thread count is chosen to keep
    that overlap at most half of each thread's rows; with too small a budget
    the oracle runs on one thread without chunking."""
    import oracle

    T, P = w["text"], w["queries"][0]
    m = P.shape[0]
    cores = os.cpu_count() or 1
    sub = oracle.scoring_table(w["sigma"], w["sa"], w["sb"])
    lmax = oracle.lmax(m, int(sub.max()), w["sg"], w["ss"], w["H"])
    # single-thread rate on a short slice
    L = max(1000, int(1e8 // m))
    t0 = time.perf_counter()
    oracle.sw_hits(T[:L], P, sub, w["sg"], w["ss"], w["H"], threads=1)
    r1 = m * L / max(time.perf_counter() - t0, 1e-6)
    rows_per_thread = r1 * budget_s / m
    threads = min(cores, 64) if rows_per_thread >= 2 * lmax else 1
    if threads > 1:
        L2 = int(threads * (rows_per_thread - lmax))
    else:
        L2 = int(rows_per_thread)
    L2 = max(L, min(T.shape[0], L2))
    t0 = time.perf_counter()
    oracle.sw_hits(T[:L2], P, sub, w["sg"], w["ss"], w["H"], threads=threads)
    dt = time.perf_counter() - t0
    return {"value": m * L2 / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"full query (m={m}) against the first {L2} text characters in {dt:.1f} s "
                      f"({threads} thread(s); L_max={lmax} rows recomputed in front of each chunk); "
                      f"host has {cores} cores"}


LEVEL_KERNEL = "k_level_tasks+k_expand_children"  # the trie-expansion step of one level (node phase, child phase)


def measured_traffic():
    """HBM bytes per level of the trie-expansion kernels from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a
    device-copy calibration), or None when the kernel sources or the host loop
    that decides which levels run changed since it was taken."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "trie_expansion_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_b = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    m_h = re.search(r"source_hash: ([0-9a-f]+)", text)
    if not m_b or not m_h:
        return None
    h = hashlib.sha256()
    for f in ("level_kernels.h", "row_update.h", "device_common.h", "search.hip"):
        h.update(open(os.path.join(ROOT, "paper_1208_0274_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != m_h.group(1):
        return None
    return int(m_b.group(1))


def learned_scheduling(alae, ws, dq, H, sc, steps, plain_ms):
    """Trace one search, train the work predictor on the GPU, then time the
    search with the learned order + partition of the walkers' queues."""
    import torch

    t0 = time.perf_counter()
    tr = alae.Trace(1 << 23)
    ws.search_device(dq, H, sc, trace=tr)
    X, W = tr.arrays()
    y = np.log2(1.0 + W)
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(y))
    ntr = int(0.8 * len(y))
    wide = np.where(X[perm[:ntr], 7] == 1)[0]
    sel = np.concatenate([perm[:ntr], np.repeat(perm[:ntr][wide], 50)])  # the wave queue is 1000x smaller
    net = alae.MLP(seed=1)
    t1 = time.perf_counter()
    loss = net.train(X[sel], y[sel], epochs=8, batch=4096, lr=2e-3)
    train_s = time.perf_counter() - t1
    pred = net.predict(X[perm[ntr:]])
    from scipy.stats import spearmanr

    rho = float(spearmanr(pred, y[perm[ntr:]]).correlation)
    out = {"trace_items": int(tr.count), "train_samples": int(len(sel)), "train_s": train_s, "train_loss": loss,
           "heldout_spearman": rho, "plain_ms": plain_ms}
    for name, kw in (("order_ms", dict(order_model=net, order_queues=2)),
                     ("order_partition_ms", dict(order_model=net, order_queues=2, partition_threshold=9.0))):
        times = []
        for _ in range(steps):
            st = alae.Stats()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ws.search_device(dq, H, sc, stats=st, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t2)
        out[name] = float(np.mean(times) * 1e3)
        out[name.replace("_ms", "_moved")] = int(st.partitioned)
    out["gain_order"] = plain_ms / out["order_ms"]
    out["gain_order_partition"] = plain_ms / out["order_partition_ms"]
    out["total_s"] = time.perf_counter() - t0
    net.free()
    return out


def batched_vs_single(alae, k=64, n=100_000_000):
    """The batched workload's shape on a smaller text: k independent DNA queries
    (log-uniform lengths 500-50,000), each with 20 planted mutated segments
    (200-2,000, 15% substitutions, 2% indels) in an i.i.d. text of n bases.
    One batched search against k single-query searches on one workspace."""
    import torch

    from paper_1208_0274_amd import synth

    w = synth.batched_dna(n=n, k=k)
    qs = w["queries"]
    t0 = time.perf_counter()
    idx = alae.Index.build(w["text"], "dna")
    build_s = time.perf_counter() - t0
    sc = alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"])
    ws = alae.Workspace(idx)
    lens = [q.shape[0] for q in qs]
    cat = torch.from_numpy(np.concatenate(qs)).to("cuda")
    dqs = [torch.from_numpy(np.ascontiguousarray(q)).to("cuda") for q in qs]
    ws.search_device_batch(cat, lens, w["H"], sc)  # warm-up
    for d in dqs[:4]:
        ws.search_device(d, w["H"], sc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb = ws.search_device_batch(cat, lens, w["H"], sc)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    ns = 0
    for d in dqs:
        ns += ws.search_device(d, w["H"], sc)
    torch.cuda.synchronize()
    tsing = time.perf_counter() - t0
    ws.free()
    idx.free()
    if nb != ns:
        raise SystemExit(f"batched hits {nb} != single-query hits {ns}")
    return {"workload": f"{k} queries, log-uniform 500-50,000, 20 planted copies each, text {n:.0e}",
            "queries": k, "sum_m": int(sum(lens)), "index_build_s": build_s, "batched_ms": tb * 1e3,
            "single_ms": tsing * 1e3, "speedup": tsing / tb, "hits": int(nb),
            "batched_cells_per_s": float(sum(lens)) * n / tb}


def serving(alae, idx, T, rates=(10.0, 100.0, 1000.0), count=48):
    """Poisson arrivals of queries with log-uniform lengths 100-100,000 (half
    carrying a mutated 200-2,000 text segment) against the resident index;
    per rate: completed requests per second and submit-to-completion p50/p99."""
    import threading

    from paper_1208_0274_amd import synth

    sc = alae.make_scoring()
    out = []
    srv = alae.Server(idx, slots=4, max_batch=16)
    qs = synth.serving_queries(T, count)
    for rate in rates:
        arrivals = synth.poisson_arrivals(rate, count)
        srv.reset_stats()
        ids = [None] * count

        def client():
            t0 = time.perf_counter()
            for k, t in enumerate(arrivals):
                d = t - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                ids[k] = srv.submit(qs[k], 30, sc)

        th = threading.Thread(target=client)
        t0 = time.perf_counter()
        th.start()
        th.join()
        for i in ids:
            srv.poll(i)
        wall = time.perf_counter() - t0
        st = srv.stats()
        out.append({"rate_qps": rate, "requests": count, "throughput_qps": count / wall, "p50_ms": st["p50_ms"],
                    "p99_ms": st["p99_ms"], "mean_batch": st["mean_batch"], "searches": st["batches"],
                    "mean_m": float(np.mean([q.shape[0] for q in qs]))})
        log(f"serving at {rate} q/s: {out[-1]}")
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dna")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the learned-scheduling and batching legs")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the search runs on a single GPU "
              "(it would shard by text range, one index part per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1208_0274_amd import alae

    w, desc = workload(args.workload)
    T, P = w["text"], w["queries"][0]
    n, m, H = int(T.shape[0]), int(P.shape[0]), int(w["H"])
    log(f"workload {w['name']}: n={n} m={m} H={H}")
    t0 = time.perf_counter()
    idx = alae.Index.build(T, w["alphabet"])
    log(f"index built in {time.perf_counter() - t0:.1f} s")
    sc = alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"])
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        st = alae.Stats()
        cnt = ws.search_device(dq, H, sc, stats=st, stream=stream)
        log(f"warmup {i}: hits={cnt} entries={st.entries} levels={st.levels} {st.device_ms:.1f} ms")
    torch.cuda.synchronize()
    times, stats = [], []
    for i in range(args.steps):
        st = alae.Stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cnt = ws.search_device(dq, H, sc, stats=st, stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(st)
        log(f"step {i}: {times[-1] * 1e3:.2f} ms hits={cnt}")
    ms = float(np.mean(times) * 1e3)
    st = stats[-1]
    entries_per_s = float(np.mean([s.entries / t for s, t in zip(stats, times)]))
    level_ms = float(np.mean([s.level_lane_ms for s in stats]))  # the two trie-expansion kernels of every level
    launches = max(1, st.level_lane_launches)
    alg_bytes = st.level_alg_bytes()
    achieved = alg_bytes / (level_ms * 1e-3) / 1e9 if level_ms > 0 else 0.0
    traffic = measured_traffic()  # HBM bytes per launch, rocprofv3 counters
    out = {
        "metric": METRIC,
        "value": m * n / (ms * 1e-3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "m": m, "H": H},
        "dp_entries_per_s": entries_per_s,
        "p50_ms": float(np.percentile(times, 50) * 1e3),
        "p99_ms": float(np.percentile(times, 99) * 1e3),
        "hits": int(cnt),
        "kernels_ms": {"level": float(np.mean([s.level_ms for s in stats])), "level_lane": level_ms,
                       "chain_start": float(np.mean([s.start_ms for s in stats])),
                       "chain_lane_with_live_wave_pass": float(np.mean([s.general_ms for s in stats])),
                       "chain_wave_leftover": float(np.mean([s.wide_ms for s in stats])),
                       "sort_merge": float(np.mean([s.merge_ms for s in stats]))},
        "search_stats": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in st.as_dict().items()},
        "roofline": {"kernel": LEVEL_KERNEL, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_GBps": (traffic / (level_ms / launches * 1e-3) / 1e9) if traffic else None,
                     "alg_bytes_per_launch": alg_bytes / launches, "avg_launch_ms": level_ms / launches,
                     "launches_per_step": int(st.level_lane_launches)},
    }
    if not args.no_extras:
        log("autotuner: launch shapes")
        shapes, rep = ws.autotune(dq, H, sc, reps=2)
        tuned = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ws.search_device(dq, H, sc, **shapes)
            torch.cuda.synchronize()
            tuned.append(time.perf_counter() - t0)
        out["autotune"] = {"shapes": shapes, "default_device_ms": rep["default_ms"], "best_device_ms": rep["best_ms"],
                           "trials": len(rep["trials"]), "tuned_step_ms": float(np.mean(tuned) * 1e3)}
        log("learned scheduling: trace, train, timed searches")
        out["learned_scheduling"] = learned_scheduling(alae, ws, dq, H, sc, args.steps, ms)
        log("serving: Poisson arrivals")
        out["serving"] = serving(alae, idx, T)
        log("batched search against single-query searches")
        out["batched"] = batched_vs_single(alae)
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
