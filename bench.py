"""Benchmark of the exact local-alignment search on one MI355X.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--no-extras]

Headline workload (batched DNA): 256 queries with log-uniform lengths
500-50,000, each with 20 planted mutated copies of its segments (200-2,000
bases, 15% substitutions, 2% indels) in a 1e9-base i.i.d. text;
<1,-3,-5,-2>, H=30.  A step is one batched search of all 256 queries against
the resident index: seeding, every trie level, chains, hit emission, sort and
max-merge, with every query's sorted hits left in device memory.  The queries
are in HBM when the timed region starts; value = sum(m) * n / step time.

Beside the headline the JSON line carries: the same step with the hits copied
to pinned host memory (to_host), the looped single-query searches of the same
256 queries (batched speedup), the roofline of the trie-expansion kernels at
this size, the filtering ratio of Equation 5 (the same search under BWT-SW's
zero-floor rule), the DNA long-query search (text 1e8, query 1e5) with its
autotuner and learned-ordering legs, serving with Poisson arrivals on the 1e9
index, and the CPU oracle timed on the host's cores.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective m*n cell-updates/s + DP entries/s at exact hits; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
LEVEL_KERNEL = "k_level_tasks+k_expand_children"  # the trie-expansion step of one level (node phase, child phase)
TRAFFIC_PROFILE = {"batched": "trie_expansion_traffic_batched_dna.md",
                   "long_query": "trie_expansion_traffic_dna_long_query.md"}
# Under BWT-SW's zero-floor rule the rows kept do not depend on H (no score or length filter
# reads it), so its entry count is taken with a threshold no score reaches: without the
# domination test every start inside a planted homolog re-emits that homolog's hit cells, and
# those duplicate records would not fit the 32-bit record offsets at these sizes.
NO_OUTPUT_H = 1 << 20
ZERO_FLOOR_NOTE = ("entries under BWT-SW's zero-floor rule counted with hit output off (the rows it keeps do not "
                   "depend on H); its time excludes emitting and merging hits, so the speedup is a lower bound")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cores() -> int:
    """Cores this process may run on (its CPU share), at most 16 (the share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    out = fn()
    sync()
    return out, time.perf_counter() - t0


def measured_traffic(workload):
    """HBM bytes per level of the trie-expansion kernels on a workload from its committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a device-copy
    calibration), or None when the kernel sources or the host loop changed since."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", TRAFFIC_PROFILE[workload])
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


def roofline(stats_list, workload):
    level_ms = float(np.mean([s.level_lane_ms for s in stats_list]))
    st = stats_list[-1]
    launches = max(1, st.level_lane_launches)
    alg = st.level_alg_bytes()
    achieved = alg / (level_ms * 1e-3) / 1e9 if level_ms > 0 else 0.0
    traffic = measured_traffic(workload)
    return {"kernel": LEVEL_KERNEL, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_GBps": (traffic / (level_ms / launches * 1e-3) / 1e9) if traffic else None,
            "alg_bytes_per_launch": alg / launches, "avg_launch_ms": level_ms / launches,
            "launches_per_step": int(st.level_lane_launches)}


def kernels_ms(stats_list):
    f = lambda k: float(np.mean([getattr(s, k) for s in stats_list]))  # noqa: E731
    return {"level": f("level_ms"), "level_lane": f("level_lane_ms"), "chain_start": f("start_ms"),
            "chain_lane_with_live_wave_pass": f("general_ms"), "chain_wave_leftover": f("wide_ms"),
            "sort_merge": f("merge_ms")}


def wave_walkers(stats_list):
    """The wave walkers' share: entries, rows stepped, the span of the pass that runs beside the
    lane walker, and the chain item that took one block longest (its rows depend on each other, so
    its walk is a serial chain of row steps: its time over its rows is the latency of one step)."""
    st = stats_list[-1]
    live = float(np.mean([s.live_ms for s in stats_list]))
    return {"entries": int(st.wide_entries), "rows": int(st.wide_steps), "max_rows_one_chain": int(st.wide_max_steps),
            "live_pass_ms": live, "entries_per_s": st.wide_entries / (live * 1e-3) if live > 0 else None,
            "entries_per_row": st.wide_entries / max(1, st.wide_steps),
            "slowest_chain_ms": float(st.wide_slowest_ms), "slowest_chain_rows": int(st.wide_slowest_rows),
            "slowest_chain_start_ms": float(st.wide_slowest_start_ms),
            "us_per_row_step": st.wide_slowest_ms * 1e3 / st.wide_slowest_rows if st.wide_slowest_rows else None}


def level_graph_leg(alae, torch, ws, H, sc):
    """Short single queries on the resident 1e9-base index, with the level loop host-driven
    (level_graph 0) and device-driven from captured graphs (level_graph 8): median search time
    of 7 after two warm-ups, and the hit counts of both, which must agree."""
    rng = np.random.default_rng(12)
    sync = torch.cuda.synchronize
    out = {"note": "random DNA queries (no homolog in the text); graphs are captured in the warm-ups "
                   "and replayed in the timed searches"}
    for m in (100, 1000, 10000):
        dq = torch.from_numpy(rng.integers(0, 4, size=m).astype(np.uint8)).to("cuda")
        row = {}
        for K in (0, 8):
            for _ in range(2):
                ws.search_device(dq, H, sc, level_graph=K)
            st = alae.Stats()
            runs = [timed(lambda: ws.search_device(dq, H, sc, stats=st, level_graph=K), sync) for _ in range(7)]
            row[f"ms_level_graph_{K}"] = float(np.median([dt for _, dt in runs]) * 1e3)
            row[f"hits_level_graph_{K}"] = int(runs[-1][0])
            if K:
                row["device_levels"] = int(st.device_levels)
                row["levels"] = int(st.levels)
                row["graph_captures_last_search"] = int(st.graph_captures)
        if row["hits_level_graph_0"] != row["hits_level_graph_8"]:
            raise SystemExit(f"level_graph changed the hit count at m={m}: {row}")
        out[f"m={m}"] = row
    log(f"level graph: {out}")
    return out


def batched_leg(alae, torch, args):
    """The headline: one batched search of 256 queries against the 1e9-base index."""
    from paper_1208_0274_amd import synth

    t0 = time.perf_counter()
    w = synth.batched_dna()
    T, qs, H = w["text"], w["queries"], int(w["H"])
    n = int(T.shape[0])
    lens = [int(q.shape[0]) for q in qs]
    sum_m = int(sum(lens))
    log(f"batched workload: n={n} queries={len(qs)} sum_m={sum_m} ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    idx = alae.Index.build(T, "dna")
    build_s = time.perf_counter() - t0
    log(f"index of 1e9 bases built on the GPU in {build_s:.1f} s")
    sc = alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"])
    ws = alae.Workspace(idx)
    cat = torch.from_numpy(np.concatenate(qs)).to("cuda")
    sync = torch.cuda.synchronize
    for i in range(args.warmup):
        st = alae.Stats()
        (cnt, dt) = timed(lambda: ws.search_device_batch(cat, lens, H, sc, stats=st), sync)
        log(f"warmup {i}: {dt * 1e3:.1f} ms hits={cnt} entries={st.entries}")
    times, stats = [], []
    for i in range(args.steps):
        st = alae.Stats()
        (cnt, dt) = timed(lambda: ws.search_device_batch(cat, lens, H, sc, stats=st), sync)
        times.append(dt)
        stats.append(st)
        log(f"step {i}: {dt * 1e3:.1f} ms hits={cnt}")
    ms = float(np.mean(times) * 1e3)
    st = stats[-1]
    res = {"ms": ms, "times": times, "stats": stats, "hits": int(cnt), "sum_m": sum_m, "n": n, "H": H,
           "index_build_s": build_s}
    # the same step with the hits taken to pinned host memory
    keys_h = torch.empty(cnt, dtype=torch.int64, pin_memory=True)
    scores_h = torch.empty(cnt, dtype=torch.int32, pin_memory=True)
    host_times = []
    for i in range(min(3, args.steps)):
        def step():
            ws.search_device_batch(cat, lens, H, sc)
            return ws.copy_result(keys_h, scores_h)

        (c2, dt) = timed(step, sync)
        host_times.append(dt)
        log(f"to host {i}: {dt * 1e3:.1f} ms ({c2} hits, {c2 * 12 / 1e9:.2f} GB)")
    hms = float(np.mean(host_times) * 1e3)
    res["to_host"] = {"ms_per_step": hms, "value": sum_m * n / (hms * 1e-3), "hit_bytes": int(cnt) * 12,
                      "note": "launch to sorted hits in pinned host memory (PCIe included)"}
    del keys_h, scores_h
    if not args.no_extras:
        # the plain single-query form: the 256 searches one after another on the same workspace
        dqs = [torch.from_numpy(np.ascontiguousarray(q)).to("cuda") for q in qs]
        ws.search_device(dqs[0], H, sc)

        def loop():
            return sum(ws.search_device(d, H, sc) for d in dqs)

        (tot, dt) = timed(loop, sync)
        if tot != cnt:
            raise SystemExit(f"single-query searches found {tot} hits, the batch {cnt}")
        res["single_query_loop"] = {"ms": dt * 1e3, "speedup_batched": dt * 1e3 / ms}
        log(f"single-query loop: {dt * 1e3:.1f} ms, batched speedup {dt * 1e3 / ms:.2f}")
        # Equation 5 on a sample of the batch: the first 16 queries under ALAE's filters and
        # under BWT-SW's zero-floor rule alone
        k = 16
        sub = cat[:sum(lens[:k])]
        st_a, st_b = alae.Stats(), alae.Stats()
        (ca, ta) = timed(lambda: ws.search_device_batch(sub, lens[:k], H, sc, stats=st_a), sync)
        (cb, tb) = timed(lambda: ws.search_device_batch(sub, lens[:k], NO_OUTPUT_H, sc, stats=st_b,
                                                        zero_floor_only=True), sync)
        res["filtering"] = {"sample": f"the first {k} queries of the batch (sum m = {sum(lens[:k])}) on the 1e9 text",
                            "entries_alae": int(st_a.entries), "entries_zero_floor_only": int(st_b.entries),
                            "filtering_ratio": (st_b.entries - st_a.entries) / max(1, st_b.entries),
                            "ms_alae": ta * 1e3, "ms_zero_floor_only_no_output": tb * 1e3, "speedup_at_least": tb / ta,
                            "note": ZERO_FLOOR_NOTE}
        log(f"filtering (batched sample): {res['filtering']}")
        res["level_graph"] = level_graph_leg(alae, torch, ws, H, sc)
        del dqs
    ws.free()
    res["idx"] = idx
    res["T"] = T
    res["queries"] = qs
    return res


def long_query_leg(alae, torch, args):
    """DNA long query (text 1e8 + 1,000 planted segments, query 1e5, H=30): one search a step."""
    from paper_1208_0274_amd import synth

    w = synth.dna_long_query()
    T, P, H = w["text"], w["queries"][0], int(w["H"])
    idx = alae.Index.build(T, "dna")
    sc = alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"])
    ws = alae.Workspace(idx)
    dq = torch.from_numpy(P).to("cuda")
    sync = torch.cuda.synchronize
    for _ in range(2):
        ws.search_device(dq, H, sc)
    times, stats = [], []
    for _ in range(max(3, args.steps // 2)):
        st = alae.Stats()
        (cnt, dt) = timed(lambda: ws.search_device(dq, H, sc, stats=st), sync)
        times.append(dt)
        stats.append(st)
    ms = float(np.mean(times) * 1e3)
    out = {"workload": "DNA long query: text 1e8 i.i.d. ACGT + 1,000 planted mutated query segments "
                       "(200-2,000, 15% subs, 2% indels); query 1e5; <1,-3,-5,-2>; H=30",
           "ms_per_search": ms, "cells_per_s": P.shape[0] * T.shape[0] / (ms * 1e-3), "hits": int(cnt),
           "dp_entries_per_s": float(np.mean([s.entries / t for s, t in zip(stats, times)])),
           "kernels_ms": kernels_ms(stats), "roofline_trie_expansion": roofline(stats, "long_query"),
           "wave_walkers": wave_walkers(stats)}
    if args.long_query_only:
        log(f"long query: {ms:.1f} ms")
        ws.free()
        idx.free()
        return out
    st_b = alae.Stats()
    (cb, tb) = timed(lambda: ws.search_device(dq, NO_OUTPUT_H, sc, stats=st_b, zero_floor_only=True), sync)
    out["filtering"] = {"entries_alae": int(stats[-1].entries), "entries_zero_floor_only": int(st_b.entries),
                        "filtering_ratio": (st_b.entries - stats[-1].entries) / max(1, st_b.entries),
                        "ms_alae": ms, "ms_zero_floor_only_no_output": tb * 1e3, "speedup_at_least": tb * 1e3 / ms,
                        "note": ZERO_FLOOR_NOTE}
    log(f"long query: {ms:.1f} ms; filtering {out['filtering']}")
    if not args.no_extras:
        shapes, rep = ws.autotune(dq, H, sc, reps=2)
        tuned = [timed(lambda: ws.search_device(dq, H, sc, **shapes), sync)[1] for _ in range(3)]
        out["autotune"] = {"shapes": shapes, "default_device_ms": rep["default_ms"], "best_device_ms": rep["best_ms"],
                           "trials": len(rep["trials"]), "tuned_step_ms": float(np.mean(tuned) * 1e3)}
        out["learned_scheduling"] = learned_scheduling(alae, torch, ws, dq, H, sc, ms)
    ws.free()
    idx.free()
    return out


def learned_scheduling(alae, torch, ws, dq, H, sc, plain_ms, reps=5):
    """Trace one search, train the work predictor on the GPU, then time the search with the
    learned order + partition of the walkers' queues."""
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
    sync = torch.cuda.synchronize
    for name, kw in (("order_ms", dict(order_model=net, order_queues=2)),
                     ("order_partition_ms", dict(order_model=net, order_queues=2, partition_threshold=9.0))):
        times = []
        for _ in range(reps):
            st = alae.Stats()
            times.append(timed(lambda: ws.search_device(dq, H, sc, stats=st, **kw), sync)[1])
        out[name] = float(np.mean(times) * 1e3)
        out[name.replace("_ms", "_moved")] = int(st.partitioned)
    out["gain_order"] = plain_ms / out["order_ms"]
    out["gain_order_partition"] = plain_ms / out["order_partition_ms"]
    out["total_s"] = time.perf_counter() - t0
    net.free()
    return out


def serving(alae, idx, T, rates=(10.0, 30.0, 100.0, 300.0, 1000.0), count=200):
    """Poisson arrivals of queries with log-uniform lengths 100-100,000 (half carrying a mutated
    200-2,000 text segment) against the resident 1e9 index; per rate: completed requests per second
    and submit-to-completion p50/p99 over `count` requests."""
    from paper_1208_0274_amd import synth

    sc = alae.make_scoring()
    out = []
    srv = alae.Server(idx, max_batch=16)  # default slots: two on a text this large
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
        results = [srv.poll(i) for i in ids]
        wall = time.perf_counter() - t0
        st = srv.stats()
        out.append({"rate_qps": rate, "requests": count, "throughput_qps": count / wall, "p50_ms": st["p50_ms"],
                    "p99_ms": st["p99_ms"], "mean_batch": st["mean_batch"], "searches": st["batches"],
                    "mean_m": float(np.mean([q.shape[0] for q in qs]))})
        log(f"serving at {rate} q/s: {out[-1]}")
    srv.close()
    # the last rate's results against the same queries searched alone (a sample of eight)
    same = 0
    sample = list(range(0, count, max(1, count // 8)))[:8]
    for k in sample:
        alone = alae.search(idx, qs[k], 30, sc)
        same += int(all(np.array_equal(x, y) for x, y in zip(alone, results[k])))
    out.append({"identical_to_alone": f"{same} of {len(sample)} sampled requests of the last rate"})
    log(f"serving: {out[-1]}")
    return out


def cpu_baseline(T, qs, budget_s: float):
    """The oracle as it stands, on every core of this host's share, on a bounded sample of the
    batched workload: the median-length query against the first rows of the text, cut into one
    chunk per thread, each chunk recomputing L_max rows in front of it (exact by Theorem 1) and
    at least 2 L_max rows long."""
    import oracle

    lens = np.array([q.shape[0] for q in qs])
    P = qs[int(np.argsort(lens)[len(lens) // 2])]
    m = int(P.shape[0])
    cores = host_cores()
    sub = oracle.scoring_table(4, 1, -3)
    lmax = oracle.lmax(m, 1, -5, -2, 30)
    L = 4 * lmax  # single-thread rate on a short slice
    t0 = time.perf_counter()
    oracle.sw_hits(T[:L], P, sub, -5, -2, 30, threads=1)
    r1 = m * L / max(time.perf_counter() - t0, 1e-6)
    rows_per_thread = max(2 * lmax, int(r1 * budget_s / m) - lmax)
    rows = min(int(T.shape[0]), cores * rows_per_thread)
    t0 = time.perf_counter()
    _, cells = oracle.sw_hits(T[:rows], P, sub, -5, -2, 30, threads=cores, return_cells=True)
    dt = time.perf_counter() - t0
    return {"value": m * rows / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "per_core": m * rows / dt / cores, "wall_s": dt, "cells_computed": int(cells),
            "sample": f"median-length query of the batch (m={m}) against the first {rows} text characters, "
                      f"{cores} threads of {rows // cores} text rows each plus L_max={lmax} rows of overlap, "
                      f"{dt:.1f} s; value counts the m x {rows} cells of the sample"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline and its to-host timing")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--level-graph-only", action="store_true",
                    help="only the short-query leg with host- and device-driven levels, on the 1e9-base index "
                         "(to profile it alone)")
    ap.add_argument("--long-query-only", action="store_true",
                    help="only the DNA long-query leg's searches, without its filtering, tuning and scheduling "
                         "extras (to profile it alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; the search would shard by text range, one index part per GPU",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1208_0274_amd import alae

    if args.level_graph_only:
        from paper_1208_0274_amd import synth

        w = synth.batched_dna()
        idx = alae.Index.build(w["text"], "dna")
        ws = alae.Workspace(idx)
        out = level_graph_leg(alae, torch, ws, int(w["H"]), alae.make_scoring(w["sa"], w["sb"], w["sg"], w["ss"]))
        ws.free()
        idx.free()
        print(json.dumps({"level_graph": out}), flush=True)
        return
    if args.long_query_only:
        args.no_extras = True
        print(json.dumps({"dna_long_query": long_query_leg(alae, torch, args)}), flush=True)
        return
    b = batched_leg(alae, torch, args)
    stats, times = b["stats"], b["times"]
    ms = b["ms"]
    out = {
        "metric": METRIC,
        "value": b["sum_m"] * b["n"] / (ms * 1e-3),
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
        "config": {"workload": "batched DNA: 256 queries (log-uniform 500-50,000), 20 planted mutated segments of "
                               "each (200-2,000, 15% subs, 2% indels) in a 1e9 i.i.d. ACGT text; <1,-3,-5,-2>; "
                               "H=30", "n": b["n"], "queries": 256, "sum_m": b["sum_m"], "H": b["H"],
                   "batch_columns": 1 << 19},
        "dp_entries_per_s": float(np.mean([s.entries / t for s, t in zip(stats, times)])),
        "p50_ms": float(np.percentile(times, 50) * 1e3),
        "p99_ms": float(np.percentile(times, 99) * 1e3),
        "hits": b["hits"],
        "to_host": b["to_host"],
        "index_build_s": b["index_build_s"],
        "kernels_ms": kernels_ms(stats),
        "search_stats": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in stats[-1].as_dict().items()},
        "roofline": roofline(stats, "batched"),
        "wave_walkers": wave_walkers(stats),
    }
    for k in ("single_query_loop", "filtering", "level_graph"):
        if k in b:
            out[k] = b[k]
    if not args.no_extras:
        log("serving: Poisson arrivals on the 1e9 index")
        out["serving"] = serving(alae, b["idx"], b["T"])
    b["idx"].free()
    if not args.no_extras:
        log("DNA long query")
        out["dna_long_query"] = long_query_leg(alae, torch, args)
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(b["T"], b["queries"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
