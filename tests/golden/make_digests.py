"""Write the oracle's hit digests for the full-size workloads.

    python tests/golden/make_digests.py dna_long_query [--threads 7]
    python tests/golden/make_digests.py batched_dna [--threads 7]

Only the CPU oracle (``oracle.sw_hits``) computes hits here; the inputs come
from the seeded generators of ``paper_1208_0274_amd.synth`` (random numbers
only, none of the method's arithmetic).  Nothing from the GPU library is
imported.

dna_long_query (text 1e8, query 1e5, <1,-3,-5,-2>, H=30): every hit of the
whole text, digested per bin of 100,000 text ends ->
``dna_long_query_digests.txt`` (lines: bin_lo bin_hi count sum1 sum2).

batched_dna (256 queries of 500-50,000, 20 planted copies each, text 1e9,
<1,-3,-5,-2>, H=30): for every query, one window per planted copy of that
query (text ends from the copy's start to 1,000 past its end) and one window
of 1,000,000 text ends at a seeded uniform position ->
``batched_dna_window_digests.txt`` (lines: query lo hi count sum1 sum2).

Exactness of windows (Theorem 1, Equation 1): an alignment scoring at least H
spans at most L_max text characters, so the hits with text end in [a, b) are
the oracle's hits on T[a - L_max .. b) restricted to those ends.  The script
appends as it goes and resumes from what a file already holds.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from hitdigest import digest, digest_by_bins, read_digest_file  # noqa: E402
from paper_1208_0274_amd import synth  # noqa: E402

DNA_BIN = 100_000
DNA_SEGMENT = 20_000_000
C4_TAIL = 1000
C4_RANDOM_WINDOW = 1_000_000
C4_WINDOW_SEED = 0xC4


def dna_long_query(threads: int):
    path = os.path.join(HERE, "dna_long_query_digests.txt")
    w = synth.dna_long_query()
    T, P, H = w["text"], w["queries"][0], w["H"]
    n, m = T.shape[0], P.shape[0]
    sub = oracle.scoring_table(4, w["sa"], w["sb"])
    lmax = oracle.lmax(m, int(sub.max()), w["sg"], w["ss"], H)
    done = set()
    if os.path.exists(path):
        done = {r[0] for r in read_digest_file(path)}
    else:
        with open(path, "w") as f:
            f.write("# DNA long query: text 1e8 i.i.d. ACGT + 1,000 planted mutated query segments, query 1e5,\n"
                    "# <1,-3,-5,-2>, H=30 (synth.dna_long_query).  Oracle hit digests per 100,000 text ends,\n"
                    "# written by tests/golden/make_digests.py from oracle.sw_hits alone.\n"
                    "# bin_lo bin_hi count sum1 sum2 (tests/hitdigest.py)\n")
    for a in range(0, n, DNA_SEGMENT):
        b = min(n, a + DNA_SEGMENT)
        edges = list(range(a, b, DNA_BIN)) + [b]
        if all(e in done for e in edges[:-1]):
            continue
        lo = max(0, a - lmax)
        t0 = time.time()
        j, t, s = oracle.sw_hits(T[lo:b], P, sub, w["sg"], w["ss"], H, t_lo=a - lo, t_hi=b - lo, threads=threads)
        t = t + lo
        dig = digest_by_bins(j, t, s, edges)
        with open(path, "a") as f:
            for k, (c, s1, s2) in enumerate(dig):
                f.write(f"{edges[k]} {edges[k + 1]} {c} {s1} {s2}\n")
        print(f"text ends [{a}, {b}): {j.shape[0]} hits in {time.time() - t0:.0f} s", flush=True)


def c4_windows(w):
    """Per query: its planted copies' windows and one seeded random window."""
    n = w["text"].shape[0]
    rng = np.random.default_rng(C4_WINDOW_SEED)
    wins = []
    for qi in range(len(w["queries"])):
        for (st, ln, owner) in w["plants"]:
            if owner == qi:
                wins.append((qi, st, min(n, st + ln + C4_TAIL)))
        a = int(rng.integers(0, n - C4_RANDOM_WINDOW + 1))
        wins.append((qi, a, a + C4_RANDOM_WINDOW))
    return wins


def batched_dna(threads: int):
    path = os.path.join(HERE, "batched_dna_window_digests.txt")
    w = synth.batched_dna()
    T, H = w["text"], w["H"]
    sub = oracle.scoring_table(4, w["sa"], w["sb"])
    wins = c4_windows(w)
    done = set()
    if os.path.exists(path):
        done = {(r[0], r[1], r[2]) for r in read_digest_file(path)}
    else:
        with open(path, "w") as f:
            f.write("# Batched DNA: 256 queries (log-uniform 500-50,000), 20 planted mutated segments of each in a\n"
                    "# 1e9 i.i.d. ACGT text, <1,-3,-5,-2>, H=30 (synth.batched_dna).  Per query: one window per\n"
                    "# planted copy (its start to 1,000 past its end) and one seeded random window of 1e6 text\n"
                    "# ends.  Oracle hit digests, written by tests/golden/make_digests.py from oracle.sw_hits.\n"
                    "# query lo hi count sum1 sum2 (tests/hitdigest.py)\n")
    todo = [x for x in wins if x not in done]
    lm = {qi: oracle.lmax(q.shape[0], int(sub.max()), w["sg"], w["ss"], H) for qi, q in enumerate(w["queries"])}
    # largest first for balance
    todo.sort(key=lambda x: -(x[2] - x[1] + lm[x[0]]) * w["queries"][x[0]].shape[0])

    def one(win):
        qi, a, b = win
        lo = max(0, a - lm[qi])
        j, t, s = oracle.sw_hits(T[lo:b], w["queries"][qi], sub, w["sg"], w["ss"], H, t_lo=a - lo, t_hi=b - lo,
                                 threads=1)
        return win, digest(j, t + lo, s)

    t0 = time.time()
    cells = 0
    with cf.ThreadPoolExecutor(max_workers=threads) as ex, open(path, "a") as f:
        for k, (win, (c, s1, s2)) in enumerate(ex.map(one, todo)):
            f.write(f"{win[0]} {win[1]} {win[2]} {c} {s1} {s2}\n")
            f.flush()
            cells += (win[2] - win[1] + lm[win[0]]) * w["queries"][win[0]].shape[0]
            if k % 100 == 0:
                print(f"{k + 1}/{len(todo)} windows, {cells:.3e} cells, {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["dna_long_query", "batched_dna"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    if a.workload == "dna_long_query":
        dna_long_query(a.threads)
    else:
        batched_dna(a.threads)


if __name__ == "__main__":
    main()
