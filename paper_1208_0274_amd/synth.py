"""Seeded synthetic inputs shaped like the paper's workloads (Section 7).

This module only draws random sequences; it holds none of the search
method's arithmetic, so both the GPU path's tests and the CPU oracle may take
their inputs from it.

Every workload is a dict with ``text`` (uint8 codes), ``queries`` (list of
uint8 code arrays), the scoring scheme, ``H``, the alphabet and the ground
truth of what was planted.  Codes: DNA A,C,G,T -> 0..3; protein
ARNDCQEGHILKMFPSTWYV -> 0..19.

The paper's data (GRCh37 human text, MGSCv37 chr1 mouse queries, UniParc
proteins) are not available; i.i.d. uniform sequences with planted mutated
copies stand in for them.  The protein background is uniform over the 20
residues (the standard background frequencies are not available here).
"""
from __future__ import annotations

import numpy as np

DNA = "ACGT"
PROTEIN = "ARNDCQEGHILKMFPSTWYV"

SEED_BASE = 0xA1AE0000


def rng_for(config_index: int, purpose: int) -> np.random.Generator:
    """Independent stream per (config, purpose): 0 text, 1 query, 2 planting, 3 arrivals."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + config_index, purpose])))


def random_seq(rng: np.random.Generator, n: int, sigma: int) -> np.ndarray:
    return rng.integers(0, sigma, size=n, dtype=np.uint8)


def mutate(rng: np.random.Generator, seg: np.ndarray, sigma: int, p_sub: float, p_indel: float) -> np.ndarray:
    """Per source position: with p_indel delete it (half the time) or insert one
    random residue before it; else with p_sub substitute it (uniformly by one of
    the other residues); else copy it."""
    L = seg.shape[0]
    u = rng.random(L)
    half = rng.random(L) < 0.5
    indel = u < p_indel
    sub = (~indel) & (u < p_indel + p_sub)
    delete = indel & half
    insert = indel & ~half
    out = seg.copy()
    shift = rng.integers(1, sigma, size=L, dtype=np.int64)
    out[sub] = ((seg[sub].astype(np.int64) + shift[sub]) % sigma).astype(np.uint8)
    ins_chars = rng.integers(0, sigma, size=L, dtype=np.uint8)
    # output layout: for each source position, the inserted residue (if any), then the residue unless deleted
    keep = ~delete
    n_out = int(keep.sum() + insert.sum())
    res = np.empty(n_out, dtype=np.uint8)
    # positions in output: inserted char comes first
    cnt = keep.astype(np.int64) + insert.astype(np.int64)
    start = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    res[start[insert]] = ins_chars[insert]
    res[(start + insert.astype(np.int64))[keep]] = out[keep]
    return res


def place_nonoverlapping(rng: np.random.Generator, n: int, lengths: np.ndarray) -> np.ndarray:
    """Uniform sorted non-overlapping start offsets for segments of the given lengths
    (in the given order) inside a text of length n."""
    total = int(lengths.sum())
    if total > n:
        raise ValueError("segments do not fit into the text")
    free = n - total
    pts = np.sort(rng.integers(0, free + 1, size=lengths.shape[0]))
    return pts + np.concatenate(([0], np.cumsum(lengths)[:-1]))


def plant_segments(rng: np.random.Generator, text: np.ndarray, sources: list, sigma: int,
                   p_sub: float, p_indel: float):
    """Mutate each source segment and overwrite the text with it at uniform
    non-overlapping positions.  Returns the list of (text_start, text_len)."""
    copies = [mutate(rng, s, sigma, p_sub, p_indel) for s in sources]
    lens = np.array([c.shape[0] for c in copies], dtype=np.int64)
    order = rng.permutation(len(copies))
    starts = place_nonoverlapping(rng, text.shape[0], lens[order])
    plants = []
    for k, idx in enumerate(order):
        st = int(starts[k])
        c = copies[idx]
        text[st:st + c.shape[0]] = c
        plants.append((st, int(c.shape[0]), int(idx)))
    return plants


def _dna_scoring():
    return dict(sa=1, sb=-3, sg=-5, ss=-2, matrix=None)


def small_dna(planted: bool = False, H: int = 18):
    """Plain method, single query: text 1e5 i.i.d. ACGT, query 1e3, <1,-3,-5,-2>, H=18.

    ``planted=True`` adds 10 query segments of 50-200 characters mutated at
    15% substitutions / 2% indels, so that the hit set is not empty."""
    text = random_seq(rng_for(0, 0), 100_000, 4)
    query = random_seq(rng_for(0, 1), 1_000, 4)
    plants = []
    if planted:
        r = rng_for(0, 2)
        srcs = []
        for _ in range(10):
            L = int(r.integers(50, 201))
            y = int(r.integers(0, query.shape[0] - L + 1))
            srcs.append(query[y:y + L])
        plants = plant_segments(r, text, srcs, 4, 0.15, 0.02)
    return dict(name="small-dna" + ("-planted" if planted else ""), alphabet="dna", sigma=4, text=text,
                queries=[query], H=H, plants=plants, **_dna_scoring())


def dna_long_query(n: int = 100_000_000, m: int = 100_000, n_plants: int = 1000, H: int = 30):
    """DNA long query: text 1e8 i.i.d. ACGT with 1,000 planted mutated query
    segments (lengths 200-2,000, 15% substitutions, 2% indels); query 1e5;
    <1,-3,-5,-2>; H=30."""
    text = random_seq(rng_for(1, 0), n, 4)
    query = random_seq(rng_for(1, 1), m, 4)
    r = rng_for(1, 2)
    srcs = []
    for _ in range(n_plants):
        L = int(r.integers(200, 2001))
        L = min(L, m)
        y = int(r.integers(0, m - L + 1))
        srcs.append(query[y:y + L])
    plants = plant_segments(r, text, srcs, 4, 0.15, 0.02)
    return dict(name="dna-long-query", alphabet="dna", sigma=4, text=text, queries=[query], H=H, plants=plants,
                **_dna_scoring())


def protein_standin(n: int = 50_000_000, m: int = 5_000, n_plants: int = 500, H: int = 45, p_sub: float = 0.10):
    """Protein: text 5e7 residues with 500 planted mutated query segments
    (lengths 50-500, 3% indels); query 5,000 residues.

    BLOSUM62 and the standard background frequencies are not available, so
    this stand-in uses a uniform background, uniform substitutions and the
    paper's own protein scheme <1,-3,-11,-1> (Section 7.5).  Under that
    scheme a 30% substitution rate scores below zero per residue (no planted
    copy would reach H), so the stand-in substitutes 10% of residues."""
    text = random_seq(rng_for(2, 0), n, 20)
    query = random_seq(rng_for(2, 1), m, 20)
    r = rng_for(2, 2)
    srcs = []
    for _ in range(n_plants):
        L = int(r.integers(50, 501))
        y = int(r.integers(0, m - L + 1))
        srcs.append(query[y:y + L])
    plants = plant_segments(r, text, srcs, 20, p_sub, 0.03)
    return dict(name="protein-standin", alphabet="protein", sigma=20, text=text, queries=[query], H=H, plants=plants,
                sa=1, sb=-3, sg=-11, ss=-1, matrix=None)


def loguniform_lengths(rng: np.random.Generator, k: int, lo: int, hi: int) -> np.ndarray:
    return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=k))).astype(np.int64)


def batched_dna(n: int = 1_000_000_000, k: int = 256, copies: int = 20, H: int = 30,
            m_lo: int = 500, m_hi: int = 50_000):
    """Batched: k DNA queries with log-uniform lengths in [500, 50000], each with
    `copies` planted mutated segments (lengths 200-2,000, 15%/2%) in an i.i.d.
    ACGT text of n bases; <1,-3,-5,-2>; H=30.  Each planted copy is a segment
    of its query (the reading that keeps the hit set within device memory)."""
    text = random_seq(rng_for(3, 0), n, 4)
    rq = rng_for(3, 1)
    lens = loguniform_lengths(rq, k, m_lo, m_hi)
    queries = [random_seq(rq, int(L), 4) for L in lens]
    r = rng_for(3, 2)
    srcs = []
    owners = []
    for qi, q in enumerate(queries):
        for _ in range(copies):
            L = min(int(r.integers(200, 2001)), q.shape[0])
            y = int(r.integers(0, q.shape[0] - L + 1))
            srcs.append(q[y:y + L])
            owners.append(qi)
    plants = plant_segments(r, text, srcs, 4, 0.15, 0.02)
    plants = [(st, ln, owners[idx]) for (st, ln, idx) in plants]
    return dict(name="batched-dna", alphabet="dna", sigma=4, text=text, queries=queries, H=H, plants=plants,
                **_dna_scoring())


def poisson_arrivals(rate: float, count: int, config_index: int = 4) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: exponential gaps."""
    r = rng_for(config_index, 3)
    return np.cumsum(r.exponential(1.0 / rate, size=count))


def serving_queries(text: np.ndarray, count: int, m_lo: int = 100, m_hi: int = 100_000,
                    homolog_frac: float = 0.5, config_index: int = 4):
    """Queries for the serving workload: log-uniform lengths; a fraction carry
    one planted homolog (a mutated text segment of 200-2,000 bases embedded at
    a uniform query offset)."""
    r = rng_for(config_index, 1)
    lens = loguniform_lengths(r, count, m_lo, m_hi)
    out = []
    for L in lens:
        q = random_seq(r, int(L), 4)
        if r.random() < homolog_frac and L >= 200:
            hl = min(int(r.integers(200, 2001)), int(L))
            st = int(r.integers(0, text.shape[0] - hl + 1))
            seg = mutate(r, text[st:st + hl], 4, 0.15, 0.02)[:L]
            off = int(r.integers(0, L - seg.shape[0] + 1))
            q[off:off + seg.shape[0]] = seg
        out.append(q)
    return out


def decode(codes: np.ndarray, alphabet: str = DNA) -> str:
    lut = np.frombuffer(alphabet.encode(), dtype=np.uint8)
    return lut[codes].tobytes().decode()
