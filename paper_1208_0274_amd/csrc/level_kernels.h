// Expansion of trie nodes that still have several occurrences (Section 5,
// search (3)): every child X.c of a node X is one backward-search step on the
// FM-index of the reversed text, and its sparse row is computed from X's row
// (Section 2.2 with the filters of Section 3).
//
//   k_expand_level       one lane per node whose row has at most kLaneRow
//                        entries (almost all nodes);
//   k_expand_level_wide  one wave per node with a longer row (stretches the
//                        text repeats, e.g. overlapping copies of a query
//                        segment).
//
// Children with several occurrences form the next level; a child with one
// occurrence becomes a chain item (BWT row + depth + row) for the chain
// kernels.  Hits of multi-occurrence children are emitted here for every
// occurrence (Algorithm 1, lines 6-10).
#pragma once

#include "row_update.h"

namespace alae {

constexpr uint32_t kLaneRow = 32;

struct LevelOut {
    Node *onodes;   // next level, rows of at most kLaneRow entries
    Node *owide;    // next level, longer rows
    Entry *oent;    // entries of both
    Node *chains;   // children with one occurrence: lo = BWT row, hi = depth
    Entry *cent;
    uint64_t *hkeys;
    uint32_t *hscores;
    unsigned long long node_base, wide_base, ent_base, chain_base, cent_base, hit_base;
};

struct LevelCounts {
    uint32_t nodes, wide, entries, chains, centries, hits;
};

// WRITE == false counts what the node will write; WRITE == true writes it at
// the bases the wave allocated.
template <bool WRITE>
__device__ void expand_node(const SearchArgs &a, const Node &nd, const Entry *prow, int32_t d1, LevelCounts &n,
                            const LevelOut &o, Caps caps, uint32_t st[5]) {
    n.nodes = n.wide = n.entries = n.chains = n.centries = n.hits = 0;
    uint32_t o_lo[4] = {0, 0, 0, 0}, o_hi[4] = {0, 0, 0, 0};
    if (a.sigma == 4) {
        occ4_dna(a, (int64_t)nd.lo - 1, o_lo);
        occ4_dna(a, (int64_t)nd.hi, o_hi);
    }
    if (!WRITE) {
        const int bc = a.sigma == 4 ? kDnaBlockChars : kGenBlockChars;
        const int64_t b0 = nd.lo == 0 ? -1 : ((int64_t)nd.lo - 1) / bc;
        const int64_t b1 = (int64_t)nd.hi / bc;
        st[3] += (b0 >= 0 && b0 != b1) ? 2u : 1u;
    }
    for (int c = 0; c < a.sigma; ++c) {
        int64_t l, r;
        if (a.sigma == 4) {
            l = (int64_t)a.C[c] + o_lo[c];
            r = (int64_t)a.C[c] + o_hi[c] - 1;
        } else {
            l = (int64_t)a.C[c] + occ1_gen(a, c, (int64_t)nd.lo - 1);
            r = (int64_t)a.C[c] + occ1_gen(a, c, (int64_t)nd.hi) - 1;
        }
        if (l > r) continue;
        RowSink s;
        sink_init(s);
        s.lo = (uint32_t)l;
        s.hi = (uint32_t)r;
        const bool multi = l < r;
        if (!multi) s.emit_hits = false;  // located and emitted by the chain kernel
        if (WRITE) {
            s.out = multi ? o.oent + o.ent_base + n.entries : o.cent + o.cent_base + n.centries;
            s.hkeys = o.hkeys;
            s.hscores = o.hscores;
            s.hit_base = o.hit_base + n.hits;
            s.hit_cap = caps.hits;
        }
        child_row<WRITE>(a, prow, nd.len, c, d1, false, 0, s);
        n.hits += s.n_hits;
        if (WRITE) {
            st[0] += s.st_diag;
            st[1] += s.st_gap2;
            st[2] += s.st_gap3;
        }
        if (s.n_entries == 0) continue;
        if (multi) {
            if (WRITE) {
                Node cn;
                cn.lo = s.lo;
                cn.hi = s.hi;
                cn.off = (uint32_t)(o.ent_base + n.entries);
                cn.len = s.n_entries;
                if (s.n_entries > kLaneRow)
                    o.owide[o.wide_base + n.wide] = cn;
                else
                    o.onodes[o.node_base + n.nodes] = cn;
            }
            if (s.n_entries > kLaneRow)
                n.wide++;
            else
                n.nodes++;
            n.entries += s.n_entries;
        } else {
            if (WRITE) {
                Node cn;
                cn.lo = (uint32_t)l;
                cn.hi = (uint32_t)d1;
                cn.off = (uint32_t)(o.cent_base + n.centries);
                cn.len = s.n_entries;
                o.chains[o.chain_base + n.chains] = cn;
            }
            n.chains++;
            n.centries += s.n_entries;
        }
    }
}

// Child rows of a node are computed once into a per-lane LDS stage of
// kStage entries; the wave then allocates its outputs with one atomic per
// buffer and each lane copies its stage out.  A node whose children do not
// fit the stage is counted and written by two passes of expand_node instead.
// A parent row of at most kParent entries is copied to LDS first, with its
// loads issued together, so that the row updates read it at LDS latency.
constexpr int kStage = 8;
constexpr int kParent = 4;
constexpr int kStageWords = (kStage + kParent) * 5 + 1;  // one pad word: lanes start in different banks
constexpr int kLevelBlock = 128;

__global__ void __launch_bounds__(kLevelBlock) k_expand_level(SearchArgs a, const Node *nodes, uint32_t nn,
                                                              const Entry *ent, int32_t d1, LevelOut o, Caps caps,
                                                              Counters *cnt) {
    __shared__ uint32_t s_stage[kLevelBlock * kStageWords];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = t < nn;
    Node nd;
    nd.lo = nd.hi = nd.off = nd.len = 0;
    if (active) nd = nodes[t];
    Entry *stage = reinterpret_cast<Entry *>(s_stage + threadIdx.x * kStageWords);
    Entry *parent = stage + kStage;
    LevelCounts n = {0, 0, 0, 0, 0, 0};
    uint32_t st[5] = {0, 0, 0, 0, 0};
    // children: BWT range and staged entry count (entries 0 .. used-1 of the stage, in child order)
    uint32_t ch_lo[4] = {0, 0, 0, 0}, ch_hi[4] = {0, 0, 0, 0}, ch_n[4] = {0, 0, 0, 0};
    bool staged = false;
    const Entry *use_prow = nullptr;  // parent row of the two-pass path (LDS copy or global)
    uint32_t nxt4 = kNoNext;
    if (active) {
        const Entry *prow = ent + nd.off;
        if (nd.len >= 1 && nd.len <= (uint32_t)kParent) {
            // four independent loads (indexes clamped into the row), then the LDS copy
            const uint32_t last = nd.len - 1;
            const Entry e0 = prow[0];
            const Entry e1 = prow[last < 1 ? last : 1];
            const Entry e2 = prow[last < 2 ? last : 2];
            const Entry e3 = prow[last < 3 ? last : 3];
            parent[0] = e0;
            parent[1] = e1;
            parent[2] = e2;
            parent[3] = e3;
            prow = parent;
            // query codes after each entry's column (the query has readable slack at its end)
            nxt4 = (uint32_t)a.query[e0.col + 1] | ((uint32_t)a.query[e1.col + 1] << 8) |
                   ((uint32_t)a.query[e2.col + 1] << 16) | ((uint32_t)a.query[e3.col + 1] << 24);
        }
        if (a.sigma == 4) {
            uint32_t o_lo[4] = {0, 0, 0, 0}, o_hi[4] = {0, 0, 0, 0};
            occ4_dna(a, (int64_t)nd.lo - 1, o_lo);
            occ4_dna(a, (int64_t)nd.hi, o_hi);
            const int64_t b0 = nd.lo == 0 ? -1 : ((int64_t)nd.lo - 1) / kDnaBlockChars;
            const int64_t b1 = (int64_t)nd.hi / kDnaBlockChars;
            st[3] += (b0 >= 0 && b0 != b1) ? 2u : 1u;
            staged = true;
            uint32_t used = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t l = (int64_t)a.C[c] + o_lo[c];
                const int64_t r = (int64_t)a.C[c] + o_hi[c] - 1;
                ch_lo[c] = (uint32_t)l;
                ch_hi[c] = (uint32_t)r;
                if (!staged || l > r) continue;
                RowSink s;
                sink_init(s);
                s.lo = (uint32_t)l;
                s.hi = (uint32_t)r;
                s.out = stage + used;
                s.cap = (uint32_t)kStage - used;
                s.hit_cap = 0;  // count hits now, write them after the allocation
                const bool multi = l < r;
                if (!multi) s.emit_hits = false;
                child_row<true>(a, prow, nd.len, c, d1, false, 0, s, nullptr, nxt4);
                if (s.n_entries > s.cap) {
                    staged = false;
                    continue;
                }
                st[0] += s.st_diag;
                st[1] += s.st_gap2;
                st[2] += s.st_gap3;
                ch_n[c] = s.n_entries;
                used += s.n_entries;
                n.hits += s.n_hits;
                if (s.n_entries == 0) continue;
                if (multi) {
                    if (s.n_entries > kLaneRow)
                        n.wide++;
                    else
                        n.nodes++;
                    n.entries += s.n_entries;
                } else {
                    n.chains++;
                    n.centries += s.n_entries;
                }
            }
        }
        if (!staged) {  // the stage overflowed, or a protein alphabet: two passes
            n = LevelCounts{0, 0, 0, 0, 0, 0};
            st[0] = st[1] = st[2] = 0;
            uint32_t dummy[5] = {0, 0, 0, 0, 0};
            expand_node<false>(a, nd, prow, d1, n, o, caps, a.sigma == 4 ? dummy : st);
            use_prow = prow;
        }
    }
    // allocate this wave's output with one atomic per buffer (per-wave counts fit 32 bits)
    uint32_t u_nodes, u_wide, u_ent, u_ch, u_ce, u_hits;
    const unsigned long long p_nodes = wave_excl_scan_u32(n.nodes, &u_nodes);
    const unsigned long long p_wide = wave_excl_scan_u32(n.wide, &u_wide);
    const unsigned long long p_ent = wave_excl_scan_u32(n.entries, &u_ent);
    const unsigned long long p_ch = wave_excl_scan_u32(n.chains, &u_ch);
    const unsigned long long p_ce = wave_excl_scan_u32(n.centries, &u_ce);
    const unsigned long long p_hits = wave_excl_scan_u32(n.hits, &u_hits);
    const unsigned long long t_nodes = u_nodes, t_wide = u_wide, t_ent = u_ent, t_ch = u_ch, t_ce = u_ce,
                             t_hits = u_hits;
    const int lane = threadIdx.x & 63;
    unsigned long long b_nodes = 0, b_wide = 0, b_ent = 0, b_ch = 0, b_ce = 0, b_hits = 0;
    if (lane == 0) {
        if (t_nodes) b_nodes = atomicAdd(&cnt->nodes, t_nodes);
        if (t_wide) b_wide = atomicAdd(&cnt->lwnodes, t_wide);
        if (t_ent) b_ent = atomicAdd(&cnt->entries, t_ent);
        if (t_ch) b_ch = atomicAdd(&cnt->cnodes, t_ch);
        if (t_ce) b_ce = atomicAdd(&cnt->centries, t_ce);
        if (t_hits) b_hits = atomicAdd(&cnt->hits, t_hits);
        unsigned long long of = 0;
        if (b_nodes + t_nodes > caps.nodes) of |= kOvNodes;
        if (b_wide + t_wide > caps.lwnodes) of |= kOvLevelWide;
        if (b_ent + t_ent > caps.entries) of |= kOvEntries;
        if (b_ch + t_ch > caps.cnodes) of |= kOvChainNodes;
        if (b_ce + t_ce > caps.centries) of |= kOvChainEntries;
        if (b_hits + t_hits > caps.hits) of |= kOvHits;
        if (of) atomicOr(&cnt->overflow, of);
    }
    b_nodes = bcast0_u64(b_nodes);
    b_wide = bcast0_u64(b_wide);
    b_ent = bcast0_u64(b_ent);
    b_ch = bcast0_u64(b_ch);
    b_ce = bcast0_u64(b_ce);
    b_hits = bcast0_u64(b_hits);
    const bool fits = b_nodes + t_nodes <= caps.nodes && b_wide + t_wide <= caps.lwnodes &&
                      b_ent + t_ent <= caps.entries && b_ch + t_ch <= caps.cnodes && b_ce + t_ce <= caps.centries;
    if (active && fits) {
        LevelOut w = o;
        w.node_base = b_nodes + p_nodes;
        w.wide_base = b_wide + p_wide;
        w.ent_base = b_ent + p_ent;
        w.chain_base = b_ch + p_ch;
        w.cent_base = b_ce + p_ce;
        w.hit_base = b_hits + p_hits;
        if (staged) {
            uint32_t used = 0, k_nodes = 0, k_wide = 0, k_ent = 0, k_ch = 0, k_ce = 0;
            unsigned long long hslot = w.hit_base;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t len = ch_n[c];
                if (len == 0) continue;
                const Entry *src = stage + used;
                used += len;
                const bool multi = ch_lo[c] < ch_hi[c];
                Node cn;
                Entry *dst;
                if (multi) {
                    cn.lo = ch_lo[c];
                    cn.hi = ch_hi[c];
                    cn.off = (uint32_t)(w.ent_base + k_ent);
                    dst = o.oent + w.ent_base + k_ent;
                    k_ent += len;
                    if (len > kLaneRow)
                        o.owide[w.wide_base + k_wide++] = Node{cn.lo, cn.hi, cn.off, len};
                    else
                        o.onodes[w.node_base + k_nodes++] = Node{cn.lo, cn.hi, cn.off, len};
                } else {
                    cn.lo = ch_lo[c];
                    cn.hi = (uint32_t)d1;
                    cn.off = (uint32_t)(w.cent_base + k_ce);
                    dst = o.cent + w.cent_base + k_ce;
                    k_ce += len;
                    o.chains[w.chain_base + k_ch++] = Node{cn.lo, cn.hi, cn.off, len};
                }
                for (uint32_t k = 0; k < len; ++k) {
                    const Entry e = src[k];
                    dst[k] = e;
                    if (multi && e.M >= a.H) {  // hits at every occurrence (chains emit their own)
                        for (uint32_t h = ch_lo[c]; h <= ch_hi[c]; ++h, ++hslot) {
                            if (hslot < caps.hits) {
                                o.hkeys[hslot] = ((uint64_t)e.col << 32) | a.sa[h];
                                o.hscores[hslot] = (uint32_t)e.M;
                            }
                        }
                    }
                }
            }
        } else {
            LevelCounts n2;
            expand_node<true>(a, nd, use_prow, d1, n2, w, caps, st);
        }
    }
    const unsigned long long s_nodes = wave_sum_u32(active ? 1u : 0u);
    const unsigned long long s_ent = wave_sum_u32(n.entries + n.centries);
    const unsigned long long s_diag = wave_sum_u32(st[0]);
    const unsigned long long s_g2 = wave_sum_u32(st[1]);
    const unsigned long long s_g3 = wave_sum_u32(st[2]);
    const unsigned long long s_occ = wave_sum_u32(st[3]);
    const unsigned long long s_in =
        wave_sum_u32(active ? (uint32_t)(sizeof(Node) + nd.len * sizeof(Entry)) : 0u);
    if (lane == 0) {
        if (s_nodes) atomicAdd(&cnt->st_nodes, s_nodes);
        if (s_ent) atomicAdd(&cnt->st_entries, s_ent);
        if (s_diag) atomicAdd(&cnt->st_diag, s_diag);
        if (s_g2) atomicAdd(&cnt->st_gap2, s_g2);
        if (s_g3) atomicAdd(&cnt->st_gap3, s_g3);
        if (s_occ) atomicAdd(&cnt->st_occ_reads, s_occ);
        atomicAdd(&cnt->st_frontier_bytes, s_in + (t_nodes + t_wide + t_ch) * sizeof(Node) +
                                               (t_ent + t_ce) * sizeof(Entry) + t_hits * 12ull);
        if (t_hits) atomicAdd(&cnt->st_emitted, t_hits);
    }
}

// Hits of a staged row for every occurrence [lo, hi] (wave-parallel).
__device__ inline void emit_row_hits_multi(const SearchArgs &a, const Entry *row, uint32_t len, uint32_t lo,
                                           uint32_t hi, uint64_t *hkeys, uint32_t *hscores, Caps caps,
                                           Counters *cnt, HitRes &hr, unsigned long long &emitted) {
    const int lane = threadIdx.x & 63;
    const uint32_t occ = hi - lo + 1;
    for (uint32_t base = 0; base < len; base += 64) {
        const uint32_t k = base + lane;
        const Entry e = k < len ? row[k] : Entry{0, kNeg, kNeg, 0, 0};
        const uint32_t nh = (k < len && e.M >= a.H) ? occ : 0u;
        uint32_t tot;
        const uint32_t pre = wave_excl_scan_u32(nh, &tot);
        if (!tot) continue;
        hit_reserve(hr, tot, hkeys, hscores, caps.hits, cnt);
        unsigned long long slot = hr.base + pre;
        for (uint32_t h = 0; h < nh; ++h, ++slot) {
            if (slot < caps.hits) {
                hkeys[slot] = ((uint64_t)e.col << 32) | a.sa[lo + h];
                hscores[slot] = (uint32_t)e.M;
            }
        }
        hr.base += tot;
        hr.left -= tot;
        emitted += tot;
    }
}

// One wave per node with a long row.  stage holds caps.srow entries per block;
// a longer child row raises kOvStageRow with its length in stage_need.
__global__ void __launch_bounds__(64) k_expand_level_wide(SearchArgs a, const Node *wnodes, uint32_t nw,
                                                          const Entry *ent, int32_t d1, LevelOut o, Caps caps,
                                                          Counters *cnt, Entry *stage) {
    const int lane = threadIdx.x & 63;
    Entry *buf = stage + (uint64_t)blockIdx.x * caps.srow;
    HitRes hr = {0, 0, 0};
    unsigned long long emitted = 0, entries = 0, diag = 0, gap2 = 0, gap3 = 0;
    for (uint32_t item = blockIdx.x; item < nw; item += gridDim.x) {
        const Node nd = wnodes[item];
        uint32_t o1[4] = {0, 0, 0, 0}, o2[4] = {0, 0, 0, 0};
        if (a.sigma == 4) {
            occ4_dna(a, (int64_t)nd.lo - 1, o1);
            occ4_dna(a, (int64_t)nd.hi, o2);
        }
        for (int c = 0; c < a.sigma; ++c) {
            int64_t l, r;
            if (a.sigma == 4) {
                l = (int64_t)a.C[c] + o1[c];
                r = (int64_t)a.C[c] + o2[c] - 1;
            } else {
                l = (int64_t)a.C[c] + occ1_gen(a, c, (int64_t)nd.lo - 1);
                r = (int64_t)a.C[c] + occ1_gen(a, c, (int64_t)nd.hi) - 1;
            }
            if (l > r) continue;
            WideOut w;
            w.cap = (uint32_t)caps.srow;
            w.hkeys = o.hkeys;
            w.hscores = o.hscores;
            w.hit_cap = caps.hits;
            w.cnt = cnt;
            w.e_child = 0;
            w.emit_hits = false;
            w.rK = 0;
            w.rdelta = nullptr;
            wide_child_row(a, AosRow{const_cast<Entry *>(ent) + nd.off}, nd.len, AosRow{buf}, c, d1, w, hr);
            __syncthreads();
            if (w.overflow) {
                if (lane == 0) {
                    atomicOr(&cnt->overflow, kOvStageRow);
                    atomicMax(&cnt->stage_need, (unsigned long long)w.len);
                }
                continue;
            }
            const uint32_t len = w.len;
            entries += len;
            diag += w.diag;
            gap2 += w.gap2;
            gap3 += w.gap3;
            if (len == 0) continue;
            const bool multi = l < r;
            if (multi)
                emit_row_hits_multi(a, buf, len, (uint32_t)l, (uint32_t)r, o.hkeys, o.hscores, caps, cnt, hr,
                                    emitted);
            unsigned long long slot = 0, off = 0;
            if (lane == 0) {
                if (multi) {
                    const bool wide = len > kLaneRow;
                    slot = atomicAdd(wide ? &cnt->lwnodes : &cnt->nodes, 1ull);
                    off = atomicAdd(&cnt->entries, (unsigned long long)len);
                    if (slot >= (wide ? caps.lwnodes : caps.nodes))
                        atomicOr(&cnt->overflow, wide ? kOvLevelWide : kOvNodes);
                    if (off + len > caps.entries) atomicOr(&cnt->overflow, kOvEntries);
                } else {
                    slot = atomicAdd(&cnt->cnodes, 1ull);
                    off = atomicAdd(&cnt->centries, (unsigned long long)len);
                    if (slot >= caps.cnodes) atomicOr(&cnt->overflow, kOvChainNodes);
                    if (off + len > caps.centries) atomicOr(&cnt->overflow, kOvChainEntries);
                }
            }
            slot = __shfl(slot, 0, 64);
            off = __shfl(off, 0, 64);
            Entry *dst = multi ? o.oent : o.cent;
            const bool wide = len > kLaneRow;
            const unsigned long long ncap = multi ? (wide ? caps.lwnodes : caps.nodes) : caps.cnodes;
            const unsigned long long ecap = multi ? caps.entries : caps.centries;
            if (slot < ncap && off + len <= ecap) {
                for (uint32_t k = lane; k < len; k += 64) dst[off + k] = buf[k];
                if (lane == 0) {
                    Node cn;
                    cn.lo = (uint32_t)l;
                    cn.hi = multi ? (uint32_t)r : (uint32_t)d1;
                    cn.off = (uint32_t)off;
                    cn.len = len;
                    if (!multi)
                        o.chains[slot] = cn;
                    else if (wide)
                        o.owide[slot] = cn;
                    else
                        o.onodes[slot] = cn;
                }
            }
            __syncthreads();
        }
    }
    hit_release(hr, o.hkeys, o.hscores, caps.hits, cnt);
    diag = wave_sum_u64(diag);  // per-lane partial counts of the row updates
    gap2 = wave_sum_u64(gap2);
    gap3 = wave_sum_u64(gap3);
    if (lane == 0) {
        atomicAdd(&cnt->st_nodes, (unsigned long long)((nw > blockIdx.x) ? (nw - 1 - blockIdx.x) / gridDim.x + 1 : 0));
        atomicAdd(&cnt->st_entries, entries);
        atomicAdd(&cnt->st_diag, diag);
        atomicAdd(&cnt->st_gap2, gap2);
        atomicAdd(&cnt->st_gap3, gap3);
        atomicAdd(&cnt->st_emitted, emitted);
    }
}

}  // namespace alae
