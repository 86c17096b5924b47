// Chains: trie nodes with a single occurrence.
//
// Below a node with one occurrence ending at text position e, the trie is a
// single path: the next character is T[e+1] (no index lookup is needed), and
// every hit of the row is located at e.  Three walkers, by row shape:
//
//   k_chain_start    one lane per chain created by a level: locates it
//                    (suffix array), tests its states for domination
//                    (Section 3.2), and walks it in registers while every
//                    entry is in the no-gap region (M <= |sg+ss|, no G_a):
//                    there the row update is the diagonal step of Eq. 3;
//   k_chain_general  one lane per chain whose row has gap states (first row
//                    up to kNarrowRow entries, later rows up to kPromoteRow,
//                    kept in private memory);
//   k_chain_wide_*   a block of waves (LDS rows) or one wave (global memory,
//                    rows beyond kWideCap entries) per chain with a longer row.
#pragma once

#include "row_update.h"

namespace alae {

constexpr int kNarrowRow = 24;  // row capacity of the lane walker (a chain's first row may fill it)
constexpr int kPromoteRow = 12; // a lane-walker row longer than this goes on to the wave walkers
constexpr int kNgrSlots = 4;
constexpr int kWideCap = 1024;  // row entries a wave walker keeps in LDS
constexpr int kWideWaves = 4;   // waves of a wave-walker block (one chain per block)

// Eight bytes arr[p .. p+7] as one little-endian word (arr carries kSlack
// readable bytes around its data).
__device__ inline uint64_t load8(const uint8_t *arr, int64_t p) {
    const uintptr_t addr = (uintptr_t)(arr + p);
    const uint32_t *b = reinterpret_cast<const uint32_t *>(addr & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(addr & 3u);
    const uint32_t r0 = b[0], r1 = b[1], r2 = b[2];
    const uint32_t w0 = __builtin_amdgcn_alignbyte(r1, r0, sh);
    const uint32_t w1 = __builtin_amdgcn_alignbyte(r2, r1, sh);
    return ((uint64_t)w1 << 32) | w0;
}

__device__ inline int32_t score_of(const SearchArgs &a, const int8_t *sub, uint32_t tc, uint32_t pc) {
    return a.matrix_mode ? (int32_t)sub[tc * (uint32_t)a.sigma + pc] : (tc == pc ? a.s_match : a.s_mismatch);
}

// Gapped domination test of a row's states (the occurrence starts at
// x = e_end - depth + 1): dominated states are set dead in place.  Returns
// the number of entries that keep a live state.
__device__ uint32_t prune_dominated(const SearchArgs &a, Entry *row, uint32_t len, uint32_t e_end, int32_t depth,
                                    unsigned long long &dom_count) {
    const int64_t x = (int64_t)e_end - depth + 1;
    uint32_t memo_y[4] = {kNoPos, kNoPos, kNoPos, kNoPos};
    bool memo_r[4] = {false, false, false, false};
    int memo_n = 0;
    auto test = [&](uint32_t y) {
        for (int q = 0; q < 4; ++q)
            if (memo_y[q] == y) return memo_r[q];
        const bool r = dominated_gapped(a, x, y);
        memo_y[memo_n & 3] = y;
        memo_r[memo_n & 3] = r;
        ++memo_n;
        return r;
    };
    uint32_t live = 0;
    for (uint32_t k = 0; k < len; ++k) {
        Entry e = row[k];
        if (e.M > 0 && test(e.yM)) {
            e.M = kNeg;
            e.yM = 0;
            ++dom_count;
        }
        if (e.Ga > 0 && test(e.yGa)) {
            e.Ga = kNeg;
            e.yGa = 0;
            ++dom_count;
        }
        row[k] = e;
        live += (e.M > 0 || e.Ga > 0) ? 1u : 0u;
    }
    return live;
}

// Append a row with live entries to a chain queue (per-lane atomics).
// Returns a pointer to the queued entries, or nullptr on overflow.
__device__ inline Entry *queue_alloc(Counters *cnt, unsigned long long *nodes_ctr, unsigned long long *ent_ctr,
                                     unsigned long long node_cap, unsigned long long ent_cap,
                                     unsigned long long ov_nodes, unsigned long long ov_ent, Node *qnodes,
                                     Entry *qents, uint32_t len, uint32_t e_end, int32_t depth,
                                     uint32_t *slot_out = nullptr) {
    const unsigned long long slot = atomicAdd(nodes_ctr, 1ull);
    if (slot_out) *slot_out = (uint32_t)slot;
    const unsigned long long off = atomicAdd(ent_ctr, (unsigned long long)len);
    if (slot >= node_cap || off + len > ent_cap) {
        atomicOr(&cnt->overflow, slot >= node_cap ? ov_nodes : ov_ent);
        return nullptr;
    }
    Node nd;
    nd.lo = kUniqueBit | e_end;
    nd.hi = (uint32_t)depth;
    nd.off = (uint32_t)off;
    nd.len = len;
    qnodes[slot] = nd;
    return qents + off;
}

// Queue a row for the wave walkers after the gapped domination test; wsrc
// (nullable) records the lane-queue item src the row continues.
// ready (nullable) publishes the item to a concurrently running wave walker:
// 1 once the row is written, 2 if the slot stays empty (capacity overflow).
__device__ void push_wide(const SearchArgs &a, Entry *row, uint32_t len, uint32_t e_end, int32_t depth,
                          Node *witems, Entry *went, Caps caps, Counters *cnt, unsigned long long &dom_count,
                          uint32_t src = 0, uint32_t *wsrc = nullptr, uint32_t *ready = nullptr) {
    uint32_t keep = len;
    if (a.use_domination) keep = prune_dominated(a, row, len, e_end, depth, dom_count);
    if (keep == 0) return;
    uint32_t slot = 0;
    Entry *dst = queue_alloc(cnt, &cnt->wnodes, &cnt->wentries, caps.wnodes, caps.wentries, kOvWideNodes,
                             kOvWideEntries, witems, went, keep, e_end, depth, &slot);
    if (!dst) {
        if (ready && slot < caps.wnodes) __hip_atomic_store(&ready[slot], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (wsrc) wsrc[slot] = src;
    uint32_t w = 0;
    for (uint32_t k = 0; k < len; ++k) {
        const Entry e = row[k];
        if (e.M <= 0 && e.Ga <= 0) continue;
        dst[w++] = e;
    }
    if (ready) {
        __threadfence();
        __hip_atomic_store(&ready[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        atomicMin(&cnt->t_push0, (unsigned long long)__builtin_amdgcn_s_memrealtime());
    }
}

__device__ inline void emit_hit_lane(Counters *cnt, uint64_t *hkeys, uint32_t *hscores, Caps caps, uint32_t col,
                                     uint32_t e_end, int32_t M) {
    const unsigned long long slot = atomicAdd(&cnt->hits, 1ull);
    if (slot < caps.hits) {
        hkeys[slot] = ((uint64_t)col << 32) | e_end;
        hscores[slot] = (uint32_t)M;
    } else {
        atomicOr(&cnt->overflow, kOvHits);
    }
}

struct ChainQueues {
    Node *gnodes;   // chains with gap states (general lane walker)
    Entry *gents;
    Node *wnodes;   // chains with long rows (wave walkers)
    Entry *wents;
    uint64_t *hkeys;
    uint32_t *hscores;
};

// Hit slots of one lane, reserved eight at a time (lanes walk independently);
// slots left over are padded with kPadKey.
constexpr unsigned long long kLaneHitChunk = 8;
struct LaneHits {
    unsigned long long base, left, pad;
};

__device__ inline void lane_hit_put(LaneHits &h, Counters *cnt, uint64_t *hkeys, uint32_t *hscores, Caps caps,
                                    uint32_t col, uint32_t e_end, int32_t M) {
    if (h.left == 0) {
        h.base = atomicAdd(&cnt->hits, kLaneHitChunk);
        h.left = kLaneHitChunk;
        if (h.base + kLaneHitChunk > caps.hits) atomicOr(&cnt->overflow, kOvHits);
    }
    if (h.base < caps.hits) {
        hkeys[h.base] = ((uint64_t)col << 32) | e_end;
        hscores[h.base] = (uint32_t)M;
    }
    ++h.base;
    --h.left;
}

__device__ inline void lane_hit_release(LaneHits &h, uint64_t *hkeys, uint32_t *hscores, Caps caps) {
    for (; h.left; --h.left, ++h.base, ++h.pad) {
        if (h.base < caps.hits) {
            hkeys[h.base] = kPadKey;
            hscores[h.base] = 0;
        }
    }
}

// Wave-aggregated reservation of `nodes` queue records and `ents` entries per
// lane; returns false (and raises the overflow bits) when the queue is full.
__device__ inline bool wave_queue_alloc(Counters *cnt, unsigned long long *nodes_ctr, unsigned long long *ent_ctr,
                                        unsigned long long node_cap, unsigned long long ent_cap,
                                        unsigned long long ov_nodes, unsigned long long ov_ent, uint32_t nodes,
                                        uint32_t ents, unsigned long long &slot, unsigned long long &off) {
    const int lane = threadIdx.x & 63;
    uint32_t tn, te;
    const uint32_t pn = wave_excl_scan_u32(nodes, &tn);
    const uint32_t pe = wave_excl_scan_u32(ents, &te);
    unsigned long long bn = 0, be = 0;
    if (lane == 0 && tn) {
        bn = atomicAdd(nodes_ctr, (unsigned long long)tn);
        be = atomicAdd(ent_ctr, (unsigned long long)te);
        if (bn + tn > node_cap) atomicOr(&cnt->overflow, ov_nodes);
        if (be + te > ent_cap) atomicOr(&cnt->overflow, ov_ent);
    }
    bn = __shfl(bn, 0, 64);
    be = __shfl(be, 0, 64);
    slot = bn + pn;
    off = be + pe;
    return bn + tn <= node_cap && be + te <= ent_cap;
}

// ---------------------------------------------------------------------------
// k_chain_start: one lane per chain created by a level.  Queue records and
// hit slots are reserved once per block where every lane takes part; the
// no-gap walk reserves its hit slots per lane in small chunks.
// ---------------------------------------------------------------------------
constexpr int kStartBlock = 256;

// Launched right behind the level kernels that make the chains, with a grid
// for the most chains the level can make: the count is read here, and after
// an overflow of the level (its outputs are incomplete and the host runs the
// level and this kernel again) nothing is done.  first_hits: write the hits
// of an item's first row (off for items split off the frontier's tail, whose
// rows' hits the level kernels wrote at every occurrence).
// Four waves per SIMD (128 VGPRs, a few spilled): the random reads of the
// suffix array and the text need the extra waves in flight more than the
// spilled registers cost; a fifth wave spills too much.
__device__ __forceinline__ void chain_start_tile(const SearchArgs &a, const int8_t *sub, const Node *items,
                                                 const Entry *ient, const ChainQueues &q, const Caps &caps,
                                                 Counters *cnt, bool first_hits, uint32_t t, uint32_t nitems,
                                                 BlockReserveLds<5, kStartBlock / 64> &s_res5,
                                                 BlockReserveLds<11, kStartBlock / 64> &s_res11) {
    const int32_t open = a.sg + a.ss;
    unsigned long long n_dom = 0, n_steps = 0, n_entries = 0, n_hits = 0, n_wide = 0;
    // phase 1: locate, test the states (ungapped domination), classify
    enum { kNone = 0, kWide = 1, kGeneral = 2, kNgr = 3 };
    int path = kNone;
    uint32_t e_end = 0, len = 0, killM = 0, killGa = 0, live = 0, nh = 0;
    int32_t depth = 0;
    const Entry *row = nullptr;
    int64_t x = 0;
    if (t < nitems) {
        const Node it = items[t];
        e_end = a.sa[it.lo];
        depth = (int32_t)it.hi;
        len = it.len;
        row = ient + it.off;
        x = (int64_t)e_end - depth + 1;
        bool ngr = true;
        // the text window before x is the same for every state of the row, and neighbouring
        // states often share their start column: the last verdict is kept
        uint32_t tw[8];
        if (a.use_domination) load_window32(a.text, x, tw);
        int64_t last_y = -1;
        bool last_dom = false;
        auto dom_at = [&](int64_t y) {
            if (y != last_y) {
                last_dom = dominated_tw(a, sub, tw, x, y);
                last_y = y;
            }
            return last_dom;
        };
        for (uint32_t k = 0; k < len; ++k) {
            const Entry e = row[k];
            bool aM = e.M > 0, aG = e.Ga > 0;
            if (a.use_domination) {
                if (aM && dom_at(e.yM)) {
                    aM = false;
                    if (k < 32) killM |= 1u << k;
                    ++n_dom;
                }
                if (aG && dom_at(e.yGa)) {
                    aG = false;
                    if (k < 32) killGa |= 1u << k;
                    ++n_dom;
                }
            }
            if (first_hits && aM && e.M >= a.H) ++nh;
            if (aM || aG) ++live;
            if (aG || (aM && e.M > -open)) ngr = false;
        }
        if (len > (uint32_t)kNarrowRow)
            path = kWide;  // long row: both domination tests, then the wave walkers
        else if (live > 0 && (!ngr || live > (uint32_t)kNgrSlots || !a.ngr_walk))
            path = kGeneral;  // gap states (or many entries): the general lane walker
        else if (live > 0)
            path = kNgr;  // no-gap region: walk in registers, diagonal steps only (Eq. 3)
    }
    // domination verdicts of phase 1: bit masks for rows of up to 32 entries,
    // recomputed for longer rows
    auto deadM = [&](uint32_t k, const Entry &e) {
        return len <= 32u ? ((killM >> k) & 1u) != 0 : (a.use_domination && e.M > 0 && dominated(a, sub, x, e.yM));
    };
    auto deadGa = [&](uint32_t k, const Entry &e) {
        return len <= 32u ? ((killGa >> k) & 1u) != 0
                          : (a.use_domination && e.Ga > 0 && dominated(a, sub, x, e.yGa));
    };
    // phase 2: one reservation per block for the first row's hits and the queue records
    {
        const bool pw = path == kWide, pg = path == kGeneral;
        uint32_t t_h, t_wn, t_we, t_gn, t_ge;
        const uint32_t p_h = wave_excl_scan_u32(nh, &t_h);
        const uint32_t p_wn = wave_excl_scan_u32(pw ? 1u : 0u, &t_wn);
        const uint32_t p_we = wave_excl_scan_u32(pw ? len : 0u, &t_we);
        const uint32_t p_gn = wave_excl_scan_u32(pg ? 1u : 0u, &t_gn);
        const uint32_t p_ge = wave_excl_scan_u32(pg ? live : 0u, &t_ge);
        unsigned long long *const ctr[5] = {&cnt->hits, &cnt->wnodes, &cnt->wentries, &cnt->gnodes, &cnt->gentries};
        const unsigned long long wtot[5] = {t_h, t_wn, t_we, t_gn, t_ge};
        const unsigned long long cap[5] = {caps.hits, caps.wnodes, caps.wentries, caps.gnodes, caps.gentries};
        const uint32_t ovb[5] = {kOvHits, kOvWideNodes, kOvWideEntries, kOvGeneralNodes, kOvGeneralEntries};
        unsigned long long b[5];
        block_reserve<5, kStartBlock / 64>(s_res5, ctr, wtot, cap, ovb, &cnt->overflow, b);
        unsigned long long hb = b[0] + p_h;
        if (nh) {
            for (uint32_t k = 0; k < len; ++k) {
                const Entry e = row[k];
                if (e.M <= 0 || e.M < a.H || deadM(k, e)) continue;
                if (hb < caps.hits) {
                    q.hkeys[hb] = ((uint64_t)e.col << 32) | e_end;
                    q.hscores[hb] = (uint32_t)e.M;
                }
                ++hb;
            }
            n_hits += nh;
        }
        if (pw && b[1] + t_wn <= caps.wnodes && b[2] + t_we <= caps.wentries) {
            const unsigned long long slot = b[1] + p_wn, off = b[2] + p_we;
            Entry *dst = q.wents + off;
            for (uint32_t k = 0; k < len; ++k) {
                Entry e = row[k];
                if (deadM(k, e)) e.M = kNeg;
                if (deadGa(k, e)) e.Ga = kNeg;
                dst[k] = e;
            }
            if (a.use_domination) prune_dominated(a, dst, len, e_end, depth, n_dom);
            Node nd;
            nd.lo = kUniqueBit | e_end;
            nd.hi = (uint32_t)depth;
            nd.off = (uint32_t)off;
            nd.len = len;
            q.wnodes[slot] = nd;
            ++n_wide;
        }
        if (pg && b[3] + t_gn <= caps.gnodes && b[4] + t_ge <= caps.gentries) {
            const unsigned long long slot = b[3] + p_gn, off = b[4] + p_ge;
            Entry *dst = q.gents + off;
            uint32_t w = 0;
            for (uint32_t k = 0; k < len; ++k) {
                Entry e = row[k];
                if (deadM(k, e)) e.M = kNeg;
                if (deadGa(k, e)) e.Ga = kNeg;
                if (e.M <= 0 && e.Ga <= 0) continue;
                dst[w++] = e;
            }
            Node nd;
            nd.lo = kUniqueBit | e_end;
            nd.hi = (uint32_t)depth;
            nd.off = (uint32_t)off;
            nd.len = live;
            q.gnodes[slot] = nd;
        }
    }
    // phase 3: the no-gap walk
    uint32_t col[kNgrSlots], y[kNgrSlots], send[kNgrSlots];
    int32_t M[kNgrSlots];
#pragma unroll
    for (int s2 = 0; s2 < kNgrSlots; ++s2) {
        col[s2] = 0;
        y[s2] = 0;
        send[s2] = 0;
        M[s2] = kNeg;
    }
    uint32_t alive = 0;
    bool handoff = false;
    LaneHits lh = {0, 0, 0};
    if (path == kNgr) {
        {
            int sidx = 0;
            for (uint32_t k = 0; k < len; ++k) {
                const Entry e = row[k];
                if (e.M <= 0 || deadM(k, e)) continue;
#pragma unroll
                for (int s2 = 0; s2 < kNgrSlots; ++s2) {
                    if (s2 == sidx) {
                        col[s2] = e.col;
                        M[s2] = e.M;
                        y[s2] = e.yM;
                        send[s2] = seg_end_of(a, e.col);
                    }
                }
                alive |= 1u << sidx;
                ++sidx;
            }
        }
        uint64_t tw = 0, qw[kNgrSlots];
        int tpos = 8;
        for (;;) {
            const int32_t d1 = depth + 1;
            if (d1 > a.lmax || (uint64_t)e_end + 1 >= a.n) break;
            if (tpos == 8) {
                tw = load8(a.text, (int64_t)e_end + 1);
#pragma unroll
                for (int s2 = 0; s2 < kNgrSlots; ++s2)
                    qw[s2] = (alive & (1u << s2)) ? load8(a.query, (int64_t)col[s2] + 1) : 0ull;
                tpos = 0;
            }
            const uint32_t c = (uint32_t)(tw >> (8 * tpos)) & 0xFFu;
            if (c >= (uint32_t)a.sigma) break;  // a record separator: the record ends here
            const int32_t rowgain = a.smax * (a.lmax - d1);
            uint32_t nalive = 0;
            bool fgoe = false;
            int32_t nM[kNgrSlots];
#pragma unroll
            for (int s2 = 0; s2 < kNgrSlots; ++s2) {
                const uint32_t ncol = col[s2] + 1;
                const uint32_t pc = (uint32_t)(qw[s2] >> (8 * tpos)) & 0xFFu;
                const int32_t v = M[s2] + score_of(a, sub, c, pc);
                const bool ok = ((alive >> s2) & 1u) && ncol < send[s2] && keep_state_e(a, v, ncol, send[s2], rowgain);
                nM[s2] = ok ? v : kNeg;
                nalive |= ok ? (1u << s2) : 0u;
                fgoe |= ok && v > -open;
            }
            if (fgoe) {  // a gap can open below this row: the general walker takes the current row
                handoff = true;
                break;
            }
            ++n_steps;
            if (!nalive) break;
#pragma unroll
            for (int s2 = 0; s2 < kNgrSlots; ++s2) {
                if (nalive & (1u << s2)) {
                    col[s2] += 1;
                    M[s2] = nM[s2];
                    ++n_entries;
                    if (M[s2] >= a.H) {
                        lane_hit_put(lh, cnt, q.hkeys, q.hscores, caps, col[s2], e_end + 1, M[s2]);
                        ++n_hits;
                    }
                }
            }
            alive = nalive;
            e_end += 1;
            depth = d1;
            ++tpos;
        }
        lane_hit_release(lh, q.hkeys, q.hscores, caps);
    }
    // phase 4: hand-offs to the general walker and the statistics, one reservation per block
    {
        const uint32_t cntlive = handoff ? (uint32_t)__popc(alive) : 0u;
        uint32_t t_n, t_e;
        const uint32_t p_n = wave_excl_scan_u32(handoff ? 1u : 0u, &t_n);
        const uint32_t p_e = wave_excl_scan_u32(cntlive, &t_e);
        const unsigned long long w_dom = wave_sum_u64(n_dom), w_steps = wave_sum_u64(n_steps),
                                 w_ent = wave_sum_u64(n_entries), w_hits = wave_sum_u64(n_hits),
                                 w_wide = wave_sum_u64(n_wide), w_pad = wave_sum_u64(lh.pad),
                                 w_items = wave_sum_u64(t < nitems ? 1ull : 0ull);
        unsigned long long *const ctr[11] = {&cnt->gnodes,       &cnt->gentries,   &cnt->st_dominated,
                                             &cnt->st_ngr_steps, &cnt->st_entries, &cnt->st_diag,
                                             &cnt->st_emitted,   &cnt->st_promoted, &cnt->hit_padding,
                                             &cnt->st_sa_reads,  &cnt->st_text_reads};
        const unsigned long long wtot[11] = {t_n,    t_e,    w_dom, w_steps, w_ent, w_ent,
                                             w_hits, w_wide, w_pad, w_items, w_items + w_steps / 8};
        const unsigned long long cap[11] = {caps.gnodes, caps.gentries, ~0ull, ~0ull, ~0ull, ~0ull,
                                            ~0ull,       ~0ull,         ~0ull, ~0ull, ~0ull};
        const uint32_t ovb[11] = {kOvGeneralNodes, kOvGeneralEntries, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        unsigned long long b[11];
        block_reserve<11, kStartBlock / 64, 2>(s_res11, ctr, wtot, cap, ovb, &cnt->overflow, b);
        if (handoff && b[0] + t_n <= caps.gnodes && b[1] + t_e <= caps.gentries) {
            const unsigned long long slot = b[0] + p_n, off = b[1] + p_e;
            Entry *dst = q.gents + off;
            uint32_t w = 0;
#pragma unroll
            for (int s2 = 0; s2 < kNgrSlots; ++s2) {
                if (alive & (1u << s2)) {
                    Entry e;
                    e.col = col[s2];
                    e.M = M[s2];
                    e.Ga = kNeg;
                    e.yM = y[s2];
                    e.yGa = 0;
                    dst[w++] = e;
                }
            }
            Node nd;
            nd.lo = kUniqueBit | e_end;
            nd.hi = (uint32_t)depth;
            nd.off = (uint32_t)off;
            nd.len = cntlive;
            q.gnodes[slot] = nd;
        }
    }
}

// The kernel: one tile per block (STRIDE false), or, for device-driven levels
// (STRIDE true, ctl), a grid of a few blocks per CU striding over the chains.
template <bool STRIDE>
__global__ void __launch_bounds__(kStartBlock, 4) k_chain_start(SearchArgs a, SubTable subt, const Node *items,
                                                             const Entry *ient, ChainQueues q, Caps caps,
                                                             Counters *cnt, bool first_hits,
                                                             const LevelCtl *ctl) {
    __shared__ int8_t sub[20 * 20];
    __shared__ BlockReserveLds<5, kStartBlock / 64> s_res5;
    __shared__ BlockReserveLds<11, kStartBlock / 64> s_res11;
    if (cnt->overflow) return;  // the whole grid: the level is run again
    if (STRIDE && ctl->stop) return;  // device-driven levels: no level was begun in this slot
    const uint64_t made = cnt->cnodes;
    const uint32_t nitems = (uint32_t)(made < caps.cnodes ? made : caps.cnodes);
    if ((uint64_t)blockIdx.x * kStartBlock >= nitems) return;  // the whole block
    for (int i = threadIdx.x; i < a.sigma * a.sigma; i += blockDim.x) sub[i] = subt.s[i];
    __syncthreads();
    if (STRIDE) {
        for (uint64_t b0 = (uint64_t)blockIdx.x * kStartBlock; b0 < nitems; b0 += (uint64_t)gridDim.x * kStartBlock)
            chain_start_tile(a, sub, items, ient, q, caps, cnt, first_hits, (uint32_t)b0 + threadIdx.x, nitems,
                             s_res5, s_res11);
    } else {
        chain_start_tile(a, sub, items, ient, q, caps, cnt, first_hits, blockIdx.x * kStartBlock + threadIdx.x,
                         nitems, s_res5, s_res11);
    }
}

// ---------------------------------------------------------------------------
// k_chain_general: one lane per chain with gap states; idle lanes take the
// next queue items.  A row wider than kPromoteRow goes to the wave walkers:
// the lane walks a row one entry at a time, a wave-walker block 256 at once.
// ---------------------------------------------------------------------------
// order (nullable) gives the sequence in which queue items are taken;
// trace_work (nullable) receives each item's work (entries computed + rows).
__global__ void __launch_bounds__(256) k_chain_general(SearchArgs a, const Node *items, uint32_t nitems,
                                                       const Entry *ient, Node *witems, Entry *went,
                                                       uint64_t *hkeys, uint32_t *hscores, Caps caps,
                                                       Counters *cnt, const uint32_t *order, float *trace_work,
                                                       uint32_t *wsrc, uint32_t *ready) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
        atomicMin(&cnt->t_gen0, (unsigned long long)__builtin_amdgcn_s_memrealtime());
        // counted before this wave's first claim: a wave walker that has seen every item
        // claimed and as many finished waves as started ones knows that no push is left
        __hip_atomic_fetch_add(&cnt->gen_started, 1ull, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
    }
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    HitRes hr = {0, 0, 0};
    Entry rows[2][kNarrowRow];
    int cur = 0;
    bool active = false;
    uint32_t my_item = 0;
    float my_work = 0.f;
    uint32_t e_end = 0, len = 0;
    int32_t depth = 0;
    bool exhausted = false;
    unsigned long long n_steps = 0, n_entries = 0, n_dom = 0, n_diag = 0, n_g2 = 0, n_g3 = 0, n_bytes = 0,
                       n_hits = 0, n_prom = 0;
    for (;;) {
        const uint64_t idle = __ballot(!active);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (!exhausted && (nidle >= 16 || nidle == 64)) {
            unsigned long long first = 0;
            if (lane == 0) first = atomicAdd(&cnt->general_head, (unsigned long long)nidle);
            first = __shfl(first, 0, 64);
            if (first + nidle >= nitems) exhausted = true;
            if (!active) {
                const unsigned long long it = first + (unsigned long long)__popcll(idle & below);
                if (it < nitems) {
                    my_item = order ? order[it] : (uint32_t)it;
                    my_work = 0.f;
                    const Node nd = items[my_item];
                    e_end = nd.lo & ~kUniqueBit;
                    depth = (int32_t)nd.hi;
                    len = nd.len;
                    n_bytes += sizeof(Node) + (unsigned long long)len * sizeof(Entry);
                    for (uint32_t k = 0; k < len; ++k) rows[0][k] = ient[nd.off + k];
                    cur = 0;
                    active = true;
                }
            }
        }
        if (__ballot(active) == 0ull) {
            if (exhausted) break;
            continue;
        }
        bool stepped = false;
        uint32_t nlen = 0;
        if (active) {
            const int32_t d1 = depth + 1;
            // the chain ends at the text's end and at a record separator
            if (d1 > a.lmax || (uint64_t)e_end + 1 >= a.n || a.text[e_end + 1] >= (uint32_t)a.sigma) {
                active = false;
            } else {
                my_work += 1.f;
                const int c = a.text[e_end + 1];
                RowSink s;
                sink_init(s);
                s.out = rows[cur ^ 1];
                s.cap = kNarrowRow;
                s.emit_hits = false;
                s.unique = true;
                s.e_end = e_end + 1;
                child_row<true>(a, rows[cur], len, c, d1, false, 0, s);
                ++n_steps;
                my_work += (float)s.n_entries;
                if (s.n_entries > (uint32_t)kPromoteRow) {
                    push_wide(a, rows[cur], len, e_end, depth, witems, went, caps, cnt, n_dom, my_item, wsrc, ready);
                    ++n_prom;
                    active = false;
                } else if (s.n_entries == 0) {
                    active = false;
                } else {
                    nlen = s.n_entries;
                    stepped = true;
                    n_entries += nlen;
                    n_diag += s.st_diag;
                    n_g2 += s.st_gap2;
                    n_g3 += s.st_gap3;
                }
            }
        }
        if (trace_work && !active && my_work > 0.f) {
            trace_work[my_item] = my_work;
            my_work = 0.f;
        }
        // hit records of the new rows (slots reserved by the wave in chunks)
        uint32_t nh = 0;
        if (stepped)
            for (uint32_t k = 0; k < nlen; ++k) nh += rows[cur ^ 1][k].M >= a.H ? 1u : 0u;
        uint32_t htot;
        const uint32_t hpre = wave_excl_scan_u32(nh, &htot);
        if (htot) {
            hit_reserve(hr, htot, hkeys, hscores, caps.hits, caps.hit_chunk, cnt);
            const unsigned long long hb = hr.base;
            hr.base += htot;
            hr.left -= htot;
            if (nh) {
                unsigned long long slot = hb + hpre;
                for (uint32_t k = 0; k < nlen; ++k) {
                    const Entry &w = rows[cur ^ 1][k];
                    if (w.M < a.H) continue;
                    if (slot < caps.hits) {
                        hkeys[slot] = ((uint64_t)w.col << 32) | (e_end + 1);
                        hscores[slot] = (uint32_t)w.M;
                    }
                    ++slot;
                }
            }
            n_hits += nh;
        }
        if (stepped) {
            cur ^= 1;
            len = nlen;
            e_end += 1;
            depth += 1;
        }
    }
    hit_release(hr, hkeys, hscores, caps.hits, cnt);
    const unsigned long long w_steps = wave_sum_u64(n_steps), w_ent = wave_sum_u64(n_entries),
                             w_dom = wave_sum_u64(n_dom), w_d = wave_sum_u64(n_diag), w_2 = wave_sum_u64(n_g2),
                             w_3 = wave_sum_u64(n_g3), w_b = wave_sum_u64(n_bytes), w_h = wave_sum_u64(n_hits),
                             w_p = wave_sum_u64(n_prom);
    if (lane == 0) {
        atomicAdd(&cnt->st_chain_steps, w_steps);
        atomicAdd(&cnt->st_entries, w_ent);
        atomicAdd(&cnt->st_dominated_gapped, w_dom);
        atomicAdd(&cnt->st_diag, w_d);
        atomicAdd(&cnt->st_gap2, w_2);
        atomicAdd(&cnt->st_gap3, w_3);
        atomicAdd(&cnt->st_chain_bytes, w_b);
        atomicAdd(&cnt->st_emitted, w_h);
        atomicAdd(&cnt->st_promoted, w_p);
        // this wave pushes nothing more: tell a live wave walker
        __threadfence();
        atomicAdd(&cnt->gen_done, 1ull);
        atomicMax(&cnt->t_gen1, (unsigned long long)__builtin_amdgcn_s_memrealtime());
    }
}

// ---------------------------------------------------------------------------
// Wave walkers
// ---------------------------------------------------------------------------

struct WideStats {
    unsigned long long steps, entries, diag, gap2, gap3, hits, bytes, reused, replay;
};

// ---------------------------------------------------------------------------
// Reuse of duplicate forks (Section 4.1, Lemmas 2 and 3)
// ---------------------------------------------------------------------------
// A chain row may consist of K+1 copies of one fork: entries k*L+i equal
// entry i with every column moved by delta_k (delta_0 = 0).  Scores in the
// copies stay equal while (a) each copy only touches columns whose query
// characters equal those under the first copy (the common prefix of the query
// suffixes at the copies' first columns) and (b) no copy reaches the next one
// (columns only influence columns to their right).  While that holds the
// walker computes the first copy alone and emits every hit once per copy;
// when the next row could break it, the copies are written out and the row is
// walked in full from there on.  The first copy is filtered with its own gain
// bound U(j) of Theorem 2, which is at least that of every later copy (U does
// not increase with j): a later copy then keeps a superset of the states its
// own bound would keep, each with a score some alignment reaches, so after the
// max-merge its hits are unchanged.
struct Replay {
    uint32_t K;         // copies besides the first (0: none)
    uint32_t col0;      // first column of the first copy
    uint32_t span_lim;  // a row may reach columns col0 .. col0 + span_lim - 1
    uint32_t dK;        // offset of the last copy
};

__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(v, d, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline int32_t wave_max_i32(int32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int32_t o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Recognise a row made of copies of its first fork; deltas[0..K] go to LDS.
template <class Row>
__device__ void replay_detect(const SearchArgs &a, const Row &cur, uint32_t len, Replay &rp, uint32_t *deltas) {
    const int lane = threadIdx.x & 63;
    rp.K = 0;
    if (len < 2) return;
    const Entry e0 = cur.load(0);
    // candidate copy length L: a column hole before entry L, the same state as
    // entry 0, and len a multiple of L with at most 63 further copies
    uint32_t L = 0;
    for (uint32_t base = 1; base < len && L == 0; base += 64) {
        const uint32_t k = base + lane;
        bool cand = false;
        if (k < len && 2 * k <= len && len % k == 0 && len / k <= 64) {
            const Entry ek = cur.load(k), ep = cur.load(k - 1);
            cand = ek.col > ep.col + 1 && ek.M == e0.M && ek.Ga == e0.Ga;
        }
        const unsigned long long b = __ballot(cand);
        if (b) L = base + (uint32_t)__ffsll((long long)b) - 1;
    }
    if (L == 0) return;
    const uint32_t K = len / L - 1;
    for (uint32_t base = L; base < len; base += 64) {
        const uint32_t k = base + lane;
        bool bad = false;
        if (k < len) {
            const uint32_t c = k / L, i = k - c * L;
            const Entry ek = cur.load(k), ei = cur.load(i), eh = cur.load(c * L);
            bad = (ek.col - eh.col) != (ei.col - e0.col) || ek.M != ei.M || ek.Ga != ei.Ga;
            if (i == 0) bad = bad || ek.col <= cur.load(k - 1).col + 1;
        }
        if (__ballot(bad)) return;
    }
    if ((uint32_t)lane <= K) deltas[lane] = cur.load((uint32_t)lane * L).col - e0.col;
    __syncthreads();
    uint32_t gap = 0xFFFFFFFFu;  // lane k < K: distance from copy k to copy k+1
    if ((uint32_t)lane < K) gap = deltas[lane + 1] - deltas[lane];
    const uint32_t mingap = wave_min_u32(gap);
    uint32_t lcp = 0xFFFFFFFFu;  // lane k < K: common prefix of the query at col0 and at col0 + delta_{k+1}
    if ((uint32_t)lane < K) {
        const uint32_t d = deltas[lane + 1];
        const uint32_t avail = a.m - (e0.col + d);
        const uint32_t lim = mingap < avail ? mingap : avail;
        uint32_t t = 0;
        while (t < lim && a.query[e0.col + t] == a.query[e0.col + d + t]) ++t;
        lcp = t;
    }
    const uint32_t minlcp = wave_min_u32(lcp);
    rp.span_lim = mingap < minlcp ? mingap : minlcp;
    rp.col0 = e0.col;
    rp.dK = deltas[K];
    rp.K = K;
}

// Rightmost column the next row of the first copy can touch: the diagonal
// reaches one column past the last entry, a G_b run continues while its value
// stays positive, and no state of the next row exceeds the largest state of
// this row plus s_max.
template <class Row>
__device__ inline int64_t replay_reach(const SearchArgs &a, const Row &cur, uint32_t len) {
    int32_t v = kNeg;
    for (uint32_t k = (uint32_t)(threadIdx.x & 63); k < len; k += 64) {
        const Entry e = cur.load(k);
        v = imax(v, imax(e.M, e.Ga));
    }
    v = wave_max_i32(v);
    const int64_t num = (int64_t)v + a.smax + a.sg;
    const int64_t ext = num > 0 ? (num - 1) / (-(int64_t)a.ss) : 0;
    return (int64_t)cur.load(len - 1).col + 1 + ext;
}

// Entry k of the row with its copies written out.
template <class Row>
__device__ inline Entry replay_entry(const Row &cur, uint32_t len, const uint32_t *deltas, uint32_t k) {
    const uint32_t c = k / len;
    Entry e = cur.load(k - c * len);
    if (c) {
        const uint32_t d = deltas[c];
        e.col += d;
        if (e.M > 0) e.yM += d;
        if (e.Ga > 0) e.yGa += d;
    }
    return e;
}

template <class Row>
__device__ void replay_materialize(Row &cur, uint32_t len, uint32_t K, const uint32_t *deltas) {
    const int lane = threadIdx.x & 63;
    for (uint32_t k = len + (uint32_t)lane; k < (K + 1) * len; k += 64) cur.store(k, replay_entry(cur, len, deltas, k));
    __syncthreads();
}

// Walk one chain whose row is held in (cur, nxt) buffers of capacity cap.
// Returns false if the row outgrew the buffers; the live row is then in cur
// (len, e_end, depth describe it) and the caller spills it.
// With reuse on, the row may be held as its first copy (rp.K > 0); on a false
// return the caller writes out the copies (replay_entry) when it spills.
// W > 1: the block's W waves update each row together (xg: their LDS
// exchange slots); everything else here is computed alike by every wave.
template <int W = 1, bool FAST = false, class Row>
__device__ bool walk_wide(const SearchArgs &a, Row &cur, Row &nxt, uint32_t &len, uint32_t &e_end, int32_t &depth,
                          uint32_t cap, uint64_t *hkeys, uint32_t *hscores, Caps caps, Counters *cnt, HitRes &hr,
                          WideStats &w, Replay &rp, uint32_t *deltas, RowXchg *xg = nullptr) {
    const int lane = threadIdx.x & 63;
    uint32_t txt = 0;
    int tpos = 64;
    rp.K = 0;
    // look for copies now and every 16 rows (background forks die early in a
    // chain, leaving the copies), until copies have been written out once
    bool look = a.use_reuse != 0;
    uint32_t since = 0;
    for (;;) {
        const int32_t d1 = depth + 1;
        if (d1 > a.lmax || (uint64_t)e_end + 1 >= a.n) return true;
        if (look && rp.K == 0 && (since++ & 15u) == 0) {
            replay_detect(a, cur, len, rp, deltas);
            if (rp.K) {
                len /= rp.K + 1;  // keep the first copy only
                w.replay++;
            }
        }
        if (rp.K) {
            const int64_t R = replay_reach(a, cur, len);
            const bool ok = R - (int64_t)rp.col0 < (int64_t)rp.span_lim && R + (int64_t)rp.dK < (int64_t)a.m;
            if (!ok) {  // the copies could diverge: write them out
                if ((uint64_t)(rp.K + 1) * len > cap) return false;
                replay_materialize(cur, len, rp.K, deltas);
                len *= rp.K + 1;
                rp.K = 0;
                look = false;
            }
        }
        if (tpos == 64) {  // next 64 text characters, one per lane
            const uint64_t p = (uint64_t)e_end + 1 + lane;
            txt = p < a.n ? a.text[p] : 0u;
            tpos = 0;
        }
        const int c = __shfl(txt, tpos, 64);
        ++tpos;
        if (c >= a.sigma) return true;  // a record separator: the record ends here
        WideOut o;
        o.emit_hits = true;
        o.cap = cap;
        o.hkeys = hkeys;
        o.hscores = hscores;
        o.hit_cap = caps.hits;
        o.hit_chunk = caps.hit_chunk;
        o.cnt = cnt;
        o.e_child = e_end + 1;
        o.rK = rp.K;
        o.rdelta = deltas;
        wide_child_row<W, FAST>(a, cur, len, nxt, c, d1, o, hr, xg);
        __syncthreads();
        w.steps++;
        w.bytes += (unsigned long long)(len + o.len) * 12ull;
        if (o.overflow) return false;
        w.entries += o.len;
        w.reused += (unsigned long long)rp.K * o.len;
        w.diag += o.diag;
        w.gap2 += o.gap2;
        w.gap3 += o.gap3;
        w.hits += o.hits;
        if (o.len == 0) return true;
        Row t = cur;
        cur = nxt;
        nxt = t;
        len = o.len;
        e_end += 1;
        depth = d1;
    }
}

// w.diag, w.gap2 and w.gap3 are per-lane partial counts and w.hits is per
// wave; the rest is the same in every wave that walked the rows together, so
// only one of them (uniform = true) adds it.
__device__ inline void wide_stats_flush(Counters *cnt, const WideStats &w, bool uniform = true) {
    const unsigned long long d = wave_sum_u64(w.diag), g2 = wave_sum_u64(w.gap2), g3 = wave_sum_u64(w.gap3);
    if ((threadIdx.x & 63) != 0) return;
    atomicAdd(&cnt->st_diag, d);
    atomicAdd(&cnt->st_gap2, g2);
    atomicAdd(&cnt->st_gap3, g3);
    atomicAdd(&cnt->st_emitted, w.hits);
    if (!uniform) return;
    atomicAdd(&cnt->st_wide_steps, w.steps);
    atomicAdd(&cnt->st_entries, w.entries);
    atomicAdd(&cnt->st_wide_entries, w.entries);
    atomicAdd(&cnt->st_chain_bytes, w.bytes);
    if (w.reused) atomicAdd(&cnt->st_reused, w.reused);
    if (w.replay) atomicAdd(&cnt->st_replay, w.replay);
}

// Rows in LDS; the kWideWaves waves of a block walk one chain together.  A
// row that outgrows kWideCap entries is spilled to the global spill queue and
// continued by k_chain_wide_global.
// A wave-walker pass that runs while the lane walker still pushes items.
struct LiveQueue {
    const uint32_t *ready;  // per slot: 0 pending, 1 written, 2 never written (nullptr: static pass)
    uint32_t nstatic;       // items 0 .. nstatic-1 were queued before the launch
    uint64_t gen_items;     // lane-walker queue items (all claimed + every started wave done: no more pushes)
    uint32_t *missed;       // items claimed but given up (the next pass takes them)
    uint64_t patience;      // ticks of the 100 MHz clock to wait without any progress
};

// Items first .. nw-1 of the queue (wide_head starts at first); order
// (nullable) is a permutation of 0 .. nw-first-1 and trace_work is indexed
// from first.  With a live queue, items are claimed in queue order as they
// are published (order applies to the static part only), and the pass ends
// when the lane walker has finished and every published item is taken; a
// block that sees no progress for `patience` gives its claimed item to the
// next pass and stops, so the pass always ends.
// FAST: see wide_child_row (single query, 31-bit prefix-max keys).
template <bool FAST>
__global__ void __launch_bounds__(64 * kWideWaves) k_chain_wide_lds(SearchArgs a, const Node *witems, uint32_t first,
                                                                    uint32_t nw, const Entry *went, Node *onodes,
                                                                    Entry *oents, uint64_t *hkeys, uint32_t *hscores,
                                                                    Caps caps, Counters *cnt, const uint32_t *order,
                                                                    float *trace_work, LiveQueue live) {
    __shared__ uint32_t s_col[2][kWideCap];
    __shared__ int32_t s_M[2][kWideCap];
    __shared__ int32_t s_Ga[2][kWideCap];
    __shared__ uint32_t s_delta[64];
    __shared__ RowXchg s_xg;
    __shared__ unsigned long long s_bc[2];  // thread 0 -> block: claimed slot and state, spill slot and offset
    const uint32_t tid = threadIdx.x;
    const bool lead = tid == 0;
    const bool wave0 = tid < 64;
    HitRes hr = {0, 0, 0};
    WideStats w = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (live.ready && lead) atomicMin(&cnt->t_live0, (unsigned long long)__builtin_amdgcn_s_memrealtime());
    for (;;) {
        if (lead) {
            const unsigned long long it = atomicAdd(&cnt->wide_head, 1ull);
            int state = 1;  // 1 take, 2 skip, 3 end, 4 give up
            if (live.ready) {
                // wait until slot `it` is published, the lane walker is done, or patience runs out
                unsigned long long seen = ~0ull;
                uint64_t since = __builtin_amdgcn_s_memrealtime();
                for (uint32_t poll = 0;; ++poll) {
                    if (it >= caps.wnodes) {
                        state = 3;
                        break;
                    }
                    // relaxed polls (an acquire load would invalidate the CU's L1 on every poll);
                    // the fence after the loop orders the item's reads
                    const uint32_t r = __hip_atomic_load(&live.ready[it], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (r == 1u) {
                        state = 1;
                        break;
                    }
                    if (r == 2u) {
                        state = 2;
                        break;
                    }
                    if (poll & 7u) {  // the shared counters are read on every eighth poll only
                        __builtin_amdgcn_s_sleep(127);
                        continue;
                    }
                    // producer finished: every item claimed and every started wave done, read in
                    // this order (a claim precedes the read of the head, a claiming wave's start
                    // precedes its claim, a wave's pushes precede its finish); polled with relaxed
                    // loads (sequentially consistent ones would invalidate the CU's caches each
                    // time) and confirmed with sequentially consistent ones
                    auto finished = [&](int order) {
                        const unsigned long long h = __hip_atomic_load(&cnt->general_head, order,
                                                                       __HIP_MEMORY_SCOPE_AGENT);
                        const unsigned long long s0 = __hip_atomic_load(&cnt->gen_started, order,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
                        const unsigned long long d0 = __hip_atomic_load(&cnt->gen_done, order,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
                        return h >= live.gen_items && d0 == s0;
                    };
                    const unsigned long long done =
                        __hip_atomic_load(&cnt->gen_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned long long made =
                        __hip_atomic_load(&cnt->wnodes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // (a lane-walker wave finishes only once every item has been claimed, so
                    // nothing needs checking before the first one has)
                    if ((done > 0 || live.gen_items == 0) && finished(__ATOMIC_RELAXED) &&
                        finished(__ATOMIC_SEQ_CST)) {
                        // every push has been published; a slot past the end stays empty
                        __atomic_thread_fence(__ATOMIC_ACQUIRE);
                        const uint32_t r2 =
                            __hip_atomic_load(&live.ready[it], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        state = r2 == 1u ? 1 : (it >= made ? 3 : 2);
                        break;
                    }
                    const unsigned long long prog = done + (made << 20);
                    const uint64_t now = __builtin_amdgcn_s_memrealtime();
                    if (prog != seen) {
                        seen = prog;
                        since = now;
                    } else if (now - since > live.patience) {
                        state = 4;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(127);
                }
                if (state == 4) {
                    const unsigned long long k = atomicAdd(&cnt->missed, 1ull);
                    live.missed[k] = (uint32_t)it;
                }
                if (state == 1) __threadfence();
            } else if (it >= nw) {
                state = 3;
            }
            s_bc[0] = it;
            s_bc[1] = (unsigned long long)state;
        }
        __syncthreads();
        const unsigned long long it = s_bc[0];
        const int state = (int)s_bc[1];
        __syncthreads();  // s_bc is written again below
        if (state == 2) continue;
        if (state == 3 || state == 4) break;
        uint32_t item;
        if (live.ready) {
            __threadfence();
            item = (it < live.nstatic && order) ? order[it] : (uint32_t)it;
        } else {
            const uint32_t rel = (uint32_t)it - first;
            item = first + (order ? order[rel] : rel);
        }
        const Node nd = witems[item];
        uint32_t e_end = nd.lo & ~kUniqueBit;
        int32_t depth = (int32_t)nd.hi;
        uint32_t len = nd.len;
        const unsigned long long work0 = w.entries + w.steps, steps0 = w.steps;
        const unsigned long long tick0 = __builtin_amdgcn_s_memrealtime();
        SoaRow cur{s_col[0], s_M[0], s_Ga[0]};
        SoaRow nxt{s_col[1], s_M[1], s_Ga[1]};
        bool done = true;
        Replay rp;
        rp.K = 0;
        if (len <= (uint32_t)kWideCap) {
            for (uint32_t k = tid; k < len; k += blockDim.x) cur.store(k, went[nd.off + k]);
            __syncthreads();
            done = walk_wide<kWideWaves, FAST>(a, cur, nxt, len, e_end, depth, (uint32_t)kWideCap, hkeys, hscores, caps,
                                         cnt, hr, w, rp, s_delta, &s_xg);
        } else {
            done = false;
        }
        if (!done) {
            // spill the live row (from LDS, or the queued row if it never fit),
            // with its copies written out
            const uint32_t part = len;
            len *= rp.K + 1;
            if (lead) {
                const unsigned long long slot = atomicAdd(&cnt->onodes, 1ull);
                const unsigned long long off = atomicAdd(&cnt->oentries, (unsigned long long)len);
                if (slot >= caps.onodes) atomicOr(&cnt->overflow, kOvSpillNodes);
                if (off + len > caps.oentries) atomicOr(&cnt->overflow, kOvSpillEntries);
                s_bc[0] = slot;
                s_bc[1] = off;
            }
            __syncthreads();
            const unsigned long long slot = s_bc[0], off = s_bc[1];
            if (slot < caps.onodes && off + len <= caps.oentries) {
                const bool from_lds = nd.len <= (uint32_t)kWideCap;
                for (uint32_t k = tid; k < len; k += blockDim.x)
                    oents[off + k] = from_lds ? replay_entry(cur, part, s_delta, k) : went[nd.off + k];
                if (lead) {
                    Node sn;
                    sn.lo = kUniqueBit | e_end;
                    sn.hi = (uint32_t)depth;
                    sn.off = (uint32_t)off;
                    sn.len = len;
                    onodes[slot] = sn;
                }
            }
        }
        if (trace_work && lead) trace_work[item - first] = (float)(w.entries + w.steps - work0);
        if (lead) {
            const unsigned long long rows = w.steps - steps0;
            atomicMax(&cnt->st_wide_max, rows);
            // duration (10 ns ticks, 26 bits), start after the pass began (µs, 20 bits), rows (18 bits)
            const unsigned long long now = __builtin_amdgcn_s_memrealtime();
            const unsigned long long ticks = now - tick0;
            const unsigned long long p0 = live.ready ? __hip_atomic_load(&cnt->t_live0, __ATOMIC_RELAXED,
                                                                          __HIP_MEMORY_SCOPE_AGENT)
                                                     : tick0;
            const unsigned long long start_us = tick0 > p0 ? (tick0 - p0) / 100 : 0;
            const unsigned long long key = (ticks < (1ull << 26) ? ticks : (1ull << 26) - 1) << 38 |
                                           (start_us < (1ull << 20) ? start_us : (1ull << 20) - 1) << 18 |
                                           (rows < (1ull << 18) ? rows : (1ull << 18) - 1);
            atomicMax(&cnt->st_wide_slow, key);
        }
        __syncthreads();
    }
    hit_release(hr, hkeys, hscores, caps.hits, cnt);
    wide_stats_flush(cnt, w, wave0);
    if (live.ready && lead) atomicMax(&cnt->t_live1, (unsigned long long)__builtin_amdgcn_s_memrealtime());
}

// Features of chain items (the layout documented with alae_mlp).
__global__ void k_item_features(SearchArgs a, const Node *items, uint32_t n, const Entry *ents, float queue,
                                float *feat) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const Node nd = items[t];
    int32_t maxM = 0, maxGa = 0;
    float sumM = 0.f;
    uint32_t lo = 0xFFFFFFFFu, hi = 0, best = 0;
    for (uint32_t k = 0; k < nd.len; ++k) {
        const Entry e = ents[nd.off + k];
        if (e.M > maxM) {
            maxM = e.M;
            best = e.col;
        }
        if (e.M > 0) sumM += (float)e.M;
        maxGa = imax(maxGa, e.Ga);
        lo = e.col < lo ? e.col : lo;
        hi = e.col > hi ? e.col : hi;
    }
    const float lm = (float)a.lmax;
    float *f = feat + (size_t)t * ALAE_MLP_FEATURES;
    f[0] = log2f(1.f + (float)nd.hi) / 8.f;
    f[1] = log2f(1.f + (float)nd.len) / 10.f;
    f[2] = (float)maxM / (float)a.H;
    f[3] = log2f(1.f + sumM) / 20.f;
    f[4] = (float)maxGa / (float)a.H;
    f[5] = nd.len ? log2f(1.f + (float)(hi - lo)) / 16.f : 0.f;
    const float left = nd.len ? (float)(seg_end_of(a, best) - best) / lm : 0.f;
    f[6] = left < 1.f ? left : 1.f;
    f[7] = queue;
    // look-ahead: positive substitution scores between the text the chain will
    // read next and the query after the best entry, over characters 1-32 and
    // 33-96 ahead (match/mismatch scoring: equal bytes, four per word)
    uint32_t near = 0, far = 0;
    if (nd.len) {
        const uint64_t e = (uint64_t)(nd.lo & ~kUniqueBit);
        const uint64_t qend = seg_end_of(a, best);
        const uint64_t avail_t = a.n - 1 - e, avail_q = qend - 1 - best;
        const uint32_t avail = (uint32_t)(avail_t < avail_q ? (avail_t < 96 ? avail_t : 96) : (avail_q < 96 ? avail_q : 96));
        for (uint32_t w0 = 0; w0 < 96; w0 += 32) {
            if (w0 >= avail) break;
            uint32_t cnt32 = 0;
            if (!a.matrix_mode) {
                uint32_t tw[8], qw[8];
                // window32 loads the 32 bytes ending before its position
                load_window32(a.text, (int64_t)(e + 1 + w0 + 32), tw);
                load_window32(a.query, (int64_t)(best + 1 + w0 + 32), qw);
                for (int i = 0; i < 8; ++i) {
                    const uint32_t v = tw[i] ^ qw[i];
                    uint32_t z = (v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
                    z = ~(z | v | 0x7F7F7F7Fu);  // 0x80 in every byte where v is zero
                    const uint32_t valid = avail - w0 >= 32 ? 8u : ((avail - w0) + 3) / 4;
                    uint32_t mask = 0x80808080u;
                    if ((uint32_t)i >= valid) mask = 0;
                    else if ((uint32_t)i == valid - 1 && avail - w0 < 32 && ((avail - w0) & 3))
                        mask = 0x80808080u >> (8 * (4 - ((avail - w0) & 3)));
                    cnt32 += __popc(z & mask);
                }
            } else {
                for (uint32_t k = 1 + w0; k <= w0 + 32 && k <= avail; ++k)
                    {
                    const uint32_t tc = a.text[e + k];  // a separator scores nothing
                    cnt32 += tc < (uint32_t)a.sigma && a.prof[(size_t)tc * a.m + best + k] > 0;
                }
            }
            if (w0 == 0)
                near = cnt32;
            else
                far += cnt32;
        }
    }
    f[8] = (float)near / 32.f;
    f[9] = (float)far / 64.f;
}

// Partition of the lane-walker queue by predicted work: heavy[i] = 1 for
// items predicted at or above the threshold, ent[i] = their entry count.
__global__ void k_partition_flags(const float *pred, const Node *items, uint32_t n, float thresh, uint32_t *heavy,
                                  uint32_t *ent) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n) return;
    const bool h = t < n && pred[t] >= thresh && items[t].len > 0;
    heavy[t] = h ? 1u : 0u;
    ent[t] = h ? items[t].len : 0u;
}

// Move the flagged items to the wave-walker queue (slots wbase + pos, entries
// at ebase + epos), after the gapped domination test every row gets on its
// way to the wave walkers, and leave an empty row in their lane-walker slot.
__global__ void k_partition_move(SearchArgs a, Node *items, Entry *ents, uint32_t n, const uint32_t *heavy,
                                 const uint32_t *pos, const uint32_t *epos, Node *witems, Entry *went, uint32_t wbase,
                                 uint32_t ebase, Counters *cnt) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || !heavy[t]) return;
    Node nd = items[t];
    Entry *row = ents + nd.off;
    unsigned long long dom = 0;
    if (a.use_domination) prune_dominated(a, row, nd.len, nd.lo & ~kUniqueBit, (int32_t)nd.hi, dom);
    if (dom) atomicAdd(&cnt->st_dominated_gapped, dom);
    const uint32_t off = ebase + epos[t];
    uint32_t w = 0;
    for (uint32_t k = 0; k < nd.len; ++k) {
        const Entry e = row[k];
        if (e.M <= 0 && e.Ga <= 0) continue;
        went[off + w++] = e;
    }
    Node wn = nd;
    wn.off = off;
    wn.len = w;  // an empty row ends its walk at once
    witems[wbase + pos[t]] = wn;
    nd.len = 0;
    items[t] = nd;
}

// A trace charges the work of a promoted chain's wave-walker continuation
// (items first .. first+n-1 of the wave queue) to its lane-queue item.
__global__ void k_link_work(const uint32_t *wsrc, uint32_t first, uint32_t n, const float *wwork, float *gwork,
                            uint32_t ng) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t g = wsrc[first + t];
    if (g < ng) atomicAdd(&gwork[g], wwork[t]);
}

// Sort keys that put the largest predicted work first.
__global__ void k_order_keys(const float *pred, uint32_t n, uint64_t *keys, uint32_t *vals) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float p = pred[t];
    p = p > 0.f ? (p < 100.f ? p : 100.f) : 0.f;  // NaN maps to 0
    keys[t] = 0xFFFFFFFFull - (uint64_t)(p * 33554432.f);
    vals[t] = t;
}

// Rows in global memory: two buffers of caps.wrow entries per block.
__global__ void __launch_bounds__(64) k_chain_wide_global(SearchArgs a, const Node *items, uint32_t nitems,
                                                          const Entry *ents, Entry *rowbuf, uint64_t *hkeys,
                                                          uint32_t *hscores, Caps caps, Counters *cnt) {
    const int lane = threadIdx.x & 63;
    Entry *buf0 = rowbuf + (uint64_t)blockIdx.x * 2ull * caps.wrow;
    Entry *buf1 = buf0 + caps.wrow;
    __shared__ uint32_t s_delta[64];
    HitRes hr = {0, 0, 0};
    WideStats w = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(&cnt->overflow_head, 1ull);
        it = __shfl(it, 0, 64);
        if (it >= nitems) break;
        const Node nd = items[it];
        uint32_t e_end = nd.lo & ~kUniqueBit;
        int32_t depth = (int32_t)nd.hi;
        uint32_t len = nd.len;
        if (len > caps.wrow) {
            if (lane == 0) atomicOr(&cnt->overflow, kOvWideRow);
            continue;
        }
        for (uint32_t k = lane; k < len; k += 64) buf0[k] = ents[nd.off + k];
        __syncthreads();
        AosRow cur{buf0}, nxt{buf1};
        Replay rp;
        const unsigned long long steps0 = w.steps;
        if (!walk_wide(a, cur, nxt, len, e_end, depth, (uint32_t)caps.wrow, hkeys, hscores, caps, cnt, hr, w, rp,
                       s_delta)) {
            if (lane == 0) atomicOr(&cnt->overflow, kOvWideRow);
        }
        if (lane == 0) atomicMax(&cnt->st_wide_max, w.steps - steps0);
        __syncthreads();
    }
    hit_release(hr, hkeys, hscores, caps.hits, cnt);
    wide_stats_flush(cnt, w);
}

}  // namespace alae
