// Expansion of trie nodes that still have several occurrences (Section 5,
// search (3)): every child X.c of a node X is one backward-search step on the
// FM-index of the reversed text, and its sparse row is computed from X's row
// (Section 2.2 with the filters of Section 3).
//
//   k_level_tasks        one lane per node whose row has at most kLaneRow
//                        entries (almost all nodes): its non-empty children
//                        as tasks;
//   k_expand_children    one lane per task: the child's row;
//   k_expand_level_wide  one wave per node with a longer row (stretches the
//                        text repeats, e.g. overlapping copies of a query
//                        segment).
//
// Children with several occurrences form the next level; a child with one
// occurrence becomes a chain item (BWT row + depth + row) for the chain
// kernels.  Hits of multi-occurrence children are emitted here for every
// occurrence (Algorithm 1).
#pragma once

#include "row_update.h"

namespace alae {

// Rows up to this length are expanded one lane per child; longer ones by a
// wave per node.  Where the frontier widens, most rows hold a few dozen
// entries: a wave per such node costs its own allocation atomics per child,
// and same-address atomics are served one at a time, while the lane kernel
// reserves once per block.
constexpr uint32_t kLaneRow = 128;

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

// Child rows are computed into a per-lane LDS stage of STAGE entries; the
// wave then allocates its outputs with one atomic per buffer and each lane
// copies its stage out.  A longer child row is counted first and computed
// again straight into its allocated place.
constexpr int kStageDefault = 4;  // the search picks 2, 4 or 8 (alae_search_opts.level_stage)
// words of one lane's stage; one pad word so that lanes start in different banks
constexpr int stage_words(int stage) { return stage * 5 + 1; }
constexpr int kLevelBlock = 256;

// ---------------------------------------------------------------------------
// Two phases per level: the node phase turns every node (one lane each) into
// child tasks (node, c, BWT range) for its non-empty children; the child
// phase computes one child row per lane.  A wave of the child phase then runs
// one row update for 64 children instead of four (mostly empty) child passes
// for 64 nodes.
// ---------------------------------------------------------------------------
struct ChildTask {
    uint32_t lo, hi;  // the child's BWT range
    uint32_t off;     // the parent's row (entries off .. off + len - 1 of the level)
    uint32_t len_c;   // parent row length | appended character << 24
};
static_assert(sizeof(ChildTask) == 16, "child task is 16 bytes");

constexpr int kTaskBlock = 1024;

// The child tasks of nodes t - threadIdx.x .. of one block (t = this lane's node).
__device__ inline void level_tasks_tile(const SearchArgs &a, const Node *nodes, uint32_t nn, uint32_t t,
                                        ChildTask *tasks, const Caps &caps, Counters *cnt,
                                        BlockReserveLds<4, kTaskBlock / 64> &s_res) {
    const bool active = t < nn;
    uint32_t mask = 0, nocc = 0, nin = 0;
    Node nd{0, 0, 0, 0};
    uint32_t o_lo[4] = {0, 0, 0, 0}, o_hi[4] = {0, 0, 0, 0};
    if (active) {
        nd = nodes[t];
        nin = (uint32_t)(sizeof(Node) + nd.len * sizeof(Entry));
        if (a.occ_packed) {
            occ4_dna(a, (int64_t)nd.lo - 1, o_lo);
            occ4_dna(a, (int64_t)nd.hi, o_hi);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (o_hi[c] > o_lo[c]) mask |= 1u << c;
            const int64_t b0 = nd.lo == 0 ? -1 : ((int64_t)nd.lo - 1) / kDnaBlockChars;
            const int64_t b1 = (int64_t)nd.hi / kDnaBlockChars;
            nocc = (b0 >= 0 && b0 != b1) ? 2u : 1u;
        } else {
            for (int c = 0; c < a.sigma; ++c)
                if (occ1_gen(a, c, (int64_t)nd.hi) > occ1_gen(a, c, (int64_t)nd.lo - 1)) mask |= 1u << c;
            const int64_t b0 = nd.lo == 0 ? -1 : ((int64_t)nd.lo - 1) / kGenBlockChars;
            const int64_t b1 = (int64_t)nd.hi / kGenBlockChars;
            nocc = (b0 >= 0 && b0 != b1) ? 4u : 2u;  // 128-byte blocks, two granules each
        }
    }
    const uint32_t ntask = (uint32_t)__popc(mask);
    uint32_t tot;
    const uint32_t pre = wave_excl_scan_u32(ntask, &tot);
    unsigned long long *const ctr[4] = {&cnt->tasks, &cnt->st_occ_reads, &cnt->st_nodes, &cnt->st_frontier_bytes};
    const unsigned long long wtot[4] = {tot, wave_sum_u32(nocc), wave_sum_u32(active ? 1u : 0u), wave_sum_u32(nin)};
    const unsigned long long cap[4] = {caps.tasks, ~0ull, ~0ull, ~0ull};
    const uint32_t ovb[4] = {kOvTasks, 0, 0, 0};
    unsigned long long bases[4];
    block_reserve<4, kTaskBlock / 64, 1>(s_res, ctr, wtot, cap, ovb, &cnt->overflow, bases);
    unsigned long long base = bases[0] + pre;
    if (a.occ_packed) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!(mask & (1u << c))) continue;
            if (base < caps.tasks)
                tasks[base] = ChildTask{a.C[c] + o_lo[c], a.C[c] + o_hi[c] - 1, nd.off, nd.len | ((uint32_t)c << 24)};
            ++base;
        }
    } else {
        for (uint32_t mm = mask; mm; mm &= mm - 1) {
            const int c = __ffs(mm) - 1;
            const uint32_t lo = a.C[c] + occ1_gen(a, c, (int64_t)nd.lo - 1);
            const uint32_t hi = a.C[c] + occ1_gen(a, c, (int64_t)nd.hi) - 1;
            if (base < caps.tasks) tasks[base] = ChildTask{lo, hi, nd.off, nd.len | ((uint32_t)c << 24)};
            ++base;
        }
    }
}

// One lane per node.  The host-driven loop launches a block per 1024 nodes
// (STRIDE false); for device-driven levels (STRIDE true, ctl) the node count
// is read from ctl and a grid of a few blocks per CU strides over the nodes.
// (Two instantiations: the loop costs the one-shot form registers.)
template <bool STRIDE>
__global__ void __launch_bounds__(kTaskBlock) k_level_tasks(SearchArgs a, const Node *nodes, uint32_t nn,
                                                            ChildTask *tasks, Caps caps, Counters *cnt,
                                                            const LevelCtl *ctl) {
    __shared__ BlockReserveLds<4, kTaskBlock / 64> s_res;
    if (STRIDE) {
        if (ctl->stop) return;  // the whole grid
        nn = (uint32_t)ctl->nn;
        for (uint64_t b0 = (uint64_t)blockIdx.x * kTaskBlock; b0 < nn; b0 += (uint64_t)gridDim.x * kTaskBlock)
            level_tasks_tile(a, nodes, nn, (uint32_t)b0 + threadIdx.x, tasks, caps, cnt, s_res);
    } else {
        if ((uint64_t)blockIdx.x * kTaskBlock >= nn) return;  // the whole block
        level_tasks_tile(a, nodes, nn, blockIdx.x * kTaskBlock + threadIdx.x, tasks, caps, cnt, s_res);
    }
}

// The tasks base .. base + kLevelBlock - 1 of one block (t = this lane's).
template <int STAGE>
__device__ inline void expand_child_tile(const SearchArgs &a, const Entry *ent, const ChildTask *tasks, int32_t d1,
                                         const LevelOut &o, const Caps &caps, Counters *cnt, uint64_t t,
                                         uint64_t ntasks, uint32_t *s_stage,
                                         BlockReserveLds<12, kLevelBlock / 64> &s_res) {
    const bool active = t < ntasks && t < caps.tasks;
    Entry *stage = reinterpret_cast<Entry *>(s_stage + threadIdx.x * stage_words(STAGE));
    ChildTask tk{1, 0, 0, 0};
    if (active) tk = tasks[t];
    const Entry *prow = ent + tk.off;
    const uint32_t plen = tk.len_c & 0xFFFFFFu;
    const int tc = (int)(tk.len_c >> 24);
    const bool multi = tk.lo < tk.hi;
    bool staged = true;
    uint32_t n_ent = 0, n_hits = 0, st_d = 0, st_2 = 0, st_3 = 0;
    if (active) {
        RowSink s;
        sink_init(s);
        s.lo = tk.lo;
        s.hi = tk.hi;
        s.out = stage;
        s.cap = (uint32_t)STAGE;
        s.hit_cap = 0;  // count hits now, write them after the allocation
        if (!multi) s.emit_hits = false;
        child_row<true>(a, prow, plen, tc, d1, false, 0, s);
        n_ent = s.n_entries;
        n_hits = s.n_hits;
        st_d = s.st_diag;
        st_2 = s.st_gap2;
        st_3 = s.st_gap3;
        staged = s.n_entries <= s.cap;
    }
    const bool has = active && n_ent > 0;
    const uint32_t c_node = has && multi && n_ent <= (uint32_t)kLaneRow ? 1u : 0u;
    const uint32_t c_wide = has && multi && n_ent > (uint32_t)kLaneRow ? 1u : 0u;
    const uint32_t c_ent = has && multi ? n_ent : 0u;
    const uint32_t c_ch = has && !multi ? 1u : 0u;
    const uint32_t c_ce = has && !multi ? n_ent : 0u;
    uint32_t u_nodes, u_wide, u_ent, u_ch, u_ce, u_hits;
    const unsigned long long p_nodes = wave_excl_scan_u32(c_node, &u_nodes);
    const unsigned long long p_wide = wave_excl_scan_u32(c_wide, &u_wide);
    const unsigned long long p_ent = wave_excl_scan_u32(c_ent, &u_ent);
    const unsigned long long p_ch = wave_excl_scan_u32(c_ch, &u_ch);
    const unsigned long long p_ce = wave_excl_scan_u32(c_ce, &u_ce);
    const unsigned long long p_hits = wave_excl_scan_u32(n_hits, &u_hits);
    // allocations (6) and statistics (6), one atomic per counter and block
    unsigned long long *const ctr[12] = {&cnt->nodes,    &cnt->lwnodes,  &cnt->entries,     &cnt->cnodes,
                                         &cnt->centries, &cnt->hits,     &cnt->st_entries,  &cnt->st_diag,
                                         &cnt->st_gap2,  &cnt->st_gap3,  &cnt->st_emitted,  &cnt->st_frontier_bytes};
    const unsigned long long fb = (unsigned long long)(u_nodes + u_wide + u_ch) * sizeof(Node) +
                                  (unsigned long long)(u_ent + u_ce) * sizeof(Entry) + u_hits * 12ull;
    const unsigned long long wtot[12] = {u_nodes, u_wide, u_ent, u_ch, u_ce, u_hits, wave_sum_u32(n_ent),
                                         wave_sum_u32(st_d), wave_sum_u32(st_2), wave_sum_u32(st_3), u_hits, fb};
    const unsigned long long cap[12] = {caps.nodes, caps.lwnodes, caps.entries, caps.cnodes, caps.centries,
                                        caps.hits,  ~0ull,        ~0ull,        ~0ull,       ~0ull,
                                        ~0ull,      ~0ull};
    const uint32_t ovb[12] = {kOvNodes, kOvLevelWide, kOvEntries, kOvChainNodes, kOvChainEntries, kOvHits,
                              0,        0,            0,          0,             0,               0};
    unsigned long long b[12];
    block_reserve<12, kLevelBlock / 64, 6>(s_res, ctr, wtot, cap, ovb, &cnt->overflow, b);
    const unsigned long long b_nodes = b[0], b_wide = b[1], b_ent = b[2], b_ch = b[3], b_ce = b[4], b_hits = b[5];
    const bool fits = b_nodes + u_nodes <= caps.nodes && b_wide + u_wide <= caps.lwnodes &&
                      b_ent + u_ent <= caps.entries && b_ch + u_ch <= caps.cnodes && b_ce + u_ce <= caps.centries;
    if (has && fits) {
        Entry *dst = multi ? o.oent + b_ent + p_ent : o.cent + b_ce + p_ce;
        const uint32_t off = (uint32_t)(multi ? b_ent + p_ent : b_ce + p_ce);
        if (multi) {
            if (c_wide)
                o.owide[b_wide + p_wide] = Node{tk.lo, tk.hi, off, n_ent};
            else
                o.onodes[b_nodes + p_nodes] = Node{tk.lo, tk.hi, off, n_ent};
        } else {
            o.chains[b_ch + p_ch] = Node{tk.lo, (uint32_t)d1, off, n_ent};
        }
        unsigned long long hslot = b_hits + p_hits;
        if (staged) {
            for (uint32_t k = 0; k < n_ent; ++k) {
                const Entry e = stage[k];
                dst[k] = e;
                if (multi && e.M >= a.H) {  // hits at every occurrence (chains emit their own)
                    for (uint32_t h = tk.lo; h <= tk.hi; ++h, ++hslot) {
                        if (hslot < caps.hits) {
                            o.hkeys[hslot] = ((uint64_t)e.col << 32) | a.sa[h];
                            o.hscores[hslot] = (uint32_t)e.M;
                        }
                    }
                }
            }
        } else {  // second pass straight to the allocated place
            RowSink s;
            sink_init(s);
            s.lo = tk.lo;
            s.hi = tk.hi;
            s.out = dst;
            s.cap = n_ent;
            s.hkeys = o.hkeys;
            s.hscores = o.hscores;
            s.hit_base = hslot;
            s.hit_cap = caps.hits;
            if (!multi) s.emit_hits = false;
            child_row<true>(a, prow, plen, tc, d1, false, 0, s);
        }
    }
}

// One child row per lane, staged in LDS (STAGE entries a lane).  The grid is
// sized for the most tasks a level can have (the host does not wait for the
// node phase's count); blocks past the tasks it made leave at once.  STRIDE
// (device-driven levels, ctl): a grid sized for a small frontier strides over
// the tasks.  Seven blocks per CU: the four-entry stage leaves LDS for seven,
// and the row update fits the 72 registers that allows without spilling (the
// waves wait on dependent reads most of the time; the seventh hides more).
// The eight-entry stage leaves LDS for three.
template <int STAGE, bool STRIDE>
__global__ void __launch_bounds__(kLevelBlock, STAGE == 8 ? 3 : 7) k_expand_children(SearchArgs a, const Entry *ent,
                                                                 const ChildTask *tasks, int32_t d1, LevelOut o,
                                                                 Caps caps, Counters *cnt, const LevelCtl *ctl) {
    __shared__ uint32_t s_stage[kLevelBlock * stage_words(STAGE)];
    __shared__ BlockReserveLds<12, kLevelBlock / 64> s_res;
    if (STRIDE) {  // device-driven levels: the depth is read there
        if (ctl->stop) return;
        d1 = ctl->d1;
    }
    // written by the node phase before this launch (beyond caps.tasks it overflowed and
    // wrote no more: the level is run again)
    const uint64_t made = cnt->tasks;
    const uint64_t ntasks = made < caps.tasks ? made : caps.tasks;
    if (STRIDE) {
        for (uint64_t base = (uint64_t)blockIdx.x * kLevelBlock; base < ntasks;
             base += (uint64_t)gridDim.x * kLevelBlock)
            expand_child_tile<STAGE>(a, ent, tasks, d1, o, caps, cnt, base + threadIdx.x, ntasks, s_stage, s_res);
    } else {
        const uint64_t base = (uint64_t)blockIdx.x * kLevelBlock;
        if (base >= ntasks) return;  // the whole block
        expand_child_tile<STAGE>(a, ent, tasks, d1, o, caps, cnt, base + threadIdx.x, ntasks, s_stage, s_res);
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
        hit_reserve(hr, tot, hkeys, hscores, caps.hits, caps.hit_chunk, cnt);
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
                                                          Counters *cnt, Entry *stage, const LevelCtl *ctl) {
    if (ctl) {  // device-driven levels: the node count and the depth are read there
        if (ctl->stop) return;
        nw = (uint32_t)ctl->nlw;
        d1 = ctl->d1;
    }
    if (blockIdx.x >= nw) return;  // a block with no node (its statistics are all zero)
    const int lane = threadIdx.x & 63;
    Entry *buf = stage + (uint64_t)blockIdx.x * caps.srow;
    HitRes hr = {0, 0, 0};
    unsigned long long emitted = 0, entries = 0, diag = 0, gap2 = 0, gap3 = 0;
    for (uint32_t item = blockIdx.x; item < nw; item += gridDim.x) {
        const Node nd = wnodes[item];
        uint32_t o1[4] = {0, 0, 0, 0}, o2[4] = {0, 0, 0, 0};
        if (a.occ_packed) {
            occ4_dna(a, (int64_t)nd.lo - 1, o1);
            occ4_dna(a, (int64_t)nd.hi, o2);
        }
        for (int c = 0; c < a.sigma; ++c) {
            int64_t l, r;
            if (a.occ_packed) {
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
            w.hit_chunk = caps.hit_chunk;
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
