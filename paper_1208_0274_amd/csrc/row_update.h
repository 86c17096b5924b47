// Sparse DP row update of a trie node (Section 2.2 recurrences with the
// filters of Section 3), in two forms:
//   child_row       -- one lane computes a whole child row sequentially;
//   wide_child_row  -- one wave (or the W waves of a block) computes a child
//                      row 64 (64*W) parent entries at a time, with G_b as a
//                      wave-level prefix-max scan carried across waves.
// Both produce the same entries (column, M, G_a, start tags) for the same
// parent row.
#pragma once

#include <type_traits>

#include "device_common.h"

namespace alae {

constexpr int64_t kNegKey = INT64_MIN / 4;
constexpr int kGapWindow = 96;  // window side of the gapped domination test

// ---------------------------------------------------------------------------
// Domination (Section 3.2, Theorem 4 case 2 and Lemma 1, tested locally)
// ---------------------------------------------------------------------------
// A state whose best alignment starts at text position x, query column y is
// dominated when an alignment ending exactly at (x-1, y-1) scores above zero:
// prepending it beats that alignment at every cell it can reach, so the state
// can never carry the maximum of a cell.

// The 32 bytes arr[p-32 .. p-1] as eight little-endian words (arr carries
// kSlack readable bytes around its data).
__device__ inline void load_window32(const uint8_t *arr, int64_t p, uint32_t w[8]) {
    const uintptr_t addr = (uintptr_t)(arr + p - 32);
    const uint32_t *base = reinterpret_cast<const uint32_t *>(addr & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(addr & 3u);
    uint32_t r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = base[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = __builtin_amdgcn_alignbyte(r[i + 1], r[i], sh);
}

// Ungapped form: some suffix of T[x-k..x-1] against P[y-k..y-1] (k <= 32)
// scores > 0.  sub is the substitution table (LDS) for matrix scoring.
// tw: the text window T[x-32..x-1] (load_window32), shared by every state
// tested at the same x.
__device__ inline bool dominated_tw(const SearchArgs &a, const int8_t *sub, const uint32_t (&tw)[8], int64_t x,
                                    int64_t y) {
    int64_t reach = a.dom_reach;
    if (x < reach) reach = x;
    const int64_t yl = (int64_t)seg_off(a, (uint32_t)y);  // columns of y's query before y
    if (yl < reach) reach = yl;
    if (reach <= 0) return false;
    if (a.has_sep) {  // an alignment never reaches across a record separator
        for (int k = 1; k <= 32 && k <= reach; ++k) {
            const int j = 32 - k;
            if (((tw[j >> 2] >> (8 * (j & 3))) & 0xFFu) >= (uint32_t)a.sigma) {
                reach = k - 1;
                break;
            }
        }
        if (reach <= 0) return false;
    }
    uint32_t qw[8];
    load_window32(a.query, y, qw);
    int32_t sum = 0;
    bool dom = false;
    // eight characters at a time; a lane stops once its sum can no longer turn
    // positive within the reach (each character adds at most s_max)
#pragma unroll
    for (int k0 = 1; k0 <= 32; k0 += 8) {
#pragma unroll
        for (int k = k0; k < k0 + 8; ++k) {
            const int j = 32 - k;
            uint32_t tc = (tw[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            const uint32_t pc = (qw[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            if (a.matrix_mode && tc >= (uint32_t)a.sigma) tc = 0;  // past the reach; keeps the table index inside
            const int32_t d = a.matrix_mode ? (int32_t)sub[tc * (uint32_t)a.sigma + pc]
                                            : (tc == pc ? a.s_match : a.s_mismatch);
            if (k <= reach) {
                sum += d;
                dom |= sum > 0;
            }
        }
        const int64_t left = reach - (k0 + 7);
        if (dom || left <= 0 || sum + (int64_t)a.smax * left <= 0) break;
    }
    return dom;
}

__device__ inline bool dominated(const SearchArgs &a, const int8_t *sub, int64_t x, int64_t y) {
    uint32_t tw[8];
    load_window32(a.text, x, tw);
    return dominated_tw(a, sub, tw, x, y);
}

// Gapped form: the best local alignment score ending exactly at (x-1, y-1),
// computed inside the window T[x-K..x-1] x P[y-K..y-1] and within a band of
// kGapBand diagonals on either side of the one through (x-1, y-1) (a lower
// bound of the true score, so the test stays sufficient).  Band cell k of
// window row i is column j = i + off + k; the band's H and vertical-gap
// values live in registers, updated in place with k ascending (cell k reads
// the previous row at k and k+1 and this row at k-1).
constexpr int kGapBand = 8;

__device__ inline bool dominated_gapped(const SearchArgs &a, int64_t x, int64_t y) {
    constexpr int W = kGapBand, B = 2 * kGapBand + 1;
    const int64_t yl = (int64_t)seg_off(a, (uint32_t)y);
    int R = (int)(x < kGapWindow ? x : kGapWindow);
    const int C = (int)(yl < kGapWindow ? yl : kGapWindow);
    // the window's text rows stop at a record separator (no alignment crosses one)
    if (a.has_sep) {
        for (int i = 1; i <= R; ++i) {
            if (a.text[x - i] >= (uint32_t)a.sigma) {
                R = i - 1;
                break;
            }
        }
    }
    if (R == 0 || C == 0) return false;
    const int32_t open = a.sg + a.ss;
    const int off = C - R;           // column of band cell 0 in row i is i + off
    const int64_t q0 = y - C;        // query index of window column 0
    int32_t Hb[B], Eb[B];
    uint32_t qc[B];                  // query code of each band cell's column in the current row
#pragma unroll
    for (int k = 0; k < B; ++k) {
        Hb[k] = 0;  // the row above the window: local-alignment boundary
        Eb[k] = kNeg;
        const int j = off + k - W - 1;  // columns of row -1; shifted in before row 0
        const bool in = j >= 0 && j < C;
        const uint32_t v = a.query[q0 + (in ? j : 0)];  // the index stays inside the window
        qc[k] = in ? v : 0xFFu;
    }
    for (int i = 0; i < R; ++i) {
        // slide the band one column to the right
#pragma unroll
        for (int k = 0; k < B - 1; ++k) qc[k] = qc[k + 1];
        {
            const int j = i + off + W;
            const bool in = j >= 0 && j < C;
            const uint32_t v = a.query[q0 + (in ? j : 0)];
            qc[B - 1] = in ? v : 0xFFu;
        }
        const uint32_t tc = a.text[x - R + i];
        const int8_t *prow = a.prof + (size_t)tc * a.m;
        int32_t Hleft = kNeg, F = kNeg;
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int j = i + off + k - W;
            const bool inside = j >= 0 && j < C;
            const int32_t upH = k + 1 < B ? Hb[k + 1] : kNeg;
            const int32_t upE = k + 1 < B ? Eb[k + 1] : kNeg;
            const int32_t E = imax(upE + a.ss, upH + open);
            F = imax(F + a.ss, Hleft + open);
            int32_t s;
            if (a.matrix_mode)
                s = (int32_t)prow[q0 + (inside ? j : 0)];
            else
                s = tc == qc[k] ? a.s_match : a.s_mismatch;
            int32_t h = imax(Hb[k] + s, imax(E, F));
            h = imax(h, 0);
            if (j < 0) h = 0;             // left of the window: where alignments start
            const bool live = inside || j < 0;
            Hb[k] = live ? h : kNeg;     // right of the window: never part of an alignment to the corner
            Eb[k] = inside ? E : kNeg;
            Hleft = Hb[k];
            if (!inside) F = kNeg;
        }
    }
    return Hb[W] > 0;  // band cell W of the last row is column C-1
}

// ---------------------------------------------------------------------------
// Filters
// ---------------------------------------------------------------------------
// Zero floor (Theorem 2 (i)) and score filter (Theorem 2 (ii)) for a state of
// value v at column col of a row at depth d1: the gain still available is at
// most min(U(col), smax * (L_max - d1)) (query columns left, text rows left
// under Theorem 1).  rowgain = smax * (L_max - d1); send is the end of col's
// query (one past its last column).
__device__ inline bool keep_state_e(const SearchArgs &a, int32_t v, uint32_t col, uint32_t send, int32_t rowgain) {
    if (v <= 0) return false;
    if (!a.use_score_filter) return true;
    int32_t g = a.u_closed ? a.smax * (int32_t)(send - 1 - col) : a.U[col];
    if (rowgain < g) g = rowgain;
    return v + g >= a.H;
}

// ---------------------------------------------------------------------------
// Sequential (one lane) row update
// ---------------------------------------------------------------------------

struct RowSink {
    Entry *out;          // output row
    uint32_t cap;        // entries that may be written to out
    bool emit_hits;      // write hit records while producing the row
    uint64_t *hkeys;
    uint32_t *hscores;
    unsigned long long hit_base;
    unsigned long long hit_cap;
    // occurrences of the child
    bool unique;
    uint32_t e_end;      // unique: text end of the occurrence
    uint32_t lo, hi;     // otherwise: BWT rows
    // results
    uint32_t n_entries;  // may exceed cap (then only cap entries were written)
    uint32_t n_hits;
    uint32_t st_diag, st_gap2, st_gap3, st_dom;
};

__device__ inline void sink_init(RowSink &s) {
    s.out = nullptr;
    s.cap = 0xFFFFFFFFu;
    s.emit_hits = true;
    s.hkeys = nullptr;
    s.hscores = nullptr;
    s.hit_base = 0;
    s.hit_cap = 0;
    s.unique = false;
    s.e_end = 0;
    s.lo = s.hi = 0;
    s.n_entries = s.n_hits = 0;
    s.st_diag = s.st_gap2 = s.st_gap3 = s.st_dom = 0;
}

template <bool WRITE>
__device__ inline void emit_entry(const SearchArgs &a, RowSink &s, uint32_t col, int32_t M, int32_t Ga, uint32_t yM,
                                  uint32_t yGa, int inputs) {
    if (WRITE) {
        if (s.n_entries < s.cap) {
            Entry e;
            e.col = col;
            e.M = M;
            e.Ga = Ga;
            e.yM = yM;
            e.yGa = yGa;
            s.out[s.n_entries] = e;
        }
        if (inputs <= 1)
            s.st_diag++;
        else if (inputs == 2)
            s.st_gap2++;
        else
            s.st_gap3++;
    }
    s.n_entries++;
    if (!s.emit_hits || M < a.H) return;
    if (s.unique) {
        if (WRITE) {
            const unsigned long long slot = s.hit_base + s.n_hits;
            if (slot < s.hit_cap) {
                s.hkeys[slot] = ((uint64_t)col << 32) | s.e_end;
                s.hscores[slot] = (uint32_t)M;
            }
        }
        s.n_hits++;
    } else {
        for (uint32_t h = s.lo; h <= s.hi; ++h) {
            if (WRITE) {
                const unsigned long long slot = s.hit_base + s.n_hits;
                if (slot < s.hit_cap) {
                    s.hkeys[slot] = ((uint64_t)col << 32) | a.sa[h];
                    s.hscores[slot] = (uint32_t)M;
                }
            }
            s.n_hits++;
        }
    }
}

// The row at depth d1 of the child reached with character c, from the parent
// row prow[0..plen) (sorted by column).  Candidate columns are the parent's
// columns (G_a: a text character against a gap) and the parent's columns + 1
// (diagonal); G_b (a query character against a gap) runs left to right along
// the row, also through columns with no candidate.  check_dom applies the
// ungapped domination test for the occurrence starting at text position x.
template <bool WRITE>
__device__ void child_row(const SearchArgs &a, const Entry *prow, uint32_t plen, int c, int32_t d1, bool check_dom,
                          int64_t x, RowSink &s, const int8_t *sub = nullptr) {
    const int8_t *pc = a.prof + (size_t)c * a.m;
    const int32_t open = a.sg + a.ss;  // first gap character
    const int32_t ext = a.ss;
    const int32_t rowgain = a.smax * (a.lmax - d1);
    int64_t last = -1;     // last column already handled
    uint32_t last_end = 0; // end of last's query (valid while gnext > 0)
    int32_t gnext = kNeg;  // G_b value for column last+1
    uint32_t gy = 0;       // its start column

    auto spread_to = [&](int64_t upto) {  // G_b-only columns last+1 .. upto
        if (gnext > 0) {
            // a query gap never runs into the next query
            const int64_t lim = upto < (int64_t)last_end - 1 ? upto : (int64_t)last_end - 1;
            while (last < lim) {
                if (gnext <= 0) break;
                const uint32_t col = (uint32_t)(last + 1);
                const int32_t v = gnext;
                if (!keep_state_e(a, v, col, last_end, rowgain)) break;  // later columns only lose more
                if (check_dom && dominated(a, sub, x, gy)) {
                    s.st_dom++;
                } else {
                    emit_entry<WRITE>(a, s, col, v, kNeg, gy, 0, 1);
                }
                last = col;
                gnext = v + ext;
            }
        }
        if (last < upto) {
            last = upto;
            gnext = kNeg;
        }
    };

    // column j (first: j starts its query; send: end of j's query)
    auto column = [&](uint32_t j, bool first, uint32_t send, int32_t D, uint32_t yD, int32_t Gav, uint32_t yGav) {
        spread_to((int64_t)j - 1);
        const int32_t Gb = (last == (int64_t)j - 1 && !first) ? gnext : kNeg;
        const uint32_t yGb = gy;
        int32_t M = D;
        uint32_t yM = yD;
        if (Gav > M) {
            M = Gav;
            yM = yGav;
        }
        if (Gb > M) {
            M = Gb;
            yM = yGb;
        }
        const bool keepM = keep_state_e(a, M, j, send, rowgain);
        const bool keepGa = keep_state_e(a, Gav, j, send, rowgain);
        // G_b for column j+1 from this column's states that survive the filters
        int32_t gn = kNeg;
        uint32_t gny = 0;
        if (keepM) {
            gn = M + open;
            gny = yM;
            if (Gb + ext > gn && Gb > 0) {
                gn = Gb + ext;
                gny = yGb;
            }
        }
        last = j;
        last_end = send;
        gnext = gn;
        gy = gny;
        bool liveM = keepM, liveGa = keepGa;
        if (check_dom) {
            if (liveM && dominated(a, sub, x, yM)) {
                liveM = false;
                s.st_dom++;
            }
            if (liveGa && dominated(a, sub, x, yGav)) {
                liveGa = false;
                s.st_dom++;
            }
        }
        if (liveM || liveGa) {
            const int inputs = (D > 0) + (Gav > 0) + (Gb > 0);
            emit_entry<WRITE>(a, s, j, liveM ? M : kNeg, liveGa ? Gav : kNeg, liveM ? yM : 0, liveGa ? yGav : 0,
                              inputs);
        }
    };

    // parent entries k-1, k, k+1 move along in registers: one load per entry,
    // issued an entry ahead (the row's stores may alias it for the compiler)
    // with the score of the diagonal step after each (clamped into the row:
    // used only where the column exists) and the column's query segment
    const uint32_t lastcol = a.m - 1;
    auto diag_score = [&](uint32_t col) -> int32_t { return pc[col < lastcol ? col + 1 : lastcol]; };
    Entry p{0, kNeg, kNeg, 0, 0};
    Entry nx{0, kNeg, kNeg, 0, 0};
    int32_t p_s = 0, nx_s = 0;
    uint32_t nx_seg = 0;
    // parent entries are read four at a time (80 contiguous bytes a lane), so that a
    // lane's row is fetched while its lines are in the cache
    Entry q0 = nx, q1 = nx, q2 = nx, q3 = nx;
    uint32_t qb = 0xFFFFFFFFu;
    auto parent = [&](uint32_t k) -> Entry {
        const uint32_t b = k & ~3u;
        if (b != qb) {
            qb = b;
            q0 = prow[b];
            if (b + 1 < plen) q1 = prow[b + 1];
            if (b + 2 < plen) q2 = prow[b + 2];
            if (b + 3 < plen) q3 = prow[b + 3];
        }
        const uint32_t r = k & 3u;
        return r == 0 ? q0 : r == 1 ? q1 : r == 2 ? q2 : q3;
    };
    if (plen > 0) {
        nx = parent(0);
        nx_s = diag_score(nx.col);
        nx_seg = seg_info(a, nx.col);
    }
    for (uint32_t k = 0; k < plen; ++k) {
        const Entry e = nx;
        const int32_t e_s = nx_s;
        const uint32_t e_seg = nx_seg;
        const bool has_next = k + 1 < plen;
        if (has_next) {
            nx = parent(k + 1);
            nx_s = diag_score(nx.col);
            nx_seg = seg_info(a, nx.col);
        }
        const uint32_t j = e.col;
        const bool first = a.multi && (e_seg & kSegFirst) != 0;
        const uint32_t send = j + seg_dist(e_seg);
        // diagonal from the previous parent entry, if it sits in column j-1
        int32_t D = kNeg;
        uint32_t yD = 0;
        if (k > 0) {
            if (p.col + 1 == j && p.M > 0 && !first) {
                D = p.M + p_s;
                yD = p.yM;
            }
        }
        // G_a: extend the parent's G_a or open from the parent's M in column j
        int32_t Gav = kNeg;
        uint32_t yGav = 0;
        if (e.Ga > 0) {
            Gav = e.Ga + ext;
            yGav = e.yGa;
        }
        if (e.M > 0 && e.M + open > Gav) {
            Gav = e.M + open;
            yGav = e.yM;
        }
        column(j, first, send, D, yD, Gav, yGav);
        // diagonal into column j+1 when no parent entry sits there
        if (e.M > 0 && j + 1 < send && !(has_next && nx.col == j + 1)) {
            column(j + 1, false, send, e.M + e_s, e.yM, kNeg, 0);
        }
        p = e;
        p_s = e_s;
    }
    spread_to((int64_t)a.m - 1);
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64)
// ---------------------------------------------------------------------------

// Cross-lane moves through DPP (no LDS round trip).  Row ops act within
// each 16-lane row; a lane with no source keeps `old`.
constexpr int kDppWaveShl1 = 0x130;   // lane L reads lane L+1
constexpr int kDppWaveShr1 = 0x138;   // lane L reads lane L-1
constexpr int kDppRowShr = 0x110;     // + n: lane L reads lane L-n of its row
constexpr int kDppRowBcast15 = 0x142; // lane 15 of a row to the next row
constexpr int kDppRowBcast31 = 0x143; // lane 31 to rows 2 and 3

template <int CTRL, int ROW_MASK = 0xF>
__device__ inline uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}

__device__ inline uint32_t lane_up1(uint32_t v) { return dpp<kDppWaveShr1>(v, v); }    // lane 0 keeps its own
__device__ inline uint32_t lane_down1(uint32_t v) { return dpp<kDppWaveShl1>(v, v); }  // lane 63 keeps its own
__device__ inline int32_t lane_up1(int32_t v) { return (int32_t)lane_up1((uint32_t)v); }

// Inclusive prefix sum over the 64 lanes.
__device__ inline uint32_t wave_incl_add_u32(uint32_t v) {
    v += dpp<kDppRowShr + 1>(0u, v);
    v += dpp<kDppRowShr + 2>(0u, v);
    v += dpp<kDppRowShr + 4>(0u, v);
    v += dpp<kDppRowShr + 8>(0u, v);
    v += dpp<kDppRowBcast15, 0xA>(0u, v);
    v += dpp<kDppRowBcast31, 0xC>(0u, v);
    return v;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_add_u32(v), 63);
}

// Lane 0's value in every lane.
__device__ inline unsigned long long bcast0_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 0);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 0);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ inline unsigned long long wave_excl_scan_u64(unsigned long long v, unsigned long long *total) {
    const int lane = threadIdx.x & 63;
    unsigned long long inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

__device__ inline uint32_t wave_excl_scan_u32(uint32_t v, uint32_t *total) {
    const uint32_t inc = wave_incl_add_u32(v);
    *total = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    return inc - v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Block-wide reservation.  Every wave passes its totals for NC global
// counters (the same value in all of its lanes); thread 0 adds the block's
// totals with one atomic per counter, and each wave gets back its first slot
// per counter.  Atomics on one address are served one at a time by the
// memory system, so allocating per block instead of per wave divides that
// serial work by the block's wave count.  A counter whose block range passes
// its capacity raises its overflow bit.  Every thread of the block calls it.
// ---------------------------------------------------------------------------
template <int NC, int NW>
struct BlockReserveLds {
    unsigned long long tot[NW][NC];
    unsigned long long base[NC];
};

// Counters from NRES on are statistics: added without waiting for the old
// value (their base[] entries are 0).
template <int NC, int NW, int NRES = NC>
__device__ inline void block_reserve(BlockReserveLds<NC, NW> &sh, unsigned long long *const (&ctr)[NC],
                                     const unsigned long long (&tot)[NC], const unsigned long long (&cap)[NC],
                                     const uint32_t (&ovbit)[NC], unsigned long long *overflow,
                                     unsigned long long (&base)[NC]) {
    const int lane = threadIdx.x & 63;
    const int wave = (int)(threadIdx.x >> 6);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) sh.tot[wave][c] = tot[c];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // lane c of the first wave takes counter c, so the block's atomics are in flight
        // together instead of one round trip after another
        unsigned long long all = 0, b = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if ((int)threadIdx.x == c) {
#pragma unroll
                for (int w = 0; w < NW; ++w) all += sh.tot[w][c];
                if (all && c < NRES)
                    b = atomicAdd(ctr[c], all);
                else if (all)
                    __hip_atomic_fetch_add(ctr[c], all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        uint32_t of = 0;
#pragma unroll
        for (int c = 0; c < NRES; ++c)
            if ((int)threadIdx.x == c && all && b + all > cap[c]) of = ovbit[c];
        if ((int)threadIdx.x < NC) sh.base[threadIdx.x] = b;
        if (of) atomicOr(overflow, (unsigned long long)of);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        unsigned long long b = sh.base[c];
#pragma unroll
        for (int w = 0; w < NW; ++w) b += w < wave ? sh.tot[w][c] : 0ull;
        base[c] = b;
    }
    __syncthreads();  // sh is free for the next call
}

// Exclusive max-scan of a 32-bit key over the lanes of a wave (no tags):
// ex = max over lanes below (kNegKey32 if none), all = over all lanes.
constexpr int32_t kNegKey32 = INT32_MIN / 4;
__device__ inline void wave_excl_max_i32(int32_t key, int32_t &ex, int32_t &all) {
    const uint32_t id = (uint32_t)kNegKey32;
    int32_t k = (int32_t)dpp<kDppWaveShr1>(id, (uint32_t)key);
    k = imax(k, (int32_t)dpp<kDppRowShr + 1, 0xF>(id, (uint32_t)k));
    k = imax(k, (int32_t)dpp<kDppRowShr + 2, 0xF>(id, (uint32_t)k));
    k = imax(k, (int32_t)dpp<kDppRowShr + 4, 0xF>(id, (uint32_t)k));
    k = imax(k, (int32_t)dpp<kDppRowShr + 8, 0xF>(id, (uint32_t)k));
    k = imax(k, (int32_t)dpp<kDppRowBcast15, 0xA>(id, (uint32_t)k));
    k = imax(k, (int32_t)dpp<kDppRowBcast31, 0xC>(id, (uint32_t)k));
    ex = k;
    all = __builtin_amdgcn_readlane(imax(k, key), 63);
}

// Exclusive max-scan of (key, tag) over the lanes of a wave; ties keep the
// lower lane.  ex: max over lanes below (kNegKey if none); all: over all lanes.
// The key moves as two 32-bit halves; kNegKey is the identity.
__device__ inline void wave_excl_max(int64_t key, uint32_t tag, int64_t &ex_key, uint32_t &ex_tag, int64_t &all_key,
                                     uint32_t &all_tag) {
    const uint32_t nlo = (uint32_t)(uint64_t)kNegKey, nhi = (uint32_t)((uint64_t)kNegKey >> 32);
    auto join = [](uint32_t lo, uint32_t hi) { return (int64_t)(((uint64_t)hi << 32) | lo); };
    // shift by one lane: lane L starts from lane L-1's value (lane 0 from the identity)
    uint32_t lo = dpp<kDppWaveShr1>(nlo, (uint32_t)(uint64_t)key);
    uint32_t hi = dpp<kDppWaveShr1>(nhi, (uint32_t)((uint64_t)key >> 32));
    uint32_t tg = dpp<kDppWaveShr1>(0u, tag);
    int64_t k = join(lo, hi);
    auto step = [&](uint32_t olo, uint32_t ohi, uint32_t otg) {
        const int64_t ok = join(olo, ohi);
        if (ok >= k) {  // the incoming value comes from lower lanes: it wins ties
            k = ok;
            tg = otg;
        }
    };
#define ALAE_MAX_STEP(CTRL, MASK)                                                          \
    {                                                                                      \
        const uint32_t klo = (uint32_t)(uint64_t)k, khi = (uint32_t)((uint64_t)k >> 32);   \
        step(dpp<CTRL, MASK>(nlo, klo), dpp<CTRL, MASK>(nhi, khi), dpp<CTRL, MASK>(0u, tg)); \
    }
    ALAE_MAX_STEP(kDppRowShr + 1, 0xF)
    ALAE_MAX_STEP(kDppRowShr + 2, 0xF)
    ALAE_MAX_STEP(kDppRowShr + 4, 0xF)
    ALAE_MAX_STEP(kDppRowShr + 8, 0xF)
    ALAE_MAX_STEP(kDppRowBcast15, 0xA)
    ALAE_MAX_STEP(kDppRowBcast31, 0xC)
#undef ALAE_MAX_STEP
    ex_key = k;
    ex_tag = tg;
    // over all lanes: lane 63's exclusive value against its own
    int64_t a63 = k;
    uint32_t t63 = tg;
    if (!(k >= key)) {
        a63 = key;
        t63 = tag;
    }
    const uint32_t alo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)a63, 63);
    const uint32_t ahi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)a63 >> 32), 63);
    all_key = join(alo, ahi);
    all_tag = (uint32_t)__builtin_amdgcn_readlane((int)t63, 63);
}

// ---------------------------------------------------------------------------
// Wave-parallel row update of a single-occurrence node
// ---------------------------------------------------------------------------
//
// With key(k) = M0(k) + |ss| * k over the candidate columns k (M0 = the
// diagonal/G_a part of M), the query-gap state is
//     G_b(j) = sg - |ss| * j + max over candidates k < j of key(k),
// an exclusive prefix maximum along the row (opening a gap from a G_b state is
// never better than extending it, because sg <= 0).  Each lane owns one
// parent entry: its column (G_a, and the diagonal of the previous entry) and
// the next column (diagonal), plus the G_b-only columns up to the next lane's
// first column.

// Row storage seen by the wave-parallel update: entries with start tags in
// global memory, or column/M/G_a arrays (no tags) in LDS.
struct AosRow {
    static constexpr bool kTags = true;
    Entry *p;
    __device__ Entry load(uint32_t k) const { return p[k]; }
    __device__ void store(uint32_t k, const Entry &e) const { p[k] = e; }
};

struct SoaRow {
    static constexpr bool kTags = false;
    uint32_t *col;
    int32_t *M;
    int32_t *Ga;
    __device__ Entry load(uint32_t k) const {
        Entry e;
        e.col = col[k];
        e.M = M[k];
        e.Ga = Ga[k];
        e.yM = 0;
        e.yGa = 0;
        return e;
    }
    __device__ void store(uint32_t k, const Entry &e) const {
        col[k] = e.col;
        M[k] = e.M;
        Ga[k] = e.Ga;
    }
};

// Hit slots reserved by one wave in chunks (of Caps::hit_chunk slots, at least
// the records needed at once); slots left unused are filled with kPadKey so
// that they sort after every real record.
constexpr unsigned long long kHitChunk = 4096;
struct HitRes {
    unsigned long long base;
    unsigned long long left;
    unsigned long long pad;
};

__device__ inline void hit_reserve(HitRes &r, unsigned long long need, uint64_t *hkeys, uint32_t *hscores,
                                   unsigned long long hit_cap, unsigned long long chunk, Counters *cnt) {
    if (need <= r.left) return;
    const int lane = threadIdx.x & 63;
    for (unsigned long long k = lane; k < r.left; k += 64) {
        const unsigned long long slot = r.base + k;
        if (slot < hit_cap) {
            hkeys[slot] = kPadKey;
            hscores[slot] = 0;
        }
    }
    r.pad += r.left;
    const unsigned long long take = need > chunk ? need : chunk;
    unsigned long long b = 0;
    if (lane == 0) {
        b = atomicAdd(&cnt->hits, take);
        if (b + take > hit_cap) atomicOr(&cnt->overflow, kOvHits);
    }
    r.base = __shfl(b, 0, 64);
    r.left = take;
}

__device__ inline void hit_release(HitRes &r, uint64_t *hkeys, uint32_t *hscores, unsigned long long hit_cap,
                                   Counters *cnt) {
    const int lane = threadIdx.x & 63;
    for (unsigned long long k = lane; k < r.left; k += 64) {
        const unsigned long long slot = r.base + k;
        if (slot < hit_cap) {
            hkeys[slot] = kPadKey;
            hscores[slot] = 0;
        }
    }
    r.pad += r.left;
    r.left = 0;
    if (lane == 0 && r.pad) atomicAdd(&cnt->hit_padding, r.pad);
    r.pad = 0;
}

struct WideOut {
    bool emit_hits;    // emit hit records at e_child (single-occurrence nodes)
    uint32_t cap;      // capacity of the output row
    uint64_t *hkeys;
    uint32_t *hscores;
    unsigned long long hit_cap;
    unsigned long long hit_chunk;
    Counters *cnt;
    uint32_t e_child;  // text end of the child occurrence (hit coordinate)
    // replayed forks: every hit is also emitted at col + rdelta[r], r = 1..rK
    uint32_t rK;
    const uint32_t *rdelta;
    // results: len and overflow are uniform over the lanes that update the
    // row, hits over a wave; diag, gap2 and gap3 are per lane
    uint32_t len;
    bool overflow;
    unsigned long long hits, diag, gap2, gap3;
};

// Exchange slots of a block whose W waves update one row together (LDS);
// two sets, used by alternate rounds.
constexpr int kMaxRowWaves = 8;
struct RowXchg {
    int64_t key[2][kMaxRowWaves];
    uint32_t tag[2][kMaxRowWaves];
    uint32_t cnt[2][kMaxRowWaves];
};

// W == 1: one wave walks the row 64 parent entries per round, carrying the
// G_b prefix maximum and the output offset in registers.  W > 1: the block's
// W waves take 64*W entries per round; the carries of the waves before each
// one (prefix maximum, output count) pass through xg, with two barriers a
// round.  Both give the same row.
// FAST: a single query whose prefix-max keys fit 31 bits ((s_max + |s_s|) m <
// 2^30) and rows without start tags; the scan then moves one 32-bit key.
template <int W = 1, bool FAST = false, class Row>
__device__ inline void wide_child_row(const SearchArgs &a, const Row cur, uint32_t len, const Row nxt, int c,
                                      int32_t d1, WideOut &o, HitRes &hr, RowXchg *xg = nullptr) {
    static_assert(W >= 1 && W <= kMaxRowWaves, "waves per row");
    static_assert(!FAST || !Row::kTags, "the 32-bit scan carries no start tags");
    const int lane = threadIdx.x & 63;
    const int wave = W > 1 ? (int)(threadIdx.x >> 6) : 0;
    int par = 0;
    const int8_t *pc = a.prof + (size_t)c * a.m;
    const int32_t open = a.sg + a.ss;
    const int32_t ext = a.ss;
    // prefix-max keys: 32-bit for FAST, else 64-bit with the query segment offset
    using Key = std::conditional_t<FAST, int32_t, int64_t>;
    constexpr Key kNoKey = FAST ? (Key)kNegKey32 : (Key)kNegKey;
    const Key absss = -(Key)a.ss;
    const int32_t rowgain = a.smax * (a.lmax - d1);
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    // carries between rounds (wave-uniform)
    uint32_t c_pcol = kNone, c_pyM = 0;
    int32_t c_pM = kNeg;
    Key c_key = kNoKey;
    uint32_t c_tag = 0;
    uint32_t out = 0;
    bool overflow = false;
    unsigned long long hits = 0, diag = 0, gap2 = 0, gap3 = 0;
    for (uint32_t rbase = 0; rbase < len; rbase += 64u * W) {
        const uint32_t base = rbase + 64u * (uint32_t)wave;
        const uint32_t k = base + lane;
        const bool valid = k < len;
        Entry e;
        if (valid) {
            e = cur.load(k);
        } else {
            e.col = kNone;
            e.M = kNeg;
            e.Ga = kNeg;
            e.yM = 0;
            e.yGa = 0;
        }
        uint32_t pcol = lane_up1(e.col);
        int32_t pM = lane_up1(e.M);
        uint32_t pyM = Row::kTags ? lane_up1(e.yM) : 0u;
        if (lane == 0) {
            if (W == 1) {
                pcol = c_pcol;
                pM = c_pM;
                pyM = c_pyM;
            } else if (valid && k > 0) {  // the entry before this wave's first
                const Entry pe = cur.load(k - 1);
                pcol = pe.col;
                pM = pe.M;
                pyM = pe.yM;
            } else {
                pcol = kNone;
                pM = kNeg;
                pyM = 0;
            }
        }
        uint32_t ncol = lane_down1(e.col);
        if (lane == 63) ncol = (k + 1 < len) ? cur.load(k + 1).col : kNone;
        if (k + 1 >= len) ncol = kNone;
        // this entry's query: its end, and whether e.col starts it (one load in a batch)
        const uint32_t sinfo = (FAST || !valid) ? 0u : seg_info(a, e.col);
        const bool sfirst = !FAST && a.multi && (sinfo & kSegFirst) != 0;
        // column A = e.col: diagonal from the previous entry and G_a
        int32_t D = kNeg;
        uint32_t yD = 0;
        if (valid && pcol != kNone && pcol + 1 == e.col && pM > 0 && !sfirst) {
            D = pM + pc[e.col];
            yD = pyM;
        }
        int32_t GaA = kNeg;
        uint32_t yGaA = 0;
        if (valid) {
            if (e.Ga > 0) {
                GaA = e.Ga + ext;
                yGaA = e.yGa;
            }
            if (e.M > 0 && e.M + open > GaA) {
                GaA = e.M + open;
                yGaA = e.yM;
            }
        }
        int32_t M0A = D;
        uint32_t yM0A = yD;
        if (GaA > M0A) {
            M0A = GaA;
            yM0A = yGaA;
        }
        // column B = e.col + 1: diagonal only, unless the next entry owns it
        const uint32_t send = FAST ? a.m : (valid ? e.col + seg_dist(sinfo) : 0u);  // end of this entry's query
        const Key skey = FAST ? 0 : (valid ? (Key)seg_key(a, e.col) : 0);
        const bool hasB = valid && e.M > 0 && e.col + 1 < send && ncol != e.col + 1;
        const int32_t M0B = hasB ? e.M + pc[e.col + 1] : kNeg;
        const uint32_t yM0B = e.yM;
        const Key kA = (valid && M0A > 0) ? (Key)M0A + absss * (Key)e.col + skey : kNoKey;
        const Key kB = (hasB && M0B > 0) ? (Key)M0B + absss * (Key)(e.col + 1) + skey : kNoKey;
        Key lk = kA;
        uint32_t lt = yM0A;
        if (kB > lk) {
            lk = kB;
            lt = yM0B;
        }
        Key exk, allk;
        uint32_t ext_tag, allt;
        if constexpr (FAST) {
            wave_excl_max_i32(lk, exk, allk);
            ext_tag = allt = 0;
        } else {
            wave_excl_max(lk, lt, exk, ext_tag, allk, allt);
        }
        // carry-in: earlier rounds, then the waves before this one (earlier wins ties)
        Key cin = c_key;
        uint32_t cint = c_tag;
        if (W > 1) {
            if (lane == 0) {
                xg->key[par][wave] = allk;
                xg->tag[par][wave] = allt;
            }
            __syncthreads();
            Key bk = c_key;
            uint32_t bt = c_tag;
#pragma unroll
            for (int w2 = 0; w2 < W; ++w2) {
                if (w2 == wave) {
                    cin = bk;
                    cint = bt;
                }
                const Key kk = (Key)xg->key[par][w2];
                if (kk > bk) {
                    bk = kk;
                    bt = xg->tag[par][w2];
                }
            }
            allk = bk;  // the whole round, for the next one
            allt = bt;
        }
        if (cin >= exk) {  // earlier rounds come first
            exk = cin;
            ext_tag = cint;
        }
        // G_b and M at A
        int32_t GbA = kNeg;
        if (valid && exk > kNoKey) {
            const Key v = exk + a.sg - absss * (Key)e.col - skey;
            GbA = v > 0 ? (int32_t)v : kNeg;
        }
        int32_t MA = M0A;
        uint32_t yMA = yM0A;
        if (GbA > MA) {
            MA = GbA;
            yMA = ext_tag;
        }
        const bool keepMA = valid && keep_state_e(a, MA, e.col, send, rowgain);
        const bool keepGaA = valid && keep_state_e(a, GaA, e.col, send, rowgain);
        // G_b and M at B
        Key kAB = exk;
        uint32_t tAB = ext_tag;
        if (kA > kAB) {
            kAB = kA;
            tAB = yM0A;
        }
        int32_t GbB = kNeg;
        if (hasB && kAB > kNoKey) {
            const Key v = kAB + a.sg - absss * (Key)(e.col + 1) - skey;
            GbB = v > 0 ? (int32_t)v : kNeg;
        }
        int32_t MB = M0B;
        uint32_t yMB = yM0B;
        if (GbB > MB) {
            MB = GbB;
            yMB = tAB;
        }
        const bool keepMB = hasB && keep_state_e(a, MB, e.col + 1, send, rowgain);
        // G_b-only columns after this lane's last candidate, up to the next candidate
        Key kinc = kAB;
        uint32_t tinc = tAB;
        if (kB > kinc) {
            kinc = kB;
            tinc = yM0B;
        }
        const uint32_t lc = hasB ? e.col + 1 : e.col;
        const uint32_t stop = (ncol == kNone || ncol > send) ? send : ncol;
        uint32_t nspread = 0, nspread_hits = 0;
        if (valid && kinc > kNoKey) {
            for (uint32_t col = lc + 1; col < stop; ++col) {
                const Key v = kinc + a.sg - absss * (Key)col - skey;
                if (v <= 0 || !keep_state_e(a, (int32_t)v, col, send, rowgain)) break;
                ++nspread;
                nspread_hits += (v >= a.H);
            }
        }
        const uint32_t nA = (keepMA || keepGaA) ? 1u : 0u;
        const uint32_t nB = keepMB ? 1u : 0u;
        const uint32_t cnt_lane = nA + nB + nspread;
        uint32_t tot;
        const uint32_t pre = wave_excl_scan_u32(cnt_lane, &tot);
        uint32_t woff = 0;  // entries of the waves before this one
        if (W > 1) {
            if (lane == 0) xg->cnt[par][wave] = tot;
            __syncthreads();
            uint32_t all = 0;
#pragma unroll
            for (int w2 = 0; w2 < W; ++w2) {
                const uint32_t v = xg->cnt[par][w2];
                woff += w2 < wave ? v : 0u;
                all += v;
            }
            tot = all;
            par ^= 1;
        }
        if (out + tot <= o.cap) {
            uint32_t p = out + woff + pre;
            if (nA) {
                Entry w;
                w.col = e.col;
                w.M = keepMA ? MA : kNeg;
                w.Ga = keepGaA ? GaA : kNeg;
                w.yM = keepMA ? yMA : 0;
                w.yGa = keepGaA ? yGaA : 0;
                nxt.store(p++, w);
            }
            if (nB) {
                Entry w;
                w.col = e.col + 1;
                w.M = MB;
                w.Ga = kNeg;
                w.yM = yMB;
                w.yGa = 0;
                nxt.store(p++, w);
            }
            for (uint32_t s = 0; s < nspread; ++s) {
                const uint32_t col = lc + 1 + s;
                Entry w;
                w.col = col;
                w.M = (int32_t)(kinc + a.sg - absss * (Key)col - skey);
                w.Ga = kNeg;
                w.yM = tinc;
                w.yGa = 0;
                nxt.store(p++, w);
            }
        } else {
            overflow = true;
        }
        // hit records of this round's entries
        const uint32_t nh = !o.emit_hits ? 0u
                                         : (nA && keepMA && MA >= a.H ? 1u : 0u) + (nB && MB >= a.H ? 1u : 0u) +
                                               nspread_hits;
        uint32_t htot;
        const uint32_t hpre = wave_excl_scan_u32(nh, &htot);
        if (htot) {
            const uint32_t copies = o.rK + 1;
            const unsigned long long hall = (unsigned long long)htot * copies;
            hit_reserve(hr, hall, o.hkeys, o.hscores, o.hit_cap, o.hit_chunk, o.cnt);
            unsigned long long slot = hr.base + (unsigned long long)hpre * copies;
            auto put = [&](uint32_t col, int32_t M) {
                for (uint32_t r = 0; r < copies; ++r) {
                    if (slot < o.hit_cap) {
                        o.hkeys[slot] = ((uint64_t)(col + (r ? o.rdelta[r] : 0u)) << 32) | o.e_child;
                        o.hscores[slot] = (uint32_t)M;
                    }
                    ++slot;
                }
            };
            if (nA && keepMA && MA >= a.H) put(e.col, MA);
            if (nB && MB >= a.H) put(e.col + 1, MB);
            for (uint32_t s = 0; s < nspread; ++s) {
                const uint32_t col = lc + 1 + s;
                const int32_t v = (int32_t)(kinc + a.sg - absss * (Key)col - skey);
                if (v < a.H) break;
                put(col, v);
            }
            hr.base += hall;
            hr.left -= hall;
            hits += hall;
        }
        // cost classes of the entries of this round
        uint32_t c1 = nspread, c2 = 0, c3 = 0;
        if (nA) {
            const int in = (D > 0) + (GaA > 0) + (GbA > 0);
            if (in <= 1)
                ++c1;
            else if (in == 2)
                ++c2;
            else
                ++c3;
        }
        if (nB) {
            if (GbB > 0)
                ++c2;
            else
                ++c1;
        }
        diag += c1;  // per lane; the callers reduce over the wave
        gap2 += c2;
        gap3 += c3;
        // carries for the next round
        if (W == 1) {
            const int lastlane = (int)((len - base - 1) < 63u ? (len - base - 1) : 63u);
            c_pcol = (uint32_t)__builtin_amdgcn_readlane((int)e.col, lastlane);
            c_pM = __builtin_amdgcn_readlane(e.M, lastlane);
            c_pyM = (uint32_t)__builtin_amdgcn_readlane((int)e.yM, lastlane);
        }
        if (allk > c_key) {
            c_key = allk;
            c_tag = allt;
        }
        out += tot;
    }
    o.len = out;
    o.overflow = overflow;
    o.hits = hits;
    o.diag = diag;
    o.gap2 = gap2;
    o.gap3 = gap3;
}

}  // namespace alae
