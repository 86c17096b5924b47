// Device-side data formats and helpers of the search path (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "alae_internal.h"

namespace alae {

// "Dead" score for a state that does not exist (-infinity in Section 2.2).
// Far enough from INT32_MIN that adding a few penalties never wraps.
constexpr int32_t kNeg = -(1 << 29);

// A trie node of the frontier.  While the node has several occurrences it is
// the BWT row range [lo, hi] of its string (Section 5).  Once it has one
// occurrence, lo holds kUniqueBit | e, where e is the 0-based text position
// where that occurrence ends, and the subtree is walked along the text.
constexpr uint32_t kUniqueBit = 0x80000000u;
struct Node {
    uint32_t lo;
    uint32_t hi;
    uint32_t off;  // first entry of the row in the level's entry buffer
    uint32_t len;  // number of entries of the row
};
static_assert(sizeof(Node) == 16, "node record is 16 bytes");

// One live entry of a sparse DP row (Section 2.2): query column (0-based end),
// M_X and G_a at this column, and the start column y of the alignment that
// gives each of the two values (used by the domination test, Section 3.2).
struct Entry {
    uint32_t col;
    int32_t M;
    int32_t Ga;
    uint32_t yM;
    uint32_t yGa;
};
static_assert(sizeof(Entry) == 20, "entry record is 20 bytes");

// Everything a kernel needs about the index and the query.
struct SearchArgs {
    const uint8_t *occ;   // occurrence blocks
    const uint32_t *sa;   // text end of every BWT row
    const uint8_t *text;  // text codes
    const int8_t *prof;   // query profile: prof[c*m + j] = s(c, P[j])
    const int32_t *U;     // U[j]: largest total score the columns after j can add
    uint32_t n;
    uint32_t dollar_row;
    uint32_t m;
    int32_t sigma;
    int32_t sg;
    int32_t ss;
    int32_t H;
    int32_t smax;
    int32_t lmax;         // Equation 1
    int32_t use_score_filter;
    int32_t use_domination;
    int32_t dom_reach;    // longest left extension tried by the domination test
    int32_t u_closed;     // U(j) = smax * (m-1-j) (match/mismatch scoring)
    int32_t matrix_mode;  // substitution scores come from a matrix
    int32_t s_match;      // s_a (match/mismatch scoring)
    int32_t s_mismatch;   // s_b
    const uint8_t *query; // query codes; 64 readable bytes before index 0 and after m-1
    int32_t ngr_walk;     // walk no-gap chains in registers (else all go to the general walker)
    // Several queries searched together: their codes are concatenated and no
    // alignment may cross from one query into the next.
    int32_t multi;
    int32_t use_reuse;       // replay forks that are copies of one another (Section 4)
    const uint32_t *qord;    // per column: ordinal of its query
    const uint32_t *segbeg;  // per query: first column
    const uint32_t *segend;  // per query: one past its last column
    const uint32_t *colseg;  // per column: columns to the end of its query, kSegFirst on a query's first column
    const uint32_t *colbeg;  // per column: columns of its query before it
    uint32_t C[21];
    int32_t occ_packed;      // occ blocks are packed DNA (else one byte a character)
    int32_t has_sep;         // the text holds record separators
};

// Query segments (batched search).  Single-query searches never read the arrays.
// The hot questions (where does col's query end or begin, does it start at
// col) take one load; the prefix-max key offset goes through the query ordinal.
constexpr uint32_t kSegFirst = 0x80000000u;
__device__ inline uint32_t seg_info(const SearchArgs &a, uint32_t col) {
    return a.multi ? a.colseg[col] : a.m - col;
}
__device__ inline uint32_t seg_dist(uint32_t info) { return info & ~kSegFirst; }
__device__ inline uint32_t seg_end_of(const SearchArgs &a, uint32_t col) {
    return a.multi ? col + seg_dist(a.colseg[col]) : a.m;
}
// columns of col's query before col
__device__ inline uint32_t seg_off(const SearchArgs &a, uint32_t col) {
    return a.multi ? a.colbeg[col] : col;
}
// col is the first column of its query (nothing may enter it from the left)
__device__ inline bool seg_first(const SearchArgs &a, uint32_t col) {
    return a.multi && (a.colseg[col] & kSegFirst) != 0;
}
// Offset that makes prefix-max keys of earlier queries useless in later ones:
// within a query a key is M + |s_s|*col < 2^44, so the query ordinal shifted
// past that keeps every later query's keys above every earlier one's and the
// G_b value an earlier key gives in a later query negative.
constexpr int kSegShift = 44;
__device__ inline int64_t seg_key(const SearchArgs &a, uint32_t col) {
    return a.multi ? ((int64_t)a.qord[col] << kSegShift) : 0;
}

// Text and query buffers carry this many readable bytes before index 0 and
// after their last character, so fixed-size windows can be loaded without
// bounds checks (the bytes outside are never used as characters).
constexpr int kSlack = 64;

// occ(c, i) for the four DNA codes at once: counts of each code in BWT[0..i].
// i may be -1 (all zero).  One 64-byte block read.
__device__ inline void occ4_dna(const SearchArgs &a, int64_t i, uint32_t out[4]) {
    if (i < 0) {
        out[0] = out[1] = out[2] = out[3] = 0;
        return;
    }
    const uint64_t b = (uint64_t)i / kDnaBlockChars;
    const int k = (int)((uint64_t)i - b * kDnaBlockChars) + 1;  // chars of this block to count
    const uint4 *p = reinterpret_cast<const uint4 *>(a.occ + b * 64);
    uint4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
    const uint32_t w[12] = {q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
    uint32_t c1 = 0, c2 = 0, c3 = 0;
    const int full = k >> 4;
    const int rem = k & 15;
#pragma unroll
    for (int t = 0; t < 12; ++t) {
        uint32_t mask;
        if (t < full)
            mask = 0x55555555u;
        else if (t == full && rem)
            mask = 0x55555555u & ((1u << (2 * rem)) - 1u);
        else
            mask = 0u;
        const uint32_t lo = w[t] & mask;
        const uint32_t hi = (w[t] >> 1) & mask;
        c1 += __popc(lo & ~hi);
        c2 += __popc(hi & ~lo);
        c3 += __popc(lo & hi);
    }
    uint32_t c0 = (uint32_t)k - c1 - c2 - c3;
    const uint64_t bstart = b * kDnaBlockChars;
    if ((uint64_t)a.dollar_row >= bstart && (uint64_t)a.dollar_row <= (uint64_t)i) c0 -= 1;
    out[0] = q0.x + c0;
    out[1] = q0.y + c1;
    out[2] = q0.z + c2;
    out[3] = q0.w + c3;
}

// occ(c, i) for one code of a byte-per-character block (protein alphabet).
__device__ inline uint32_t occ1_gen(const SearchArgs &a, int c, int64_t i) {
    if (i < 0) return 0;
    const uint64_t b = (uint64_t)i / kGenBlockChars;
    const int k = (int)((uint64_t)i - b * kGenBlockChars) + 1;
    const uint32_t *blk = reinterpret_cast<const uint32_t *>(a.occ + b * 128);
    uint32_t cnt = blk[c];
    const uint32_t pat = 0x01010101u * (uint32_t)c;
#pragma unroll
    for (int t = 0; t < 12; ++t) {
        const int first = t * 4;
        if (first >= k) break;
        const uint32_t v = blk[20 + t] ^ pat;  // zero bytes where the char equals c
        uint32_t z = (v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
        z = ~(z | v | 0x7F7F7F7Fu);  // 0x80 in each zero byte
        const int take = k - first;
        if (take < 4) z &= (1u << (8 * take)) - 1u;
        cnt += __popc(z);
    }
    return cnt;
}

// ---------------------------------------------------------------------------
// Counters shared by the kernels of one search
// ---------------------------------------------------------------------------

// Device counters, each on its own 128-byte line: wave-level atomics on
// different counters then go to different L2 lines instead of queueing on one.
#define kCounter alignas(128) unsigned long long
struct Counters {
    kCounter nodes;     // child nodes allocated in the output level
    kCounter entries;   // entries allocated in the output level
    kCounter hits;      // hit records allocated in total
    kCounter overflow;  // bit 0 nodes, bit 1 entries, bit 2 hits
    // statistics
    kCounter st_nodes;
    kCounter st_entries;
    kCounter st_diag;
    kCounter st_gap2;
    kCounter st_gap3;
    kCounter st_dominated;
    kCounter st_emitted;
    kCounter bad_query;
    // random-access reads of the expansion kernel (64-byte granules)
    kCounter st_occ_reads;
    kCounter st_sa_reads;
    kCounter st_text_reads;
    // frontier bytes read and written by the expansion kernel
    kCounter st_frontier_bytes;
    // chains: nodes with a single occurrence, walked along the text
    kCounter cnodes;     // chain items allocated by the level kernel
    kCounter centries;   // their row entries
    kCounter chain_head; // next chain item to start (narrow chain kernel)
    kCounter wnodes;     // wide chain items (rows too wide for one lane)
    kCounter wentries;   // their row entries
    kCounter wide_head;  // next wide item to start (wide chain kernel)
    kCounter st_chain_steps;
    kCounter st_wide_steps;
    kCounter st_promoted;
    kCounter st_dominated_gapped;
    kCounter st_chain_bytes;  // row bytes moved by the chain kernels
    kCounter hit_padding;     // reserved hit slots left unused (padding keys)
    kCounter onodes;          // wide chains whose row outgrew the on-chip buffers
    kCounter oentries;
    kCounter overflow_head;
    kCounter lwnodes;         // next-level nodes with rows too long for a lane
    kCounter gnodes;          // chains with gaps, walked by the general lane kernel
    kCounter gentries;
    kCounter general_head;
    kCounter st_ngr_steps;    // chain steps taken in the no-gap fast path
    kCounter stage_need;      // longest row that did not fit a level-wide staging buffer
    kCounter st_reused;       // entries replayed from an identical fork instead of computed
    kCounter st_replay;       // chains recognised as copies of one fork
    kCounter gen_done;        // lane-walker waves that have finished
    kCounter gen_started;     // lane-walker waves that have begun (before their first claim)
    kCounter missed;          // wave-queue items a live consumer left for the next pass
    kCounter t_gen0, t_gen1;  // first start / last end of lane-walker waves (100 MHz clock)
    kCounter t_live0, t_live1;  // same for the live wave pass
    kCounter t_push0;         // first item published to the live pass
    kCounter st_wide_entries; // DP entries computed by the wave walkers
    kCounter st_wide_max;     // most rows one wave walker stepped through for one item
    kCounter st_wide_slow;    // slowest wave-walker item: ticks << 38 | start (µs into the pass) << 18 | rows
    kCounter st_qdom;         // seed states dropped by the q-gram domination table
    kCounter tasks;           // child tasks of the current level (node phase)
};

// State of a device-driven run of levels (the level loop on the device, a
// batch of level slots replayed from one captured graph).  k_level_step,
// between the slots, commits the level before (its frontier sizes and depth)
// and begins the next, or stops the batch; the level kernels read the sizes
// and the depth here and do nothing once `stop` is set.
enum : uint32_t { kStopNone = 0, kStopDone = 1, kStopSplit = 2, kStopOverflow = 3, kStopLarge = 4 };
// Device-driven levels take frontiers of at most this many nodes (their grids
// are sized for it; a larger level goes back to the host-driven loop, whose
// per-level round trip is small beside its kernels).
constexpr unsigned long long kDeviceFrontier = 1ull << 18;
struct LevelCtl {
    unsigned long long nn, nlw;   // nodes (lane rows, long rows) of the level being expanded
    unsigned long long peak;      // largest frontier seen (nodes of a level)
    unsigned long long split_below;  // the frontier's tail goes to the chain walkers at this size
    unsigned long long max_depth; // deepest level that made nodes or chains
    int32_t depth;                // depth of the frontier being expanded
    int32_t d1;                   // depth of its children
    int32_t lmax;
    uint32_t stop;                // kStop*: the batch's remaining slots do nothing
    uint32_t pending;             // a level was begun and not yet committed
    uint32_t ran;                 // levels committed by this batch
    Counters snap;                // the counters as the pending level found them (for a rerun)
};

// Key of an unused hit slot: sorts after every real (column, text end) key.
constexpr uint64_t kPadKey = ~0ull;

// overflow bits
constexpr unsigned long long kOvNodes = 1, kOvEntries = 2, kOvHits = 4, kOvChainNodes = 8, kOvChainEntries = 16,
                             kOvWideNodes = 32, kOvWideEntries = 64, kOvWideRow = 128, kOvSpillNodes = 256,
                             kOvSpillEntries = 512, kOvLevelWide = 1024, kOvGeneralNodes = 2048,
                             kOvGeneralEntries = 4096, kOvStageRow = 8192,
                             kOvTasks = 16384;

struct Caps {
    unsigned long long nodes;
    unsigned long long entries;
    unsigned long long hits;
    unsigned long long cnodes;
    unsigned long long centries;
    unsigned long long wnodes;
    unsigned long long wentries;
    unsigned long long wrow;  // entries per wide row buffer
    unsigned long long onodes;    // spill queue of rows too wide for on-chip buffers
    unsigned long long oentries;
    unsigned long long lwnodes;   // next-level nodes with long rows
    unsigned long long gnodes;    // general chain queue
    unsigned long long gentries;
    unsigned long long srow;      // entries per staging buffer of the level-wide kernel
    unsigned long long tasks;     // child tasks of one level
    unsigned long long hit_chunk; // hit slots a wave reserves at a time
};

struct SubTable {
    int8_t s[20 * 20];
};

__device__ inline int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
__device__ inline int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

}  // namespace alae
