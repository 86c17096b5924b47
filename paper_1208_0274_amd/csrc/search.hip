// Exact local-alignment search over the FM-index of the reversed text.
//
// Path of one search (Sections 2.2-5 of the paper):
//   1. query preparation: profile s(c, P[j]), the gain bound U(j), q (Eq. 2),
//      L_max (Eq. 1);
//   2. seeding at depth q_eff (Theorem 3): one trie node per q-gram of P that
//      occurs in T, its row holding the columns where the q-gram ends;
//      in matrix mode every depth-1 node with its positive columns;
//   3. level by level, every frontier node is extended by each character c
//      (backward search on the reversed text, Section 5 (3)); the child's
//      sparse row of M_X / G_a is computed from the parent's (Section 2.2),
//      keeping only entries that pass the zero floor (Theorem 2 (i)), the
//      score filter (Theorem 2 (ii)) and the length filter (Theorem 1); when a
//      node becomes unique its states are checked for domination
//      (Section 3.2); entries with M >= H are emitted for every occurrence
//      (Algorithm 1, lines 6-10);
//   4. the emitted records are sorted by (query end, text end) and merged,
//      keeping the largest score per pair (Algorithm 1, line 8-9).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "alae_internal.h"
#include "device_algos.h"
#include "device_common.h"

namespace alae {

// ---------------------------------------------------------------------------
// Device index upload
// ---------------------------------------------------------------------------

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
            return ALAE_E_DEVICE;                                                                \
        }                                                                                        \
    } while (0)

alae_status ensure_device(const alae_index *idx) {
    std::lock_guard<std::mutex> lock(idx->mu);
    if (idx->on_device) return ALAE_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        set_error("no HIP device is available");
        return ALAE_E_DEVICE;
    }
    if (idx->device < 0 || idx->device >= ndev) {
        set_error("device %d does not exist (%d devices)", idx->device, ndev);
        return ALAE_E_DEVICE;
    }
    HIP_TRY(hipSetDevice(idx->device));
    HIP_TRY(hipMalloc(&idx->d_text, idx->text.size() + 64));
    HIP_TRY(hipMalloc(&idx->d_sa, idx->sa_end.size() * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&idx->d_occ, idx->occ.size()));
    HIP_TRY(hipMemcpy(idx->d_text, idx->text.data(), idx->text.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(idx->d_sa, idx->sa_end.data(), idx->sa_end.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(idx->d_occ, idx->occ.data(), idx->occ.size(), hipMemcpyHostToDevice));
    idx->on_device = true;
    return ALAE_OK;
}

void release_device(const alae_index *idx) {
    std::lock_guard<std::mutex> lock(idx->mu);
    if (!idx->on_device) return;
    hipSetDevice(idx->device);
    hipFree(idx->d_text);
    hipFree(idx->d_sa);
    hipFree(idx->d_occ);
    idx->d_text = nullptr;
    idx->d_sa = nullptr;
    idx->d_occ = nullptr;
    idx->on_device = false;
}

// ---------------------------------------------------------------------------
// Counters shared by the kernels of one search
// ---------------------------------------------------------------------------

struct Counters {
    unsigned long long nodes;     // child nodes allocated in the output level
    unsigned long long entries;   // entries allocated in the output level
    unsigned long long hits;      // hit records allocated in total
    unsigned long long overflow;  // bit 0 nodes, bit 1 entries, bit 2 hits
    // statistics
    unsigned long long st_nodes;
    unsigned long long st_entries;
    unsigned long long st_diag;
    unsigned long long st_gap2;
    unsigned long long st_gap3;
    unsigned long long st_dominated;
    unsigned long long st_emitted;
    unsigned long long bad_query;
    // random-access reads of the expansion kernel (64-byte granules)
    unsigned long long st_occ_reads;
    unsigned long long st_sa_reads;
    unsigned long long st_text_reads;
    // frontier bytes read and written by the expansion kernel
    unsigned long long st_frontier_bytes;
};

struct Caps {
    unsigned long long nodes;
    unsigned long long entries;
    unsigned long long hits;
};

struct SubTable {
    int8_t s[20 * 20];
};

// ---------------------------------------------------------------------------
// Query preparation kernels
// ---------------------------------------------------------------------------

__global__ void k_check_query(const uint8_t *q, uint32_t m, int sigma, Counters *cnt) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m && q[j] >= sigma) atomicAdd(&cnt->bad_query, 1ull);
}

// prof[c*m + j] = s(c, P[j]); colrev[m-1-j] = max over c of s(c, P[j]).
__global__ void k_profile(const uint8_t *q, uint32_t m, int sigma, SubTable sub, int8_t *prof, uint32_t *colrev) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int pj = q[j];
    int best = -128;
    for (int c = 0; c < sigma; ++c) {
        int v = sub.s[c * sigma + pj];
        prof[(size_t)c * m + j] = (int8_t)v;
        best = v > best ? v : best;
    }
    colrev[m - 1 - j] = (uint32_t)(best > 0 ? best : 0);
}

// U[j] = sum over j' > j of colmax(P[j']) from the exclusive scan of colrev.
__global__ void k_gain_bound(const uint32_t *scan_rev, uint32_t m, int32_t *U) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) U[j] = (int32_t)scan_rev[m - 1 - j];
}

// Seed keys.  q-gram mode: key = code of P[j-q+1..j] (first char most
// significant), one per end column j >= q-1; other slots get the invalid key.
// Matrix mode: slot c*m + j holds key c when s(c, P[j]) > 0.
__global__ void k_seed_keys(const uint8_t *q, uint32_t m, int sigma, int qeff, int matrix_mode, SubTable sub,
                            uint64_t invalid, uint64_t *keys, uint32_t *vals) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!matrix_mode) {
        if (t >= m) return;
        uint32_t j = (uint32_t)t;
        uint64_t key = invalid;
        if ((int)j >= qeff - 1) {
            key = 0;
            for (int k = qeff - 1; k >= 0; --k) key = key * sigma + q[j - k];
        }
        keys[t] = key;
        vals[t] = j;
    } else {
        if (t >= (uint64_t)m * sigma) return;
        uint32_t c = (uint32_t)(t / m);
        uint32_t j = (uint32_t)(t % m);
        keys[t] = sub.s[c * sigma + q[j]] > 0 ? c : invalid;
        vals[t] = j;
    }
}

__device__ inline void backward_step(const SearchArgs &a, int c, int64_t &l, int64_t &r) {
    uint32_t ol, orr;
    if (a.sigma == 4) {
        uint32_t o1[4], o2[4];
        occ4_dna(a, l - 1, o1);
        occ4_dna(a, r, o2);
        ol = o1[c];
        orr = o2[c];
    } else {
        ol = occ1_gen(a, c, l - 1);
        orr = occ1_gen(a, c, r);
    }
    l = (int64_t)a.C[c] + ol;
    r = (int64_t)a.C[c] + orr - 1;
}

// Seed entries and nodes from the sorted (key, column) pairs.
__global__ void k_seed_nodes(SearchArgs a, const uint64_t *keys, const uint32_t *vals, uint64_t count,
                             uint64_t invalid, int qeff, int matrix_mode, int32_t seedM, Entry *ent, Node *nodes,
                             Counters *cnt) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t key = keys[i];
    if (key >= invalid) return;
    const uint32_t col = vals[i];
    Entry e;
    e.col = col;
    e.M = matrix_mode ? (int32_t)a.prof[(size_t)key * a.m + col] : seedM;
    e.Ga = kNeg;
    e.yM = col + 1 - (uint32_t)qeff;
    e.yGa = 0;
    ent[i] = e;
    if (i > 0 && keys[i - 1] == key) return;
    uint64_t end = i + 1;
    while (end < count && keys[end] == key) ++end;
    // backward search of the seed string, first character first
    int64_t l = 0, r = a.n;
    uint64_t code = key;
    int chars[32];
    for (int k = qeff - 1; k >= 0; --k) {
        chars[k] = (int)(code % (uint64_t)a.sigma);
        code /= (uint64_t)a.sigma;
    }
    for (int k = 0; k < qeff && l <= r; ++k) backward_step(a, chars[k], l, r);
    if (l > r) return;
    unsigned long long slot = atomicAdd(&cnt->nodes, 1ull);
    Node nd;
    nd.lo = (uint32_t)l;
    nd.hi = (uint32_t)r;
    nd.off = (uint32_t)i;
    nd.len = (uint32_t)(end - i);
    nodes[slot] = nd;
}

// Hits of the seed level (only when a seed entry already reaches H).
__global__ void k_seed_hits(SearchArgs a, const Node *nodes, uint32_t nn, const Entry *ent, Caps caps,
                            uint64_t *hkeys, uint32_t *hscores, Counters *cnt) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn) return;
    Node nd = nodes[t];
    for (uint32_t k = 0; k < nd.len; ++k) {
        Entry e = ent[nd.off + k];
        if (e.M < a.H) continue;
        for (uint64_t h = nd.lo; h <= nd.hi; ++h) {
            unsigned long long slot = atomicAdd(&cnt->hits, 1ull);
            if (slot >= caps.hits) {
                atomicOr(&cnt->overflow, 4ull);
                continue;
            }
            hkeys[slot] = ((uint64_t)e.col << 32) | a.sa[h];
            hscores[slot] = (uint32_t)e.M;
        }
        atomicAdd(&cnt->st_emitted, (unsigned long long)(nd.hi - nd.lo + 1));
    }
}

// ---------------------------------------------------------------------------
// Row update
// ---------------------------------------------------------------------------

// Section 3.2 (Theorem 4, case 2), tested locally: the state whose best
// alignment starts at text position x and query column y is dominated when
// an ungapped alignment ending at (x-1, y-1) scores above zero, because
// prepending it would beat that alignment at every cell it reaches.
__device__ inline bool dominated(const SearchArgs &a, int64_t x, int64_t y) {
    int64_t reach = a.dom_reach;
    if (x < reach) reach = x;
    if (y < reach) reach = y;
    int32_t sum = 0;
    for (int64_t k = 1; k <= reach; ++k) {
        sum += a.prof[(size_t)a.text[x - k] * a.m + (y - k)];
        if (sum > 0) return true;
        if (sum + a.smax * (int32_t)(reach - k) <= 0) return false;
    }
    return false;
}

struct RowSink {
    // output row (WRITE mode)
    Entry *out;
    uint64_t *hkeys;
    uint32_t *hscores;
    unsigned long long hit_base;
    unsigned long long hit_cap;
    // occurrences of the child
    bool unique;
    uint32_t e_end;  // unique: text end
    uint32_t lo, hi; // otherwise: BWT rows
    // results
    uint32_t n_entries;
    uint32_t n_hits;
    uint32_t st_diag, st_gap2, st_gap3, st_dom;
};

template <bool WRITE>
__device__ inline void emit_entry(const SearchArgs &a, RowSink &s, uint32_t col, int32_t M, int32_t Ga, uint32_t yM,
                                  uint32_t yGa, int inputs) {
    if (WRITE) {
        Entry e;
        e.col = col;
        e.M = M;
        e.Ga = Ga;
        e.yM = yM;
        e.yGa = yGa;
        s.out[s.n_entries] = e;
        if (inputs <= 1)
            s.st_diag++;
        else if (inputs == 2)
            s.st_gap2++;
        else
            s.st_gap3++;
    }
    s.n_entries++;
    if (M >= a.H) {
        if (s.unique) {
            if (WRITE) {
                unsigned long long slot = s.hit_base + s.n_hits;
                if (slot < s.hit_cap) {
                    s.hkeys[slot] = ((uint64_t)col << 32) | s.e_end;
                    s.hscores[slot] = (uint32_t)M;
                }
            }
            s.n_hits++;
        } else {
            for (uint32_t h = s.lo; h <= s.hi; ++h) {
                if (WRITE) {
                    unsigned long long slot = s.hit_base + s.n_hits;
                    if (slot < s.hit_cap) {
                        s.hkeys[slot] = ((uint64_t)col << 32) | a.sa[h];
                        s.hscores[slot] = (uint32_t)M;
                    }
                }
                s.n_hits++;
            }
        }
    }
}

// Filters applied to one state value at column `col` of a row at depth d1:
// zero floor (Theorem 2 (i)) and score filter (Theorem 2 (ii)) with the gain
// bound min(U(col), smax * (L_max - d1)).
__device__ inline bool keep_state(const SearchArgs &a, int32_t v, uint32_t col, int32_t rowgain) {
    if (v <= 0) return false;
    if (!a.use_score_filter) return true;
    int32_t g = a.U[col];
    if (rowgain < g) g = rowgain;
    return v + g >= a.H;
}

// Computes the row at depth d1 of the child reached with character c from the
// parent row prow[0..plen).  Candidate columns are the parent's columns (G_a:
// a text character against a gap) and the parent's columns + 1 (diagonal);
// G_b (a query character against a gap) runs left to right along the row,
// including through columns with no candidate.  `check_dom` applies the
// domination test with the occurrence starting at text position x.
template <bool WRITE>
__device__ void child_row(const SearchArgs &a, const Entry *prow, uint32_t plen, int c, int32_t d1, bool check_dom,
                          int64_t x, RowSink &s) {
    const int8_t *pc = a.prof + (size_t)c * a.m;
    const int32_t open = a.sg + a.ss;  // first gap character
    const int32_t ext = a.ss;
    const int32_t rowgain = a.smax * (a.lmax - d1);
    int64_t last = -1;       // last column already handled
    int32_t gnext = kNeg;    // G_b value for column last+1
    uint32_t gy = 0;         // its start column

    auto spread_to = [&](int64_t upto) {  // G_b-only columns last+1 .. upto
        while (last < upto) {
            if (gnext <= 0) {
                last = upto;
                gnext = kNeg;
                break;
            }
            const uint32_t col = (uint32_t)(last + 1);
            const int32_t v = gnext;
            if (keep_state(a, v, col, rowgain)) {
                bool dom = check_dom && dominated(a, x, gy);
                if (dom) {
                    s.st_dom++;
                } else {
                    emit_entry<WRITE>(a, s, col, v, kNeg, gy, 0, 1);
                }
            }
            last = col;
            gnext = v + ext;
        }
    };

    auto column = [&](uint32_t j, int32_t D, uint32_t yD, int32_t Gav, uint32_t yGav) {
        spread_to((int64_t)j - 1);
        const int32_t Gb = (last == (int64_t)j - 1) ? gnext : kNeg;
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
        const bool keepM = keep_state(a, M, j, rowgain);
        const bool keepGa = keep_state(a, Gav, j, rowgain);
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
        gnext = gn;
        gy = gny;
        bool liveM = keepM, liveGa = keepGa;
        if (check_dom) {
            if (liveM && dominated(a, x, yM)) {
                liveM = false;
                s.st_dom++;
            }
            if (liveGa && dominated(a, x, yGav)) {
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

    for (uint32_t k = 0; k < plen; ++k) {
        const Entry e = prow[k];
        const uint32_t j = e.col;
        // diagonal from the previous parent entry, if it sits in column j-1
        int32_t D = kNeg;
        uint32_t yD = 0;
        if (k > 0) {
            const Entry p = prow[k - 1];
            if (p.col + 1 == j && p.M > 0) {
                D = p.M + pc[j];
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
        column(j, D, yD, Gav, yGav);
        // diagonal into column j+1 when no parent entry sits there
        if (e.M > 0 && j + 1 < a.m && !(k + 1 < plen && prow[k + 1].col == j + 1)) {
            column(j + 1, e.M + pc[j + 1], e.yM, kNeg, 0);
        }
    }
    spread_to((int64_t)a.m - 1);
}

// ---------------------------------------------------------------------------
// Level expansion: one lane per frontier node
// ---------------------------------------------------------------------------

__device__ inline unsigned long long wave_excl_scan_u64(unsigned long long v, unsigned long long *total) {
    const int lane = threadIdx.x & 63;
    unsigned long long inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned long long o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

struct ChildIter {
    int64_t lo[20];
    int64_t hi[20];
};

template <bool WRITE>
__device__ void expand_node(const SearchArgs &a, const Node &nd, const Entry *prow, int32_t d1, uint32_t &nodes_out,
                            uint32_t &entries_out, uint32_t &hits_out, Node *onodes, Entry *oent,
                            uint64_t *hkeys, uint32_t *hscores, unsigned long long node_base,
                            unsigned long long ent_base, unsigned long long hit_base, Caps caps,
                            uint32_t st[7]) {
    nodes_out = entries_out = hits_out = 0;
    const bool parent_unique = (nd.lo & kUniqueBit) != 0;
    uint32_t o_lo[4] = {0, 0, 0, 0}, o_hi[4] = {0, 0, 0, 0};
    if (!parent_unique) {
        if (a.sigma == 4) {
            occ4_dna(a, (int64_t)nd.lo - 1, o_lo);
            occ4_dna(a, (int64_t)nd.hi, o_hi);
        }
        const int bc = a.sigma == 4 ? kDnaBlockChars : kGenBlockChars;
        const int64_t b0 = nd.lo == 0 ? -1 : ((int64_t)nd.lo - 1) / bc;
        const int64_t b1 = (int64_t)nd.hi / bc;
        st[4] += (b0 >= 0 && b0 != b1) ? 2u : 1u;
    } else {
        st[6] += 1;  // the next text character
    }
    for (int c = 0; c < a.sigma; ++c) {
        RowSink s;
        int64_t x = 0;
        bool check = false;
        if (parent_unique) {
            const uint32_t e = nd.lo & ~kUniqueBit;
            if ((uint64_t)e + 1 >= a.n || a.text[e + 1] != c) continue;
            s.unique = true;
            s.e_end = e + 1;
            s.lo = s.hi = 0;
        } else {
            int64_t l, r;
            if (a.sigma == 4) {
                l = (int64_t)a.C[c] + o_lo[c];
                r = (int64_t)a.C[c] + o_hi[c] - 1;
            } else {
                l = (int64_t)a.C[c] + occ1_gen(a, c, (int64_t)nd.lo - 1);
                r = (int64_t)a.C[c] + occ1_gen(a, c, (int64_t)nd.hi) - 1;
            }
            if (l > r) continue;
            if (l == r) {
                s.unique = true;
                s.e_end = a.sa[l];
                st[5] += 1;
                check = a.use_domination != 0;
            } else {
                s.unique = false;
                s.lo = (uint32_t)l;
                s.hi = (uint32_t)r;
            }
        }
        if (check) x = (int64_t)s.e_end - d1 + 1;
        s.out = oent + ent_base + entries_out;
        s.hkeys = hkeys;
        s.hscores = hscores;
        s.hit_base = hit_base + hits_out;
        s.hit_cap = caps.hits;
        s.n_entries = s.n_hits = 0;
        s.st_diag = s.st_gap2 = s.st_gap3 = s.st_dom = 0;
        child_row<WRITE>(a, prow, nd.len, c, d1, check, x, s);
        if (s.n_entries > 0) {
            if (WRITE) {
                Node cn;
                if (s.unique) {
                    cn.lo = kUniqueBit | s.e_end;
                    cn.hi = 0;
                } else {
                    cn.lo = s.lo;
                    cn.hi = s.hi;
                }
                cn.off = (uint32_t)(ent_base + entries_out);
                cn.len = s.n_entries;
                onodes[node_base + nodes_out] = cn;
            }
            nodes_out++;
        }
        entries_out += s.n_entries;
        hits_out += s.n_hits;
        st[0] += s.st_diag;
        st[1] += s.st_gap2;
        st[2] += s.st_gap3;
        st[3] += s.st_dom;
    }
}

__global__ void __launch_bounds__(256) k_expand_level(SearchArgs a, const Node *nodes, uint32_t nn, const Entry *ent,
                                                      int32_t d1, Node *onodes, Entry *oent, uint64_t *hkeys,
                                                      uint32_t *hscores, Caps caps, Counters *cnt) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = t < nn;
    Node nd;
    nd.lo = nd.hi = nd.off = nd.len = 0;
    if (active) nd = nodes[t];
    uint32_t n_nodes = 0, n_ent = 0, n_hits = 0;
    uint32_t st[7] = {0, 0, 0, 0, 0, 0, 0};
    if (active) {
        expand_node<false>(a, nd, ent + nd.off, d1, n_nodes, n_ent, n_hits, nullptr, nullptr, nullptr, nullptr, 0,
                           0, 0, caps, st);
    }
    // allocate this wave's output with one atomic per counter
    unsigned long long tot_nodes, tot_ent, tot_hits;
    unsigned long long pre_nodes = wave_excl_scan_u64(n_nodes, &tot_nodes);
    unsigned long long pre_ent = wave_excl_scan_u64(n_ent, &tot_ent);
    unsigned long long pre_hits = wave_excl_scan_u64(n_hits, &tot_hits);
    const int lane = threadIdx.x & 63;
    unsigned long long b_nodes = 0, b_ent = 0, b_hits = 0;
    if (lane == 0) {
        if (tot_nodes) b_nodes = atomicAdd(&cnt->nodes, tot_nodes);
        if (tot_ent) b_ent = atomicAdd(&cnt->entries, tot_ent);
        if (tot_hits) b_hits = atomicAdd(&cnt->hits, tot_hits);
    }
    b_nodes = __shfl(b_nodes, 0, 64);
    b_ent = __shfl(b_ent, 0, 64);
    b_hits = __shfl(b_hits, 0, 64);
    bool fits = true;
    if (lane == 0) {
        unsigned long long of = 0;
        if (b_nodes + tot_nodes > caps.nodes) of |= 1ull;
        if (b_ent + tot_ent > caps.entries) of |= 2ull;
        if (b_hits + tot_hits > caps.hits) of |= 4ull;
        if (of) atomicOr(&cnt->overflow, of);
    }
    if (b_nodes + tot_nodes > caps.nodes || b_ent + tot_ent > caps.entries) fits = false;
    uint32_t st2[7] = {0, 0, 0, 0, 0, 0, 0};
    if (active && fits && n_nodes > 0) {
        uint32_t w_nodes, w_ent, w_hits;
        expand_node<true>(a, nd, ent + nd.off, d1, w_nodes, w_ent, w_hits, onodes, oent, hkeys, hscores,
                          b_nodes + pre_nodes, b_ent + pre_ent, b_hits + pre_hits, caps, st2);
    }
    unsigned long long s_nodes = wave_sum_u64(active ? 1 : 0);
    unsigned long long s_ent = wave_sum_u64(n_ent);
    unsigned long long s_diag = wave_sum_u64(st2[0]);
    unsigned long long s_g2 = wave_sum_u64(st2[1]);
    unsigned long long s_g3 = wave_sum_u64(st2[2]);
    unsigned long long s_dom = wave_sum_u64(st[3]);
    unsigned long long s_occ = wave_sum_u64(st[4]);
    unsigned long long s_sa = wave_sum_u64(st[5]);
    unsigned long long s_txt = wave_sum_u64(st[6]);
    unsigned long long s_in = wave_sum_u64(active ? (unsigned long long)(sizeof(Node) + nd.len * sizeof(Entry)) : 0ull);
    if (lane == 0) {
        if (s_occ) atomicAdd(&cnt->st_occ_reads, s_occ);
        if (s_sa) atomicAdd(&cnt->st_sa_reads, s_sa);
        if (s_txt) atomicAdd(&cnt->st_text_reads, s_txt);
        atomicAdd(&cnt->st_frontier_bytes,
                  s_in + tot_nodes * sizeof(Node) + tot_ent * sizeof(Entry) + tot_hits * 12ull);
        if (s_nodes) atomicAdd(&cnt->st_nodes, s_nodes);
        if (s_ent) atomicAdd(&cnt->st_entries, s_ent);
        if (s_diag) atomicAdd(&cnt->st_diag, s_diag);
        if (s_g2) atomicAdd(&cnt->st_gap2, s_g2);
        if (s_g3) atomicAdd(&cnt->st_gap3, s_g3);
        if (s_dom) atomicAdd(&cnt->st_dominated, s_dom);
        if (tot_hits) atomicAdd(&cnt->st_emitted, tot_hits);
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

template <typename T>
static alae_status grow(T *&ptr, uint64_t &cap, uint64_t need, bool keep, uint64_t keep_count, hipStream_t s) {
    if (need <= cap && ptr) return ALAE_OK;
    uint64_t ncap = cap ? cap : 1024;
    while (ncap < need) ncap *= 2;
    T *np = nullptr;
    hipError_t e = hipMalloc(&np, ncap * sizeof(T));
    if (e != hipSuccess) {
        hipGetLastError();
        set_error("device allocation of %llu bytes failed: %s", (unsigned long long)(ncap * sizeof(T)),
                  hipGetErrorString(e));
        return ALAE_E_NOMEM;
    }
    if (keep && ptr && keep_count) {
        e = hipMemcpyAsync(np, ptr, keep_count * sizeof(T), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            set_error("device copy failed: %s", hipGetErrorString(e));
            hipFree(np);
            return ALAE_E_DEVICE;
        }
        hipStreamSynchronize(s);
    }
    if (ptr) hipFree(ptr);
    ptr = np;
    cap = ncap;
    return ALAE_OK;
}

// Grow a (uint64 key, uint32 value) buffer pair together; keep_count records survive.
static alae_status grow_pair(uint64_t *&keys, uint32_t *&vals, uint64_t &cap, uint64_t need, uint64_t keep_count,
                             hipStream_t s) {
    if (need <= cap && keys && vals) return ALAE_OK;
    uint64_t kc = cap, vc = cap;
    if (!vals) vc = 0;
    if (!keys) kc = 0;
    alae_status st = grow(keys, kc, need, keep_count > 0, keep_count, s);
    if (st != ALAE_OK) return st;
    st = grow(vals, vc, kc, keep_count > 0, keep_count, s);
    if (st != ALAE_OK) return st;
    cap = std::min(kc, vc);
    return ALAE_OK;
}

}  // namespace alae

using namespace alae;

struct alae_workspace {
    const alae_index *idx = nullptr;
    int device = 0;
    // frontier levels (ping-pong)
    Node *nodes[2] = {nullptr, nullptr};
    uint64_t node_cap[2] = {0, 0};
    Entry *ents[2] = {nullptr, nullptr};
    uint64_t ent_cap[2] = {0, 0};
    // emitted hits and sort ping-pong
    uint64_t *hkeys = nullptr;
    uint32_t *hscores = nullptr;
    uint64_t hit_cap = 0;
    uint64_t *hkeys_alt = nullptr;
    uint32_t *hscores_alt = nullptr;
    uint64_t alt_cap = 0;
    uint32_t *scratch = nullptr;
    uint64_t scratch_cap = 0;
    uint32_t *flags = nullptr;
    uint64_t flags_cap = 0;
    uint32_t *pos = nullptr;
    uint64_t pos_cap = 0;
    // result
    uint64_t *res_keys = nullptr;
    uint32_t *res_scores = nullptr;
    uint64_t res_cap = 0;
    uint64_t res_count = 0;
    // query
    uint8_t *d_query = nullptr;
    uint64_t q_cap = 0;
    int8_t *prof = nullptr;
    uint64_t prof_cap = 0;
    int32_t *U = nullptr;
    uint64_t U_cap = 0;
    uint32_t *colrev = nullptr;
    uint64_t colrev_cap = 0;
    uint64_t *seed_keys = nullptr;
    uint32_t *seed_vals = nullptr;
    uint64_t seed_cap = 0;
    uint64_t *seed_keys_alt = nullptr;
    uint32_t *seed_vals_alt = nullptr;
    uint64_t seed_alt_cap = 0;
    // counters
    Counters *d_cnt = nullptr;
    Counters *h_cnt = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evk0 = nullptr, evk1 = nullptr;  // around each expansion launch
};

namespace alae {

static void ws_release(alae_workspace *ws) {
    hipSetDevice(ws->device);
    for (int i = 0; i < 2; ++i) {
        hipFree(ws->nodes[i]);
        hipFree(ws->ents[i]);
    }
    hipFree(ws->hkeys);
    hipFree(ws->hscores);
    hipFree(ws->hkeys_alt);
    hipFree(ws->hscores_alt);
    hipFree(ws->scratch);
    hipFree(ws->flags);
    hipFree(ws->pos);
    hipFree(ws->res_keys);
    hipFree(ws->res_scores);
    hipFree(ws->d_query);
    hipFree(ws->prof);
    hipFree(ws->U);
    hipFree(ws->colrev);
    hipFree(ws->seed_keys);
    hipFree(ws->seed_vals);
    hipFree(ws->seed_keys_alt);
    hipFree(ws->seed_vals_alt);
    hipFree(ws->d_cnt);
    if (ws->h_cnt) hipHostFree(ws->h_cnt);
    if (ws->ev0) hipEventDestroy(ws->ev0);
    if (ws->ev1) hipEventDestroy(ws->ev1);
    if (ws->evk0) hipEventDestroy(ws->evk0);
    if (ws->evk1) hipEventDestroy(ws->evk1);
}

struct Scheme {
    int sigma;
    int8_t sub[400];
    int smax;
    int matrix_mode;
    int sa;
};

static alae_status check_scoring(const alae_scoring *sc, int sigma, int32_t H, Scheme &out) {
    if (!sc) {
        set_error("scoring is NULL");
        return ALAE_E_ARG;
    }
    if (sc->ss >= 0 || sc->sg > 0) {
        set_error("gap scores must satisfy sg <= 0 and ss < 0 (got sg=%d ss=%d)", sc->sg, sc->ss);
        return ALAE_E_SCORING;
    }
    if (sc->sg < -1000000 || sc->ss < -1000000) {
        set_error("gap scores below -1e6 are not supported");
        return ALAE_E_SCORING;
    }
    if (H < 1) {
        set_error("H must be at least 1 (the zero floor makes every score >= 0)");
        return ALAE_E_SCORING;
    }
    out.sigma = sigma;
    out.matrix_mode = sc->use_matrix ? 1 : 0;
    if (!sc->use_matrix) {
        if (sc->sa <= 0 || sc->sb >= 0 || sc->sa > 127 || sc->sb < -128) {
            set_error("match/mismatch scoring needs 0 < sa <= 127 and -128 <= sb < 0 (got %d, %d)", sc->sa, sc->sb);
            return ALAE_E_SCORING;
        }
        for (int x = 0; x < sigma; ++x)
            for (int y = 0; y < sigma; ++y) out.sub[x * sigma + y] = (int8_t)(x == y ? sc->sa : sc->sb);
        out.smax = sc->sa;
        out.sa = sc->sa;
    } else {
        if (!sc->matrix) {
            set_error("use_matrix set but matrix is NULL");
            return ALAE_E_ARG;
        }
        int smax = -128;
        for (int x = 0; x < sigma; ++x) {
            if (sc->matrix[x * sigma + x] <= 0) {
                set_error("substitution matrix needs a positive diagonal");
                return ALAE_E_SCORING;
            }
            for (int y = 0; y < sigma; ++y) {
                if (sc->matrix[x * sigma + y] != sc->matrix[y * sigma + x]) {
                    set_error("substitution matrix must be symmetric");
                    return ALAE_E_SCORING;
                }
                out.sub[x * sigma + y] = sc->matrix[x * sigma + y];
                smax = std::max<int>(smax, sc->matrix[x * sigma + y]);
            }
        }
        out.smax = smax;
        out.sa = smax;
    }
    return ALAE_OK;
}

// Equation 1 (Theorem 1) with the largest substitution score in place of s_a.
static int64_t lmax_of(int64_t m, int64_t smax, int64_t sg, int64_t ss, int64_t H) {
    int64_t num = H - (smax * m + sg);
    int64_t q = num / ss;
    if ((num % ss != 0) && ((num < 0) != (ss < 0))) q -= 1;
    return std::max<int64_t>(m, m + q);
}

static int bit_length(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

static alae_status run_search(alae_workspace *ws, const uint8_t *d_query, uint64_t m, const alae_scoring *scoring,
                              int32_t H, const alae_search_opts *opts, hipStream_t s, uint64_t *hit_count) {
    const alae_index *idx = ws->idx;
    Scheme sch;
    alae_status st = check_scoring(scoring, idx->sigma, H, sch);
    if (st != ALAE_OK) return st;
    if (m == 0) {
        set_error("empty query");
        return ALAE_E_ARG;
    }
    if (m >= 0x7FFFFFFFull) {
        set_error("query of %llu characters is too long", (unsigned long long)m);
        return ALAE_E_TOO_LONG;
    }
    const int sigma = idx->sigma;
    const bool use_score_filter = opts ? opts->use_score_filter != 0 : true;
    const bool use_dom = opts ? opts->use_domination != 0 : true;
    const bool use_q = opts ? opts->use_qprefix != 0 : true;
    const int64_t lmax = lmax_of((int64_t)m, sch.smax, scoring->sg, scoring->ss, H);
    if ((int64_t)sch.smax * (lmax + 2) > (1ll << 28)) {
        set_error("scores could exceed the 32-bit range of the kernels (m too long for this scheme)");
        return ALAE_E_TOO_LONG;
    }
    // Equation 2 and the reading q_eff = min(q, ceil(H / s_a)).
    int qeff = 1;
    bool matrix_seeds = sch.matrix_mode || !use_q;
    if (!matrix_seeds) {
        const int q = std::min<int>(-scoring->sb, -(scoring->sg + scoring->ss)) / sch.sa + 1;
        const int hq = (H + sch.sa - 1) / sch.sa;
        qeff = std::max(1, std::min(q, hq));
        // keep the seed key inside 64 bits and the seed table small
        uint64_t space = 1;
        int fit = 0;
        while (fit < qeff && space * (uint64_t)sigma < (1ull << 40)) {
            space *= (uint64_t)sigma;
            ++fit;
        }
        qeff = fit;
        if (qeff < 1) qeff = 1;
    }
    if (qeff == 1 && !sch.matrix_mode) matrix_seeds = true;  // depth-1 seeds are the same in both modes

    // ---- buffers for the query ------------------------------------------------
    if ((st = grow(ws->prof, ws->prof_cap, (uint64_t)sigma * m, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->U, ws->U_cap, m, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->colrev, ws->colrev_cap, m + 1, false, 0, s)) != ALAE_OK) return st;
    const uint64_t nseed = matrix_seeds ? (uint64_t)sigma * m : m;
    if ((st = grow_pair(ws->seed_keys, ws->seed_vals, ws->seed_cap, nseed, 0, s)) != ALAE_OK) return st;
    if ((st = grow_pair(ws->seed_keys_alt, ws->seed_vals_alt, ws->seed_alt_cap, nseed, 0, s)) != ALAE_OK) return st;

    SearchArgs a;
    memset(&a, 0, sizeof(a));
    a.occ = idx->d_occ;
    a.sa = idx->d_sa;
    a.text = idx->d_text;
    a.prof = ws->prof;
    a.U = ws->U;
    a.n = (uint32_t)idx->n;
    a.dollar_row = (uint32_t)idx->dollar_row;
    a.m = (uint32_t)m;
    a.sigma = sigma;
    a.sg = scoring->sg;
    a.ss = scoring->ss;
    a.H = H;
    a.smax = sch.smax;
    a.lmax = (int32_t)lmax;
    a.use_score_filter = use_score_filter ? 1 : 0;
    a.use_domination = use_dom ? 1 : 0;
    a.dom_reach = 32;
    for (int c = 0; c <= sigma; ++c) a.C[c] = (uint32_t)idx->C[c];

    SubTable sub;
    memset(&sub, 0, sizeof(sub));
    memcpy(sub.s, sch.sub, (size_t)sigma * sigma);

    HIP_TRY(hipMemsetAsync(ws->d_cnt, 0, sizeof(Counters), s));
    const uint32_t tb = 256;
    const uint32_t gm = (uint32_t)((m + tb - 1) / tb);
    k_check_query<<<gm, tb, 0, s>>>(d_query, (uint32_t)m, sigma, ws->d_cnt);
    k_profile<<<gm, tb, 0, s>>>(d_query, (uint32_t)m, sigma, sub, ws->prof, ws->colrev);
    // scratch for scans/sorts, sized for the largest user below
    {
        uint64_t need = std::max<uint64_t>(scan_scratch_words(m + 1), radix_scratch_words(nseed));
        if ((st = grow(ws->scratch, ws->scratch_cap, need, false, 0, s)) != ALAE_OK) return st;
    }
    HIP_TRY(scan_exclusive_u32(ws->colrev, ws->colrev, m, ws->scratch, s));
    k_gain_bound<<<gm, tb, 0, s>>>(ws->colrev, (uint32_t)m, ws->U);

    // ---- seeds ---------------------------------------------------------------
    uint64_t space = 1;
    for (int k = 0; k < (matrix_seeds ? 1 : qeff); ++k) space *= (uint64_t)sigma;
    const uint64_t invalid = space;  // keys >= invalid are not seeds
    const int seed_depth = matrix_seeds ? 1 : qeff;
    k_seed_keys<<<(uint32_t)((nseed + tb - 1) / tb), tb, 0, s>>>(d_query, (uint32_t)m, sigma, seed_depth,
                                                                  matrix_seeds ? 1 : 0, sub, invalid, ws->seed_keys,
                                                                  ws->seed_vals);
    bool alt = false;
    HIP_TRY(radix_sort_pairs(ws->seed_keys, ws->seed_vals, ws->seed_keys_alt, ws->seed_vals_alt, nseed,
                             bit_length(invalid), ws->scratch, &alt, s));
    const uint64_t *sk = alt ? ws->seed_keys_alt : ws->seed_keys;
    const uint32_t *sv = alt ? ws->seed_vals_alt : ws->seed_vals;

    // level buffers: seeds need nseed entries and at most nseed nodes
    uint64_t ent_want = std::max<uint64_t>(opts && opts->entry_capacity ? opts->entry_capacity : (1ull << 22), nseed);
    for (int i = 0; i < 2; ++i) {
        if ((st = grow(ws->ents[i], ws->ent_cap[i], ent_want, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->nodes[i], ws->node_cap[i], std::max<uint64_t>(nseed, 1ull << 20), false, 0, s)) != ALAE_OK)
            return st;
    }
    uint64_t hit_want = opts && opts->hit_capacity ? opts->hit_capacity : (1ull << 20);
    if ((st = grow_pair(ws->hkeys, ws->hscores, ws->hit_cap, hit_want, 0, s)) != ALAE_OK) return st;

    const int32_t seedM = matrix_seeds ? 0 : qeff * sch.sa;
    k_seed_nodes<<<(uint32_t)((nseed + tb - 1) / tb), tb, 0, s>>>(a, sk, sv, nseed, invalid, seed_depth,
                                                                   matrix_seeds ? 1 : 0, seedM, ws->ents[0],
                                                                   ws->nodes[0], ws->d_cnt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ws->h_cnt->bad_query) {
        set_error("query holds codes outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    uint64_t nn = ws->h_cnt->nodes;
    int cur = 0;

    Caps caps;
    caps.hits = ws->hit_cap;
    // seed-level hits (only when a seed score reaches H)
    int32_t seed_best = matrix_seeds ? sch.smax : seedM;
    if (seed_best >= H && nn > 0) {
        for (;;) {
            caps.hits = ws->hit_cap;
            k_seed_hits<<<(uint32_t)((nn + tb - 1) / tb), tb, 0, s>>>(a, ws->nodes[cur], (uint32_t)nn, ws->ents[cur],
                                                                     caps, ws->hkeys, ws->hscores, ws->d_cnt);
            HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (!(ws->h_cnt->overflow & 4ull)) break;
            if ((st = grow_pair(ws->hkeys, ws->hscores, ws->hit_cap, ws->h_cnt->hits, 0, s)) != ALAE_OK) return st;
            Counters z = *ws->h_cnt;
            z.hits = 0;
            z.overflow = 0;
            z.st_emitted = 0;
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }

    uint64_t levels = 0, retries = 0, max_depth = nn ? (uint64_t)seed_depth : 0;
    uint64_t launches = 0;
    double expand_ms = 0.0;
    int32_t depth = seed_depth;
    while (nn > 0 && depth < lmax) {
        const int32_t d1 = depth + 1;
        const int nxt = cur ^ 1;
        // reset the per-level allocation counters; keep hits and statistics
        Counters before = *ws->h_cnt;
        for (;;) {
            Counters z = before;
            z.nodes = 0;
            z.entries = 0;
            z.overflow = 0;
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
            caps.nodes = ws->node_cap[nxt];
            caps.entries = ws->ent_cap[nxt];
            caps.hits = ws->hit_cap;
            HIP_TRY(hipEventRecord(ws->evk0, s));
            k_expand_level<<<(uint32_t)((nn + tb - 1) / tb), tb, 0, s>>>(a, ws->nodes[cur], (uint32_t)nn,
                                                                        ws->ents[cur], d1, ws->nodes[nxt],
                                                                        ws->ents[nxt], ws->hkeys, ws->hscores, caps,
                                                                        ws->d_cnt);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipEventRecord(ws->evk1, s));
            HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            {
                float kms = 0.f;
                HIP_TRY(hipEventElapsedTime(&kms, ws->evk0, ws->evk1));
                expand_ms += kms;
                ++launches;
            }
            const Counters &c = *ws->h_cnt;
            if (!c.overflow) break;
            ++retries;
            if (c.overflow & 1ull)
                if ((st = grow(ws->nodes[nxt], ws->node_cap[nxt], c.nodes, false, 0, s)) != ALAE_OK) return st;
            if (c.overflow & 2ull)
                if ((st = grow(ws->ents[nxt], ws->ent_cap[nxt], c.entries, false, 0, s)) != ALAE_OK) return st;
            if (c.overflow & 4ull)
                if ((st = grow_pair(ws->hkeys, ws->hscores, ws->hit_cap, c.hits, before.hits, s)) != ALAE_OK)
                    return st;
        }
        nn = ws->h_cnt->nodes;
        cur = nxt;
        depth = d1;
        ++levels;
        if (nn) max_depth = (uint64_t)d1;
    }

    // ---- max-merge and sort --------------------------------------------------
    const uint64_t emitted = ws->h_cnt->hits;
    uint64_t unique = 0;
    float merge_ms = 0.f;
    HIP_TRY(hipEventRecord(ws->evk0, s));
    if (emitted > 0) {
        if ((st = grow_pair(ws->hkeys_alt, ws->hscores_alt, ws->alt_cap, emitted, 0, s)) != ALAE_OK) return st;
        uint64_t need = std::max(radix_scratch_words(emitted), scan_scratch_words(emitted + 1));
        if ((st = grow(ws->scratch, ws->scratch_cap, need, false, 0, s)) != ALAE_OK) return st;
        const int bits = 32 + std::max(1, bit_length(m - 1));
        bool in_alt = false;
        HIP_TRY(radix_sort_pairs(ws->hkeys, ws->hscores, ws->hkeys_alt, ws->hscores_alt, emitted, bits, ws->scratch,
                                 &in_alt, s));
        const uint64_t *k = in_alt ? ws->hkeys_alt : ws->hkeys;
        const uint32_t *v = in_alt ? ws->hscores_alt : ws->hscores;
        if ((st = grow(ws->flags, ws->flags_cap, emitted + 1, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->pos, ws->pos_cap, emitted + 1, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow_pair(ws->res_keys, ws->res_scores, ws->res_cap, emitted, 0, s)) != ALAE_OK) return st;
        HIP_TRY(max_merge_sorted(k, v, emitted, ws->res_keys, ws->res_scores, ws->flags, ws->pos, ws->scratch, s));
        uint32_t cnt32 = 0;
        HIP_TRY(hipEventRecord(ws->evk1, s));
        HIP_TRY(hipMemcpyAsync(&cnt32, ws->pos + emitted, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipEventElapsedTime(&merge_ms, ws->evk0, ws->evk1));
        unique = cnt32;
    }
    ws->res_count = unique;
    *hit_count = unique;
    if (opts && opts->stats) {
        alae_stats *o = opts->stats;
        const Counters &c = *ws->h_cnt;
        o->nodes = c.st_nodes;
        o->entries = c.st_entries;
        o->entries_diag = c.st_diag;
        o->entries_gap2 = c.st_gap2;
        o->entries_gap3 = c.st_gap3;
        o->dominated = c.st_dominated;
        o->emitted = emitted;
        o->hits = unique;
        o->levels = levels;
        o->retries = retries;
        o->max_depth = max_depth;
        o->occ_reads = c.st_occ_reads;
        o->sa_reads = c.st_sa_reads;
        o->text_reads = c.st_text_reads;
        o->frontier_bytes = c.st_frontier_bytes;
        o->expand_launches = launches;
        o->expand_ms = expand_ms;
        o->merge_ms = merge_ms;
    }
    return ALAE_OK;
}

}  // namespace alae

extern "C" {

alae_status alae_workspace_create(const alae_index *index, alae_workspace **out) {
    if (!index || !out) {
        set_error("alae_workspace_create: null argument");
        return ALAE_E_ARG;
    }
    alae_status st = ensure_device(index);
    if (st != ALAE_OK) return st;
    std::unique_ptr<alae_workspace> ws(new (std::nothrow) alae_workspace());
    if (!ws) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    ws->idx = index;
    ws->device = index->device;
    HIP_TRY(hipSetDevice(ws->device));
    HIP_TRY(hipMalloc(&ws->d_cnt, sizeof(Counters)));
    HIP_TRY(hipHostMalloc(&ws->h_cnt, sizeof(Counters), hipHostMallocDefault));
    HIP_TRY(hipEventCreate(&ws->ev0));
    HIP_TRY(hipEventCreate(&ws->ev1));
    HIP_TRY(hipEventCreate(&ws->evk0));
    HIP_TRY(hipEventCreate(&ws->evk1));
    *out = ws.release();
    return ALAE_OK;
}

void alae_workspace_free(alae_workspace *ws) {
    if (!ws) return;
    ws_release(ws);
    delete ws;
}

alae_status alae_search_device(alae_workspace *ws, const uint8_t *d_query_codes, size_t m,
                               const alae_scoring *scoring, int32_t H, const alae_search_opts *opts, void *stream,
                               size_t *hit_count) {
    if (!ws || !d_query_codes || !hit_count) {
        set_error("alae_search_device: null argument");
        return ALAE_E_ARG;
    }
    HIP_TRY(hipSetDevice(ws->device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(ws->ev0, s));
    uint64_t cnt = 0;
    alae_status st = run_search(ws, d_query_codes, m, scoring, H, opts, s, &cnt);
    if (st != ALAE_OK) return st;
    HIP_TRY(hipEventRecord(ws->ev1, s));
    HIP_TRY(hipEventSynchronize(ws->ev1));
    if (opts && opts->stats) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ws->ev0, ws->ev1);
        opts->stats->device_ms = ms;
    }
    *hit_count = (size_t)cnt;
    return ALAE_OK;
}

alae_status alae_workspace_result(const alae_workspace *ws, const uint64_t **d_keys, const int32_t **d_scores,
                                  size_t *count) {
    if (!ws || !d_keys || !d_scores || !count) {
        set_error("alae_workspace_result: null argument");
        return ALAE_E_ARG;
    }
    *d_keys = ws->res_keys;
    *d_scores = reinterpret_cast<const int32_t *>(ws->res_scores);
    *count = (size_t)ws->res_count;
    return ALAE_OK;
}

alae_status alae_workspace_copy_result(const alae_workspace *ws, uint64_t *d_keys, int32_t *d_scores, void *stream) {
    if (!ws || !d_keys || !d_scores) {
        set_error("alae_workspace_copy_result: null argument");
        return ALAE_E_ARG;
    }
    if (ws->res_count == 0) return ALAE_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(d_keys, ws->res_keys, ws->res_count * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_scores, ws->res_scores, ws->res_count * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    return ALAE_OK;
}

void alae_hits_free(alae_hits *hits) {
    if (!hits) return;
    free(hits->query_end);
    free(hits->text_end);
    free(hits->score);
    hits->query_end = nullptr;
    hits->text_end = nullptr;
    hits->score = nullptr;
    hits->count = 0;
}

}  // extern "C"

namespace alae {

// Copy the workspace result to freshly allocated host arrays.
alae_status download_hits(alae_workspace *ws, hipStream_t s, alae_hits *out) {
    const uint64_t n = ws->res_count;
    alae_hits h;
    memset(&h, 0, sizeof(h));
    h.count = (size_t)n;
    const size_t alloc = n ? n : 1;
    h.query_end = (uint32_t *)malloc(alloc * sizeof(uint32_t));
    h.text_end = (uint64_t *)malloc(alloc * sizeof(uint64_t));
    h.score = (int32_t *)malloc(alloc * sizeof(int32_t));
    std::vector<uint64_t> keys;
    if (!h.query_end || !h.text_end || !h.score) {
        alae_hits_free(&h);
        set_error("out of host memory for %llu hits", (unsigned long long)n);
        return ALAE_E_NOMEM;
    }
    if (n) {
        try {
            keys.resize(n);
        } catch (const std::bad_alloc &) {
            alae_hits_free(&h);
            set_error("out of host memory for %llu hits", (unsigned long long)n);
            return ALAE_E_NOMEM;
        }
        hipError_t e1 = hipMemcpyAsync(keys.data(), ws->res_keys, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
        hipError_t e2 = hipMemcpyAsync(h.score, ws->res_scores, n * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        hipError_t e3 = hipStreamSynchronize(s);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            alae_hits_free(&h);
            set_error("copying hits to the host failed");
            return ALAE_E_DEVICE;
        }
        for (uint64_t i = 0; i < n; ++i) {
            h.query_end[i] = (uint32_t)(keys[i] >> 32);
            h.text_end[i] = keys[i] & 0xFFFFFFFFull;
        }
    }
    *out = h;
    return ALAE_OK;
}

}  // namespace alae

extern "C" {

alae_status alae_search(const alae_index *index, const char *query, size_t m, const alae_scoring *scoring, int32_t H,
                        const alae_search_opts *opts, alae_hits *out) {
    if (!index || !query || !out) {
        set_error("alae_search: null argument");
        return ALAE_E_ARG;
    }
    if (m == 0) {
        set_error("alae_search: empty query");
        return ALAE_E_ARG;
    }
    std::vector<uint8_t> codes;
    try {
        codes.resize(m);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    if (!encode(query, m, index->alphabet, codes.data())) {
        set_error("alae_search: query character outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    {
        Scheme sch;
        alae_status vs = check_scoring(scoring, index->sigma, H, sch);
        if (vs != ALAE_OK) return vs;
    }
    alae_workspace *ws = nullptr;
    alae_status st = alae_workspace_create(index, &ws);
    if (st != ALAE_OK) return st;
    std::unique_ptr<alae_workspace, void (*)(alae_workspace *)> guard(ws, alae_workspace_free);
    if ((st = grow(ws->d_query, ws->q_cap, m, false, 0, nullptr)) != ALAE_OK) return st;
    HIP_TRY(hipMemcpy(ws->d_query, codes.data(), m, hipMemcpyHostToDevice));
    size_t cnt = 0;
    st = alae_search_device(ws, ws->d_query, m, scoring, H, opts, nullptr, &cnt);
    if (st != ALAE_OK) return st;
    return download_hits(ws, nullptr, out);
}

alae_status alae_search_batch(const alae_index *index, const char *const *queries, const size_t *lens, size_t k,
                              const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                              alae_hits *outs) {
    if (!index || !queries || !lens || !outs || k == 0) {
        set_error("alae_search_batch: null argument or empty batch");
        return ALAE_E_ARG;
    }
    for (size_t i = 0; i < k; ++i) memset(&outs[i], 0, sizeof(alae_hits));
    for (size_t i = 0; i < k; ++i) {
        alae_status st = alae_search(index, queries[i], lens[i], scoring, H, opts, &outs[i]);
        if (st != ALAE_OK) {
            for (size_t j = 0; j < i; ++j) alae_hits_free(&outs[j]);
            return st;
        }
    }
    return ALAE_OK;
}

}  // extern "C"
