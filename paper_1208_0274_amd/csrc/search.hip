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
//      (Algorithm 1);
//   4. the emitted records are sorted by (query end, text end) and merged,
//      keeping the largest score per pair (Algorithm 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "alae_internal.h"
#include "device_algos.h"
#include "device_common.h"
#include "row_update.h"
#include "level_kernels.h"
#include "chain_kernels.h"
#include "mlp_internal.h"

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
    HIP_TRY(hipMalloc(&idx->d_text_alloc, idx->text.size() + 2 * kSlack));
    HIP_TRY(hipMemset(idx->d_text_alloc, 0, idx->text.size() + 2 * kSlack));
    idx->d_text = idx->d_text_alloc + kSlack;
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
    hipFree(idx->d_text_alloc);
    hipFree(idx->d_sa);
    hipFree(idx->d_occ);
    idx->d_text = nullptr;
    idx->d_text_alloc = nullptr;
    idx->d_sa = nullptr;
    idx->d_occ = nullptr;
    idx->on_device = false;
}

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

// U[j] = sum over the later columns j' of j's query of colmax(P[j']), from the
// exclusive scan of colrev.
__global__ void k_gain_bound(const uint32_t *scan_rev, uint32_t m, const uint32_t *qord, const uint32_t *segend,
                             int32_t *U) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    uint32_t u = scan_rev[m - 1 - j];
    if (qord) u -= scan_rev[m - segend[qord[j]]];
    U[j] = (int32_t)u;
}

// Columns to the end of each column's query, with kSegFirst on first columns,
// and the columns of its query before it.
__global__ void k_colseg(const uint32_t *qord, const uint32_t *segbeg, const uint32_t *segend, uint32_t m,
                         uint32_t *colseg, uint32_t *colbeg) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint32_t q = qord[j];
    colseg[j] = (segend[q] - j) | (segbeg[q] == j ? kSegFirst : 0u);
    colbeg[j] = j - segbeg[q];
}

// Query ordinal of every column of a batch (segbeg is increasing).
__global__ void k_qord(const uint32_t *segbeg, uint32_t nseg, uint32_t m, uint32_t *qord) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    uint32_t lo = 0, hi = nseg - 1;  // last segment whose first column is <= j
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (segbeg[mid] <= j)
            lo = mid;
        else
            hi = mid - 1;
    }
    qord[j] = lo;
}

// Split a batch result: off[q] = first record of query q (records are sorted
// by column, so each query's records are contiguous), then keys get the
// column inside their own query.
__global__ void k_batch_offsets(const uint64_t *keys, uint64_t count, const uint32_t *segbeg, uint32_t nseg,
                                uint64_t *off) {
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > nseg) return;
    if (q == nseg) {
        off[q] = count;
        return;
    }
    const uint64_t target = (uint64_t)segbeg[q] << 32;
    uint64_t lo = 0, hi = count;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    off[q] = lo;
}

__global__ void k_batch_localize(uint64_t *keys, uint64_t count, const uint32_t *qord, const uint32_t *segbeg) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t k = keys[i];
    const uint32_t col = (uint32_t)(k >> 32);
    keys[i] = ((uint64_t)(col - segbeg[qord[col]]) << 32) | (k & 0xFFFFFFFFull);
}

// Seed keys.  q-gram mode: key = code of P[j-q+1..j] (first char most
// significant), one per end column j >= q-1; other slots get the invalid key.
// Matrix mode: slot c*m + j holds key c when s(c, P[j]) > 0.
// In a batch a q-gram never spans two queries.
// qdom (nullable): left characters of the text's q-grams (k_qgram_left); a
// seed whose q-gram is preceded in the text by P[j - qeff] alone starts only
// alignments that one more match to the left beats everywhere (Section 3.2.2,
// Definition 1 and Lemma 1): its column is dropped.
__global__ void k_seed_keys(const uint8_t *q, uint32_t m, int sigma, int qeff, int matrix_mode, SubTable sub,
                            const uint32_t *qord, const uint32_t *segbeg, uint64_t invalid, uint64_t *keys,
                            uint32_t *vals, const uint32_t *qdom, Counters *cnt) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!matrix_mode) {
        if (t >= m) return;
        uint32_t j = (uint32_t)t;
        uint64_t key = invalid;
        const uint32_t first = qord ? segbeg[qord[j]] : 0u;
        if ((int64_t)j - (int64_t)first >= qeff - 1) {
            key = 0;
            for (int k = qeff - 1; k >= 0; --k) key = key * sigma + q[j - k];
            if (qdom && key < invalid && (int64_t)j - (int64_t)first >= qeff) {
                const uint32_t left = q[j - qeff];
                if (left < (uint32_t)sigma && qdom[key] == (1u << left)) {
                    key = invalid;
                    atomicAdd(&cnt->st_qdom, 1ull);
                }
            }
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

// Left characters of the text's q-grams (Section 3.2.2, Definition 1):
// mask[g] bit c is set when an occurrence of g is preceded by character c,
// bit 31 when one starts the text or follows a record separator.  g is the
// q-gram's code with its first character most significant (the seed keys'
// order); q-grams holding a separator are skipped.  mask starts at zero.
constexpr uint32_t kLeftNone = 1u << 31;
constexpr int kQgramPerThread = 256;  // windows a thread takes, 256 apart (a block: 65,536 consecutive)
constexpr uint32_t kQgramLds = 4096;  // tables up to this size are gathered in LDS first
constexpr uint64_t kQgramTableMax = 1ull << 24;  // larger tables (sigma^q) are not built
__global__ void __launch_bounds__(256) k_qgram_left(const uint8_t *text, uint64_t n, int sigma, int q, uint32_t ng,
                                                    uint32_t *mask) {
    __shared__ uint32_t lmask[kQgramLds];
    const bool local = ng <= kQgramLds;
    if (local)
        for (uint32_t g = threadIdx.x; g < ng; g += blockDim.x) lmask[g] = 0;
    __syncthreads();
    const uint64_t windows = n - (uint64_t)q + 1;  // the launch has n >= q
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * kQgramPerThread;
    for (int i = 0; i < kQgramPerThread; ++i) {
        // neighbouring lanes take neighbouring windows: every load below is one contiguous span
        const uint64_t x = base + (uint64_t)i * blockDim.x + threadIdx.x;
        if (x >= windows) break;
        uint32_t g = 0;
        bool letters = true;
        for (int k = 0; k < q; ++k) {
            const uint32_t c = text[x + (uint64_t)k];
            letters = letters && c < (uint32_t)sigma;
            g = g * (uint32_t)sigma + (c < (uint32_t)sigma ? c : 0u);
        }
        if (!letters) continue;
        const uint32_t left = x == 0 ? 0xFFu : (uint32_t)text[x - 1];
        const uint32_t bit = left < (uint32_t)sigma ? (1u << left) : kLeftNone;
        if (local) {
            if ((lmask[g] & bit) == 0) atomicOr(&lmask[g], bit);
        } else {
            if ((mask[g] & bit) == 0) atomicOr(&mask[g], bit);
        }
    }
    if (!local) return;
    __syncthreads();
    for (uint32_t g = threadIdx.x; g < ng; g += blockDim.x)
        if (lmask[g]) atomicOr(&mask[g], lmask[g]);
}

__device__ inline void backward_step(const SearchArgs &a, int c, int64_t &l, int64_t &r) {
    uint32_t ol, orr;
    if (a.occ_packed) {
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
                             Node *wide_nodes,
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
    Node nd;
    nd.lo = (uint32_t)l;
    nd.hi = (uint32_t)r;
    nd.off = (uint32_t)i;
    nd.len = (uint32_t)(end - i);
    if (nd.len > kLaneRow) {  // long seed rows are expanded by a whole wave
        const unsigned long long slot = atomicAdd(&cnt->lwnodes, 1ull);
        wide_nodes[slot] = nd;
    } else {
        const unsigned long long slot = atomicAdd(&cnt->nodes, 1ull);
        nodes[slot] = nd;
    }
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

// The tail of the frontier turned into chains: one chain item per occurrence
// of every node (a node with r occurrences gives r items that share its row,
// which stays in the level's entry buffer), so that the last sparse levels
// are walked along the text like any other chain instead of one FM-index
// level (and host round trip) per character.  The item count goes to
// cnt->cnodes; items past caps.cnodes are not written (kOvChainNodes).
__global__ void __launch_bounds__(256) k_split_nodes(const Node *nodes, uint32_t nn, const Node *wide, uint32_t nw,
                                                     uint32_t depth, Node *items, Caps caps, Counters *cnt) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = t < nn + nw;
    Node nd{0, 0, 0, 0};
    if (active) nd = t < nn ? nodes[t] : wide[t - nn];
    const uint32_t r = active ? nd.hi - nd.lo + 1 : 0u;
    uint32_t tot;
    const uint32_t pre = wave_excl_scan_u32(r, &tot);
    unsigned long long base = 0;
    if ((threadIdx.x & 63) == 0 && tot) base = atomicAdd(&cnt->cnodes, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    if (!r) return;
    const unsigned long long first = base + pre;
    if (first + r > caps.cnodes) {
        atomicOr(&cnt->overflow, kOvChainNodes);
        return;
    }
    for (uint32_t i = 0; i < r; ++i) items[first + i] = Node{nd.lo + i, depth, nd.off, nd.len};
}

// The frontier's tail goes to the chain walkers once a level has at most
// kSplitNodes nodes and a kSplitShrink-th of the largest level (so that the
// levels have done the shared work), and makes at most kSplitChains chains.
constexpr uint64_t kSplitNodes = 1ull << 15, kSplitChains = 1ull << 17, kSplitShrink = 64;

// Between two slots of a device-driven batch of levels (one block): commit
// the level the previous slot ran (or stop the batch on its overflow), then,
// when `begin`, test the loop's end and the tail split as the host loop does
// and begin the next level: keep the counters for a rerun and clear the
// per-level ones.
__global__ void __launch_bounds__(64) k_level_step(LevelCtl *ctl, Counters *cnt, bool begin) {
    __shared__ uint32_t s_go;
    if (threadIdx.x == 0) {
        uint32_t go = 0;
        if (ctl->stop == kStopNone) {
            if (ctl->pending) {
                if (cnt->overflow) {
                    ctl->stop = kStopOverflow;  // the host grows what overflowed and runs the level again
                } else {
                    const unsigned long long nn = cnt->nodes, nlw = cnt->lwnodes;
                    if (nn || nlw || cnt->cnodes) ctl->max_depth = (unsigned long long)ctl->d1;
                    ctl->depth = ctl->d1;
                    ctl->nn = nn;
                    ctl->nlw = nlw;
                    ctl->pending = 0;
                    ctl->ran += 1;
                }
            }
            if (begin && ctl->stop == kStopNone) {
                const unsigned long long f = ctl->nn + ctl->nlw;
                if (f == 0 || ctl->depth >= ctl->lmax) {
                    ctl->stop = kStopDone;
                } else if (f > kDeviceFrontier) {
                    ctl->stop = kStopLarge;  // the host-driven loop takes the large levels
                } else {
                    if (f > ctl->peak) ctl->peak = f;
                    if (f <= ctl->split_below && f * kSplitShrink <= ctl->peak)
                        ctl->stop = kStopSplit;  // the host hands the tail to the chain walkers
                    else
                        go = 1;
                }
            }
        }
        s_go = go;
    }
    __syncthreads();
    if (!s_go) return;
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(cnt);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(&ctl->snap);
    for (uint32_t i = threadIdx.x; i < sizeof(Counters) / sizeof(unsigned long long); i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt->nodes = cnt->entries = cnt->lwnodes = cnt->cnodes = cnt->centries = 0;
        cnt->overflow = 0;
        cnt->stage_need = 0;
        cnt->tasks = 0;
        ctl->d1 = ctl->depth + 1;
        ctl->pending = 1;
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

// Device memory of a search comes from hipMalloc, except in the entry point
// for callers that cannot allocate: there every buffer is cut from one fixed
// region (a bump arena, emptied before each search; space given up by a
// buffer that grows is not reused until then).  The arena of the calling
// thread is set only for the duration of such a search.
static thread_local FixedRegion *t_region = nullptr;

static hipError_t dev_alloc(void **p, uint64_t bytes) {
    if (!t_region) return hipMalloc(p, bytes);
    const uint64_t off = (t_region->used + 255) & ~255ull;
    if (off > t_region->size || bytes > t_region->size - off) return hipErrorOutOfMemory;
    *p = t_region->base + off;
    t_region->used = off + bytes;
    return hipSuccess;
}

static void dev_free(void *p) {
    if (!t_region && p) hipFree(p);
}

static void alloc_error(uint64_t bytes, hipError_t e) {
    if (t_region)
        set_error("the search needs more than the %llu-byte fixed scratch region (%llu bytes more requested)",
                  (unsigned long long)t_region->size, (unsigned long long)bytes);
    else
        set_error("device allocation of %llu bytes failed: %s", (unsigned long long)bytes, hipGetErrorString(e));
}

template <typename T>
static alae_status grow(T *&ptr, uint64_t &cap, uint64_t need, bool keep, uint64_t keep_count, hipStream_t s) {
    if (need <= cap && ptr) return ALAE_OK;
    uint64_t ncap = cap ? cap : 1024;
    while (ncap < need) ncap *= 2;
    T *np = nullptr;
    hipError_t e = dev_alloc(reinterpret_cast<void **>(&np), ncap * sizeof(T));
    if (e != hipSuccess) {
        hipGetLastError();
        alloc_error(ncap * sizeof(T), e);
        return ALAE_E_NOMEM;
    }
    if (keep && ptr && keep_count) {
        e = hipMemcpyAsync(np, ptr, keep_count * sizeof(T), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            set_error("device copy failed: %s", hipGetErrorString(e));
            dev_free(np);
            return ALAE_E_DEVICE;
        }
        hipStreamSynchronize(s);
    }
    dev_free(ptr);
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

struct QueueBufs {
    float *feat = nullptr;
    uint64_t feat_cap = 0;
    float *pred = nullptr;
    uint64_t pred_cap = 0;
    float *twork = nullptr;
    uint64_t twork_cap = 0;
    uint64_t *okeys = nullptr;
    uint32_t *ovals = nullptr;
    uint64_t o_cap = 0;
    uint64_t *okeys_alt = nullptr;
    uint32_t *ovals_alt = nullptr;
    uint64_t o_alt_cap = 0;
    uint32_t *part = nullptr;  // partition: heavy flags, positions, entry counts, entry positions
    uint64_t part_cap = 0;
    uint32_t *scratch = nullptr;
    uint64_t scratch_cap = 0;
};

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
    // results of a batch run in several groups, appended group by group
    uint64_t *acc_keys = nullptr;
    uint32_t *acc_scores = nullptr;
    uint64_t acc_cap = 0;
    // query
    uint8_t *d_query = nullptr;
    uint64_t q_cap = 0;
    uint8_t *qpad = nullptr;
    uint64_t qpad_cap = 0;
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
    // wide queue (whole search), its spill queue, global row buffers
    Node *lwide[2] = {nullptr, nullptr};  // level nodes with rows longer than a lane takes
    uint64_t lwide_cap[2] = {0, 0};
    Node *cnodes = nullptr;               // chains created by one level
    uint64_t cnode_cap = 0;
    Entry *cents = nullptr;
    uint64_t cent_cap = 0;
    Node *gnodes = nullptr;               // chains with gap states
    uint64_t gnode_cap = 0;
    Entry *gents = nullptr;
    uint64_t gent_cap = 0;
    Entry *stage = nullptr;               // per-block row staging of k_expand_level_wide
    uint64_t stage_cap = 0;
    Node *onodes = nullptr;
    uint64_t onode_cap = 0;
    Entry *oents = nullptr;
    uint64_t oent_cap = 0;
    Node *wnodes = nullptr;
    uint64_t wnode_cap = 0;
    Entry *wents = nullptr;
    uint64_t went_cap = 0;
    Entry *rowbuf = nullptr;
    uint64_t rowbuf_cap = 0;
    uint64_t wrow_cap = 0;
    // learned ordering, partition and traces of the walkers' queues (one set
    // per queue that can be in flight at once)
    QueueBufs qb[2];
    uint32_t *wsrc = nullptr;  // lane-queue origin of promoted wave-queue items (traces)
    uint64_t wsrc_cap = 0;
    uint32_t *ready = nullptr;  // publication flags of wave-queue slots (live pass)
    uint64_t ready_cap = 0;
    uint32_t *missed = nullptr;  // items the live pass gave up
    uint64_t missed_cap = 0;
    uint32_t *left = nullptr;  // items of the pass after it
    uint64_t left_cap = 0;
    hipStream_t s2 = nullptr;  // the concurrent wave-walker pass
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // child tasks of a level (node phase -> child phase)
    ChildTask *tasks = nullptr;
    uint64_t task_cap = 0;
    // batch segments
    uint32_t *qord = nullptr;
    uint64_t qord_cap = 0;
    uint32_t *colseg = nullptr;  // per column: columns to its query's end | kSegFirst
    uint64_t colseg_cap = 0;
    uint32_t *colbeg = nullptr;  // per column: columns of its query before it
    uint64_t colbeg_cap = 0;
    uint32_t *qdom = nullptr;    // left characters of the text's q-grams (k_qgram_left)
    uint64_t qdom_cap = 0;
    int qdom_q = 0;              // q of the table in qdom (0: none)
    uint32_t *segbeg = nullptr;  // nseg first columns, then nseg ends
    uint64_t seg_cap = 0;
    uint64_t *d_off = nullptr;
    uint64_t off_cap = 0;
    std::vector<uint32_t> h_seg;       // staging of segbeg/segend for the upload
    std::vector<uint64_t> h_off;       // per-query result offsets of the last batch
    uint64_t nseg = 0;                 // queries of the last search (1 for a single query)
    // counters
    Counters *d_cnt = nullptr;
    Counters *h_cnt = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evk0 = nullptr, evk1 = nullptr;  // around each expansion launch
    hipEvent_t evkm = nullptr;                  // after the lane kernel of a level
    hipEvent_t evks = nullptr;                  // after all level kernels, before the chain start
    // fixed device region every buffer is cut from (callers that cannot allocate)
    FixedRegion region{nullptr, 0, 0};
    // device-driven levels: their state, and one captured batch of level slots per
    // start parity with the launch parameters it was captured with
    LevelCtl *d_ctl = nullptr;
    LevelCtl *h_ctl = nullptr;
    hipGraphExec_t lg_exec[2] = {nullptr, nullptr};
    std::vector<uint8_t> lg_sig[2];
};

namespace alae {

static void ws_release_buffers(alae_workspace *ws);

static void ws_release(alae_workspace *ws) {
    ws_release_buffers(ws);
    hipFree(ws->qdom);  // kept by ws_release_buffers when small
    for (int i = 0; i < 2; ++i)
        if (ws->lg_exec[i]) hipGraphExecDestroy(ws->lg_exec[i]);
    hipFree(ws->d_ctl);
    if (ws->h_ctl) hipHostFree(ws->h_ctl);
    hipFree(ws->d_cnt);
    if (ws->h_cnt) hipHostFree(ws->h_cnt);
    if (ws->s2) hipStreamDestroy(ws->s2);
    if (ws->ev_fork) hipEventDestroy(ws->ev_fork);
    if (ws->ev_join) hipEventDestroy(ws->ev_join);
    if (ws->ev0) hipEventDestroy(ws->ev0);
    if (ws->ev1) hipEventDestroy(ws->ev1);
    if (ws->evk0) hipEventDestroy(ws->evk0);
    if (ws->evk1) hipEventDestroy(ws->evk1);
    if (ws->evkm) hipEventDestroy(ws->evkm);
    if (ws->evks) hipEventDestroy(ws->evks);
}

// Free the buffers a workspace grew (frontier, queues, hits, sort, result);
// its counters, stream and events stay.  The next search grows them again.
static void ws_release_buffers(alae_workspace *ws) {
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
    hipFree(ws->acc_keys);
    hipFree(ws->acc_scores);
    hipFree(ws->d_query);
    hipFree(ws->qpad);
    hipFree(ws->prof);
    hipFree(ws->U);
    hipFree(ws->colrev);
    hipFree(ws->seed_keys);
    hipFree(ws->seed_vals);
    hipFree(ws->seed_keys_alt);
    hipFree(ws->seed_vals_alt);
    hipFree(ws->onodes);
    hipFree(ws->oents);
    hipFree(ws->lwide[0]);
    hipFree(ws->lwide[1]);
    hipFree(ws->cnodes);
    hipFree(ws->cents);
    hipFree(ws->gnodes);
    hipFree(ws->gents);
    hipFree(ws->stage);
    hipFree(ws->wnodes);
    hipFree(ws->wents);
    hipFree(ws->rowbuf);
    for (int i = 0; i < 2; ++i) {
        QueueBufs &q = ws->qb[i];
        hipFree(q.feat);
        hipFree(q.pred);
        hipFree(q.twork);
        hipFree(q.okeys);
        hipFree(q.ovals);
        hipFree(q.okeys_alt);
        hipFree(q.ovals_alt);
        hipFree(q.part);
        hipFree(q.scratch);
    }
    hipFree(ws->wsrc);
    hipFree(ws->ready);
    hipFree(ws->missed);
    hipFree(ws->left);
    hipFree(ws->tasks);
    hipFree(ws->qord);
    hipFree(ws->colseg);
    hipFree(ws->colbeg);
    const bool keep_qdom = ws->qdom_cap <= (1ull << 18);  // a small q-gram table outlives a trim
    if (!keep_qdom) hipFree(ws->qdom);
    hipFree(ws->segbeg);
    hipFree(ws->d_off);
    alae_workspace fresh;
    fresh.idx = ws->idx;
    fresh.device = ws->device;
    fresh.d_cnt = ws->d_cnt;
    fresh.h_cnt = ws->h_cnt;
    fresh.ev0 = ws->ev0;
    fresh.ev1 = ws->ev1;
    fresh.evk0 = ws->evk0;
    fresh.evk1 = ws->evk1;
    fresh.evkm = ws->evkm;
    fresh.evks = ws->evks;
    fresh.ev_fork = ws->ev_fork;
    fresh.ev_join = ws->ev_join;
    fresh.s2 = ws->s2;
    fresh.region = ws->region;
    // the captured level batches name the freed buffers: the next search captures them again
    for (int i = 0; i < 2; ++i)
        if (ws->lg_exec[i]) hipGraphExecDestroy(ws->lg_exec[i]);
    fresh.d_ctl = ws->d_ctl;
    fresh.h_ctl = ws->h_ctl;
    if (keep_qdom) {
        fresh.qdom = ws->qdom;
        fresh.qdom_cap = ws->qdom_cap;
        fresh.qdom_q = ws->qdom_q;
    }
    *ws = fresh;
}

void workspace_trim(alae_workspace *ws) {
    if (ws && !ws->region.base) ws_release_buffers(ws);
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

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_f32(float *p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Before a walker drains a queue of n items: features (for a model or a
// trace), predictions, the order by predicted work (largest first) and a
// zeroed work record.  Buffers come from qb; everything runs on stream s.
struct QueuePrep {
    const float *pred = nullptr;
    const uint32_t *order = nullptr;
    float *twork = nullptr;
};

static alae_status prepare_queue(QueueBufs &q, const SearchArgs &a, const Node *items, const Entry *ents, uint64_t n,
                                 float queue, const alae_mlp *model, bool want_order, bool trace, hipStream_t s,
                                 QueuePrep &out) {
    out = QueuePrep();
    if (n == 0 || (!model && !trace)) return ALAE_OK;
    alae_status st;
    if ((st = grow(q.feat, q.feat_cap, n * ALAE_MLP_FEATURES, false, 0, s)) != ALAE_OK) return st;
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    k_item_features<<<blocks, 256, 0, s>>>(a, items, (uint32_t)n, ents, queue, q.feat);
    HIP_TRY(hipGetLastError());
    if (trace) {
        if ((st = grow(q.twork, q.twork_cap, n, false, 0, s)) != ALAE_OK) return st;
        k_zero_f32<<<blocks, 256, 0, s>>>(q.twork, n);
        out.twork = q.twork;
    }
    if (model) {
        if ((st = grow(q.pred, q.pred_cap, n, false, 0, s)) != ALAE_OK) return st;
        if ((st = mlp_predict_device(model, q.feat, (uint32_t)n, q.pred, s)) != ALAE_OK) return st;
        out.pred = q.pred;
    }
    if (model && want_order) {
        if ((st = grow_pair(q.okeys, q.ovals, q.o_cap, n, 0, s)) != ALAE_OK) return st;
        if ((st = grow_pair(q.okeys_alt, q.ovals_alt, q.o_alt_cap, n, 0, s)) != ALAE_OK) return st;
        if ((st = grow(q.scratch, q.scratch_cap, radix_scratch_words(n), false, 0, s)) != ALAE_OK) return st;
        k_order_keys<<<blocks, 256, 0, s>>>(q.pred, (uint32_t)n, q.okeys, q.ovals);
        bool in_alt = false;
        HIP_TRY(radix_sort_pairs(q.okeys, q.ovals, q.okeys_alt, q.ovals_alt, n, 32, q.scratch, &in_alt, s));
        out.order = in_alt ? q.ovals_alt : q.ovals;
    }
    return ALAE_OK;
}

// Append a drained queue's (features, work) to the caller's trace.
static alae_status record_trace(const QueueBufs &q, uint64_t n, alae_trace *tr, hipStream_t s) {
    if (!tr || n == 0) return ALAE_OK;
    const uint64_t room = tr->capacity > tr->count ? tr->capacity - tr->count : 0;
    const uint64_t take = std::min<uint64_t>(room, n);
    if (take && tr->features && tr->work) {
        HIP_TRY(hipMemcpyAsync(tr->features + tr->count * ALAE_MLP_FEATURES, q.feat,
                               take * ALAE_MLP_FEATURES * sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(tr->work + tr->count, q.twork, take * sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        tr->count += take;
    }
    tr->total += n;
    return ALAE_OK;
}

// Batches are at most this many queries (their ordinals are folded into the
// 64-bit prefix-max keys of the G_b scan).
constexpr uint64_t kMaxBatch = 65536;

// One search of d_query[0..m).  With nseg > 1 the query is the concatenation
// of nseg queries of lengths seg_lens[] (each > 0): they share the trie
// traversal but no alignment crosses from one into the next.
static alae_status run_search(alae_workspace *ws, const uint8_t *d_query, uint64_t m, const uint64_t *seg_lens,
                              uint64_t nseg, const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                              hipStream_t s, uint64_t *hit_count) {
    const alae_index *idx = ws->idx;
    Scheme sch;
    alae_status st = check_scoring(scoring, idx->sigma, H, sch);
    if (st != ALAE_OK) return st;
    ws->nseg = 0;
    ws->res_count = 0;
    if (m == 0) {
        set_error("empty query");
        return ALAE_E_ARG;
    }
    if (m >= 0x7FFFFFFFull) {
        set_error("query of %llu characters is too long", (unsigned long long)m);
        return ALAE_E_TOO_LONG;
    }
    const bool multi = nseg > 1;
    uint64_t mlong = m;  // longest query (Equation 1 bounds each query's alignments)
    if (multi) {
        if (nseg > kMaxBatch) {
            set_error("batch of %llu queries exceeds the limit of %llu", (unsigned long long)nseg,
                      (unsigned long long)kMaxBatch);
            return ALAE_E_ARG;
        }
        uint64_t sum = 0;
        mlong = 0;
        ws->h_seg.resize(2 * nseg);
        for (uint64_t i = 0; i < nseg; ++i) {
            if (seg_lens[i] == 0) {
                set_error("query %llu of the batch is empty", (unsigned long long)i);
                return ALAE_E_ARG;
            }
            ws->h_seg[i] = (uint32_t)sum;
            sum += seg_lens[i];
            ws->h_seg[nseg + i] = (uint32_t)sum;
            mlong = std::max(mlong, seg_lens[i]);
        }
        if (sum != m) {
            set_error("batch lengths add up to %llu, not %llu", (unsigned long long)sum, (unsigned long long)m);
            return ALAE_E_ARG;
        }
        // the G_b scan keys of a batch must stay below 2^44 (see seg_key)
        if ((uint64_t)(-(int64_t)scoring->ss) * m + (1ull << 30) >= (1ull << 44)) {
            set_error("batch of %llu columns is too long for gap extension %d", (unsigned long long)m, scoring->ss);
            return ALAE_E_TOO_LONG;
        }
    }
    const int sigma = idx->sigma;
    // BWT-SW's rule alone (Section 2.4): rows are kept while they hold a positive entry.  The
    // length filter then prunes nothing more: with threshold 1 in Equation 1, L_max bounds every
    // alignment of positive score, so no row with a positive entry is deeper.
    const bool zero_floor_only = opts && opts->zero_floor_only;
    const bool use_score_filter = !zero_floor_only && (opts ? opts->use_score_filter != 0 : true);
    const bool use_dom = !zero_floor_only && (opts ? opts->use_domination != 0 : true);
    const bool use_q = !zero_floor_only && (opts ? opts->use_qprefix != 0 : true);
    const int64_t lmax = lmax_of((int64_t)mlong, sch.smax, scoring->sg, scoring->ss, zero_floor_only ? 1 : H);
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
    a.u_closed = sch.matrix_mode ? 0 : 1;
    a.ngr_walk = getenv("ALAE_NO_NGR") ? 0 : 1;
    // reuse replays forks along text the copies share; it is kept to texts without separators
    a.use_reuse = (opts && opts->use_reuse && !multi && idx->nsep == 0) ? 1 : 0;
    a.occ_packed = idx->occ_packed ? 1 : 0;
    a.has_sep = idx->nsep > 0 ? 1 : 0;
    a.matrix_mode = sch.matrix_mode;
    a.s_match = sch.matrix_mode ? 0 : scoring->sa;
    a.s_mismatch = sch.matrix_mode ? 0 : scoring->sb;
    a.dom_reach = 32;
    for (int c = 0; c <= sigma; ++c) a.C[c] = (uint32_t)idx->C[c];
    if (multi) {
        if ((st = grow(ws->qord, ws->qord_cap, m, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->segbeg, ws->seg_cap, 2 * nseg, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->colseg, ws->colseg_cap, m, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->colbeg, ws->colbeg_cap, m, false, 0, s)) != ALAE_OK) return st;
        HIP_TRY(hipMemcpyAsync(ws->segbeg, ws->h_seg.data(), 2 * nseg * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        k_qord<<<(uint32_t)((m + 255) / 256), 256, 0, s>>>(ws->segbeg, (uint32_t)nseg, (uint32_t)m, ws->qord);
        k_colseg<<<(uint32_t)((m + 255) / 256), 256, 0, s>>>(ws->qord, ws->segbeg, ws->segbeg + nseg, (uint32_t)m,
                                                              ws->colseg, ws->colbeg);
        a.multi = 1;
        a.qord = ws->qord;
        a.segbeg = ws->segbeg;
        a.segend = ws->segbeg + nseg;
        a.colseg = ws->colseg;
        a.colbeg = ws->colbeg;
    }

    SubTable sub;
    memset(&sub, 0, sizeof(sub));
    memcpy(sub.s, sch.sub, (size_t)sigma * sigma);

    // the query with readable slack around it (windows of the domination test)
    if ((st = grow(ws->qpad, ws->qpad_cap, m + 2 * kSlack, false, 0, s)) != ALAE_OK) return st;
    HIP_TRY(hipMemsetAsync(ws->qpad, 0, kSlack, s));
    HIP_TRY(hipMemsetAsync(ws->qpad + kSlack + m, 0, kSlack, s));
    HIP_TRY(hipMemcpyAsync(ws->qpad + kSlack, d_query, m, hipMemcpyDeviceToDevice, s));
    a.query = ws->qpad + kSlack;
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
    k_gain_bound<<<gm, tb, 0, s>>>(ws->colrev, (uint32_t)m, multi ? a.qord : nullptr, a.segend, ws->U);

    // ---- seeds ---------------------------------------------------------------
    uint64_t space = 1;
    for (int k = 0; k < (matrix_seeds ? 1 : qeff); ++k) space *= (uint64_t)sigma;
    const uint64_t invalid = space;  // keys >= invalid are not seeds
    const int seed_depth = matrix_seeds ? 1 : qeff;
    // left characters of the text's q-grams, once per workspace and q (not in a fixed region)
    const uint32_t *qdom = nullptr;
    if (use_dom && !matrix_seeds && !t_region && space <= kQgramTableMax) {
        if (ws->qdom_q != qeff) {
            ws->qdom_q = 0;
            if ((st = grow(ws->qdom, ws->qdom_cap, space, false, 0, s)) != ALAE_OK) return st;
            k_fill_u32<<<(uint32_t)((space + 255) / 256), 256, 0, s>>>(ws->qdom, 0u, space);
            const uint64_t per_block = 256ull * kQgramPerThread;
            if (idx->n >= (uint64_t)qeff)
                k_qgram_left<<<(uint32_t)((idx->n - (uint64_t)qeff + 1 + per_block - 1) / per_block), 256, 0, s>>>(
                    idx->d_text, idx->n, sigma, qeff, (uint32_t)space, ws->qdom);
            HIP_TRY(hipGetLastError());
            ws->qdom_q = qeff;
        }
        qdom = ws->qdom;
    }
    k_seed_keys<<<(uint32_t)((nseed + tb - 1) / tb), tb, 0, s>>>(d_query, (uint32_t)m, sigma, seed_depth,
                                                                  matrix_seeds ? 1 : 0, sub,
                                                                  multi ? a.qord : nullptr, a.segbeg, invalid,
                                                                  ws->seed_keys, ws->seed_vals, qdom, ws->d_cnt);
    bool alt = false;
    HIP_TRY(radix_sort_pairs(ws->seed_keys, ws->seed_vals, ws->seed_keys_alt, ws->seed_vals_alt, nseed,
                             bit_length(invalid), ws->scratch, &alt, s));
    const uint64_t *sk = alt ? ws->seed_keys_alt : ws->seed_keys;
    const uint32_t *sv = alt ? ws->seed_vals_alt : ws->seed_vals;

    // level buffers: seeds need nseed entries and at most nseed nodes
    // first sizes of the buffers that grow on demand (sixteen times smaller in a fixed region)
    const int sh = t_region ? 4 : 0;
    uint64_t ent_want = std::max<uint64_t>(opts && opts->entry_capacity ? opts->entry_capacity : (1ull << 22) >> sh, nseed);
    for (int i = 0; i < 2; ++i) {
        if ((st = grow(ws->ents[i], ws->ent_cap[i], ent_want, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->nodes[i], ws->node_cap[i], std::max<uint64_t>(nseed, (1ull << 20) >> sh), false, 0, s)) != ALAE_OK)
            return st;
    }
    if ((st = grow(ws->lwide[0], ws->lwide_cap[0], std::max<uint64_t>(nseed, 1ull << 12), false, 0, s)) != ALAE_OK)
        return st;
    if ((st = grow(ws->lwide[1], ws->lwide_cap[1], 1ull << 12, false, 0, s)) != ALAE_OK) return st;
    uint64_t hit_want = opts && opts->hit_capacity ? opts->hit_capacity : (1ull << 20) >> sh;
    if ((st = grow_pair(ws->hkeys, ws->hscores, ws->hit_cap, hit_want, 0, s)) != ALAE_OK) return st;

    const int32_t seedM = matrix_seeds ? 0 : qeff * sch.sa;
    k_seed_nodes<<<(uint32_t)((nseed + tb - 1) / tb), tb, 0, s>>>(a, sk, sv, nseed, invalid, seed_depth,
                                                                   matrix_seeds ? 1 : 0, seedM, ws->ents[0],
                                                                   ws->nodes[0], ws->lwide[0], ws->d_cnt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ws->h_cnt->bad_query) {
        set_error("query holds codes outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    uint64_t nn = ws->h_cnt->nodes;
    int cur = 0;

    Caps caps{};
    caps.hits = ws->hit_cap;
    caps.hit_chunk = t_region ? 256 : kHitChunk;
    // seed-level hits (only when a seed score reaches H)
    uint64_t nlw0 = ws->h_cnt->lwnodes;
    int32_t seed_best = matrix_seeds ? sch.smax : seedM;
    if (seed_best >= H && (nn > 0 || nlw0 > 0)) {
        for (;;) {
            caps.hits = ws->hit_cap;
            if (nn > 0)
                k_seed_hits<<<(uint32_t)((nn + tb - 1) / tb), tb, 0, s>>>(a, ws->nodes[cur], (uint32_t)nn,
                                                                         ws->ents[cur], caps, ws->hkeys, ws->hscores,
                                                                         ws->d_cnt);
            if (nlw0 > 0)
                k_seed_hits<<<(uint32_t)((nlw0 + tb - 1) / tb), tb, 0, s>>>(a, ws->lwide[cur], (uint32_t)nlw0,
                                                                           ws->ents[cur], caps, ws->hkeys,
                                                                           ws->hscores, ws->d_cnt);
            HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (!(ws->h_cnt->overflow & kOvHits)) break;
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
    uint64_t launches = 0, level_launches = 0;  // launches counts every timed kernel
    double expand_ms = 0.0, start_ms = 0.0, general_ms = 0.0, wide_ms = 0.0, lane_ms = 0.0;
    uint64_t lane_launches = 0;
    int32_t depth = seed_depth;
    int cus = 256;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ws->device);
    // launch shapes (alae_search_opts; validated by the entry points)
    const int level_stage = (opts && opts->level_stage) ? opts->level_stage : kStageDefault;
    // device-driven levels (not in a fixed region, whose buffers cannot be sized for them)
    const int32_t level_batch = (opts && !t_region) ? opts->level_graph : 0;
    uint64_t device_levels = 0, graph_captures = 0;
    const uint32_t wide_bpc = (opts && opts->wide_blocks_per_cu) ? (uint32_t)opts->wide_blocks_per_cu : 3u;
    const uint32_t lane_wpc = (opts && opts->lane_waves_per_cu) ? (uint32_t)opts->lane_waves_per_cu : 8u;
    const uint32_t max_waves = (uint32_t)cus * lane_wpc;
    const uint64_t wrow = m + 2;  // a row never holds more than m entries
    // staging rows of the level-wide kernel start short and grow to the longest child row met
    uint64_t srow = std::min<uint64_t>(wrow, 4096);
    // (8 GiB: at the first levels of a wide batch every node's rows are long, and the
    // stage per block is what limits how many nodes expand at once)
    const uint64_t stage_budget = (t_region ? ((2ull << 30) >> (2 * sh)) : (8ull << 30)) / sizeof(Entry);
    // queues that live through the whole search
    for (int i = 0; i < 2; ++i)
        if ((st = grow(ws->lwide[i], ws->lwide_cap[i], 1ull << 12, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->cnodes, ws->cnode_cap, (1ull << 20) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->cents, ws->cent_cap, (1ull << 21) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->gnodes, ws->gnode_cap, (1ull << 16) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->gents, ws->gent_cap, (1ull << 20) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->wnodes, ws->wnode_cap, (1ull << 14) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->wents, ws->went_cap, (1ull << 20) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->onodes, ws->onode_cap, (1ull << 10) >> sh, false, 0, s)) != ALAE_OK) return st;
    if ((st = grow(ws->oents, ws->oent_cap, (1ull << 18) >> sh, false, 0, s)) != ALAE_OK) return st;
    auto timed = [&](double &acc) -> alae_status {
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(ws->evk1, s));
        HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        float kms = 0.f;
        HIP_TRY(hipEventElapsedTime(&kms, ws->evk0, ws->evk1));
        acc += kms;
        ++launches;
        return ALAE_OK;
    };
    auto set_caps = [&](int nxt) {
        caps.nodes = ws->node_cap[nxt];
        caps.entries = ws->ent_cap[nxt];
        caps.lwnodes = ws->lwide_cap[nxt];
        caps.hits = ws->hit_cap;
        caps.cnodes = ws->cnode_cap;
        caps.centries = ws->cent_cap;
        caps.gnodes = ws->gnode_cap;
        caps.gentries = ws->gent_cap;
        caps.wnodes = ws->wnode_cap;
        caps.wentries = ws->went_cap;
        caps.wrow = wrow;
        caps.srow = srow;
        caps.tasks = ws->task_cap;
        caps.onodes = ws->onode_cap;
        caps.oentries = ws->oent_cap;
        caps.hit_chunk = t_region ? 256 : kHitChunk;  // a fixed region holds fewer padding slots
    };
    // Grow what overflowed; queues that outlive one launch keep their first `keep` records.
    auto grow_overflowed = [&](const Counters &c, const Counters &keep, int nxt) -> alae_status {
        alae_status g = ALAE_OK;
        // record offsets are 32-bit: a count beyond that is a runaway, not a capacity problem
        const unsigned long long lim = 0xFFFFFFFFull;
        const struct {
            const char *name;
            unsigned long long v;
        } checks[] = {{"nodes", c.nodes},         {"entries", c.entries},   {"level-wide nodes", c.lwnodes},
                      {"chains", c.cnodes},       {"chain entries", c.centries}, {"general", c.gnodes},
                      {"general entries", c.gentries}, {"wide", c.wnodes}, {"wide entries", c.wentries},
                      {"spill", c.onodes},        {"spill entries", c.oentries}, {"hits", c.hits}};
        for (const auto &ck : checks) {
            if (ck.v > lim) {
                set_error("internal counter '%s' ran away to %llu (overflow bits %llx, depth %d)", ck.name, ck.v,
                          c.overflow, depth);
                return ALAE_E_INTERNAL;
            }
        }
        if ((c.overflow & kOvNodes) && (g = grow(ws->nodes[nxt], ws->node_cap[nxt], c.nodes, false, 0, s))) return g;
        if ((c.overflow & kOvEntries) && (g = grow(ws->ents[nxt], ws->ent_cap[nxt], c.entries, false, 0, s)))
            return g;
        if ((c.overflow & kOvLevelWide) &&
            (g = grow(ws->lwide[nxt], ws->lwide_cap[nxt], c.lwnodes, false, 0, s)))
            return g;
        if ((c.overflow & kOvChainNodes) && (g = grow(ws->cnodes, ws->cnode_cap, c.cnodes, false, 0, s))) return g;
        if ((c.overflow & kOvChainEntries) && (g = grow(ws->cents, ws->cent_cap, c.centries, false, 0, s)))
            return g;
        if ((c.overflow & kOvGeneralNodes) &&
            (g = grow(ws->gnodes, ws->gnode_cap, c.gnodes, true, keep.gnodes, s)))
            return g;
        if ((c.overflow & kOvGeneralEntries) &&
            (g = grow(ws->gents, ws->gent_cap, c.gentries, true, keep.gentries, s)))
            return g;
        if ((c.overflow & kOvWideNodes) && (g = grow(ws->wnodes, ws->wnode_cap, c.wnodes, true, keep.wnodes, s)))
            return g;
        if ((c.overflow & kOvWideEntries) &&
            (g = grow(ws->wents, ws->went_cap, c.wentries, true, keep.wentries, s)))
            return g;
        if ((c.overflow & kOvSpillNodes) && (g = grow(ws->onodes, ws->onode_cap, c.onodes, true, keep.onodes, s)))
            return g;
        if ((c.overflow & kOvSpillEntries) &&
            (g = grow(ws->oents, ws->oent_cap, c.oentries, true, keep.oentries, s)))
            return g;
        if ((c.overflow & kOvHits) && (g = grow_pair(ws->hkeys, ws->hscores, ws->hit_cap, c.hits, keep.hits, s)))
            return g;
        if (c.overflow & kOvStageRow) srow = std::min<uint64_t>(wrow, std::max<uint64_t>(2 * srow, c.stage_need));
        if (c.overflow & kOvWideRow) {
            set_error("a row exceeded the query length (internal error)");
            return ALAE_E_INTERNAL;
        }
        return ALAE_OK;
    };
    static const bool trace = getenv("ALAE_TRACE") != nullptr;
    uint64_t nlw = nlw0;  // nodes of the current level with long rows (in ws->lwide[cur])
    // The frontier's tail goes to the chain walkers (k_split_nodes) once it is
    // small and has few occurrences (kSplitNodes, kSplitShrink, kSplitChains).
    uint64_t peak_nodes = nn + nlw, split_below = (opts && opts->no_tail_split) ? 0 : kSplitNodes;
    uint64_t tail_chains = 0, tail_depth = 0;
    // One device-driven batch (level_batch != 0) from the current frontier.  On
    // return the host state (frontier, depth, parity, counters) is that after the
    // levels the batch committed; `rerun`: the next level overflowed, its buffers
    // are grown and the host copy of the counters is the one it started from.
    auto run_level_batch = [&](bool &rerun) -> alae_status {
        rerun = false;
        const uint32_t K = (uint32_t)(level_batch < 0 ? -level_batch : level_batch);
        if (!ws->d_ctl) {
            HIP_TRY(hipMalloc(&ws->d_ctl, sizeof(LevelCtl)));
            HIP_TRY(hipHostMalloc(&ws->h_ctl, sizeof(LevelCtl), hipHostMallocDefault));
        }
        // child tasks of the largest frontier a slot expands
        if ((st = grow(ws->tasks, ws->task_cap, (uint64_t)sigma * kDeviceFrontier, false, 0, s)) != ALAE_OK)
            return st;
        uint32_t wblocks[2];
        for (int p = 0; p < 2; ++p)
            wblocks[p] = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>({ws->lwide_cap[p], kDeviceFrontier, (uint64_t)cus * 16, stage_budget / srow}));
        if ((st = grow(ws->stage, ws->stage_cap, (uint64_t)std::max(wblocks[0], wblocks[1]) * srow, false, 0, s)) !=
            ALAE_OK)
            return st;
        Caps cp[2];  // the caps of a slot whose output parity is p
        set_caps(0);
        cp[0] = caps;
        set_caps(1);
        cp[1] = caps;
        // grids for a frontier of kDeviceFrontier nodes (sigma children each), fewer when the
        // buffers hold less; the kernels stride over anything beyond
        const uint64_t most_nodes = std::min<uint64_t>(kDeviceFrontier, std::max(ws->node_cap[0], ws->node_cap[1]));
        auto sgrid = [&](uint64_t cap, uint64_t want, uint64_t per_block) {
            return (uint32_t)std::max<uint64_t>(1, (std::min(cap, want) + per_block - 1) / per_block);
        };
        const uint32_t g_tasks = sgrid(ws->task_cap, (uint64_t)sigma * most_nodes, kLevelBlock);
        const uint32_t g_chains = sgrid(ws->cnode_cap, (uint64_t)sigma * most_nodes, kStartBlock);
        const ChainQueues cq{ws->gnodes, ws->gents, ws->wnodes, ws->wents, ws->hkeys, ws->hscores};
        auto enqueue = [&](int p0, hipStream_t es) {
            for (uint32_t j = 0; j < K; ++j) {
                const int p = p0 ^ (int)(j & 1u), q = p ^ 1;
                LevelOut o;
                o.onodes = ws->nodes[q];
                o.owide = ws->lwide[q];
                o.oent = ws->ents[q];
                o.chains = ws->cnodes;
                o.cent = ws->cents;
                o.hkeys = ws->hkeys;
                o.hscores = ws->hscores;
                o.node_base = o.wide_base = o.ent_base = o.chain_base = o.cent_base = o.hit_base = 0;
                const uint32_t g_nodes = sgrid(ws->node_cap[p], most_nodes, kTaskBlock);
                k_level_step<<<1, 64, 0, es>>>(ws->d_ctl, ws->d_cnt, true);
                k_level_tasks<true><<<g_nodes, kTaskBlock, 0, es>>>(a, ws->nodes[p], 0u, ws->tasks, cp[q], ws->d_cnt,
                                                             ws->d_ctl);
                if (level_stage == 2)
                    k_expand_children<2, true><<<g_tasks, kLevelBlock, 0, es>>>(a, ws->ents[p], ws->tasks, 0, o, cp[q],
                                                                         ws->d_cnt, ws->d_ctl);
                else if (level_stage == 8)
                    k_expand_children<8, true><<<g_tasks, kLevelBlock, 0, es>>>(a, ws->ents[p], ws->tasks, 0, o, cp[q],
                                                                         ws->d_cnt, ws->d_ctl);
                else
                    k_expand_children<4, true><<<g_tasks, kLevelBlock, 0, es>>>(a, ws->ents[p], ws->tasks, 0, o, cp[q],
                                                                         ws->d_cnt, ws->d_ctl);
                k_expand_level_wide<<<wblocks[p], 64, 0, es>>>(a, ws->lwide[p], 0u, ws->ents[p], 0, o, cp[q],
                                                              ws->d_cnt, ws->stage, ws->d_ctl);
                k_chain_start<true><<<g_chains, kStartBlock, 0, es>>>(a, sub, ws->cnodes, ws->cents, cq, cp[q], ws->d_cnt,
                                                               true, ws->d_ctl);
            }
            k_level_step<<<1, 64, 0, es>>>(ws->d_ctl, ws->d_cnt, false);  // commits the last slot's level
        };
        LevelCtl &h = *ws->h_ctl;
        h.nn = nn;
        h.nlw = nlw;
        h.peak = peak_nodes;
        h.split_below = split_below;
        h.max_depth = max_depth;
        h.depth = depth;
        h.d1 = depth + 1;
        h.lmax = (int32_t)lmax;
        h.stop = kStopNone;
        h.pending = 0;
        h.ran = 0;
        HIP_TRY(hipMemcpyAsync(ws->d_ctl, ws->h_ctl, offsetof(LevelCtl, snap), hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ws->evk0, s));
        if (level_batch > 0) {
            // the launch parameters of the batch: a captured graph is replayed while they hold
            std::vector<uint8_t> sig;
            auto put = [&](const void *v, size_t n) {
                const uint8_t *b = static_cast<const uint8_t *>(v);
                sig.insert(sig.end(), b, b + n);
            };
            put(&K, sizeof K);
            put(&level_stage, sizeof level_stage);
            put(&a, sizeof a);
            put(&sub, sizeof sub);
            put(cp, sizeof cp);
            put(wblocks, sizeof wblocks);
            put(&g_tasks, sizeof g_tasks);
            put(&g_chains, sizeof g_chains);
            const void *ptrs[] = {ws->nodes[0], ws->nodes[1], ws->ents[0],   ws->ents[1],  ws->lwide[0],
                                  ws->lwide[1], ws->tasks,    ws->cnodes,    ws->cents,    ws->gnodes,
                                  ws->gents,    ws->wnodes,   ws->wents,     ws->hkeys,    ws->hscores,
                                  ws->stage,    ws->d_ctl,    ws->d_cnt};
            put(ptrs, sizeof ptrs);
            const uint64_t ncap[2] = {ws->node_cap[0], ws->node_cap[1]};
            put(ncap, sizeof ncap);
            hipGraphExec_t &ex = ws->lg_exec[cur];
            if (!ex || ws->lg_sig[cur] != sig) {
                if (ex) {
                    HIP_TRY(hipGraphExecDestroy(ex));
                    ex = nullptr;
                }
                // captured on the second stream (idle during the levels; the caller's stream
                // may be the null stream, which cannot be captured), replayed on s
                hipGraph_t g = nullptr;
                HIP_TRY(hipStreamBeginCapture(ws->s2, hipStreamCaptureModeRelaxed));
                enqueue(cur, ws->s2);
                const hipError_t ce = hipStreamEndCapture(ws->s2, &g);
                if (ce != hipSuccess) {
                    if (g) hipGraphDestroy(g);
                    set_error("capturing the level batch failed: %s", hipGetErrorString(ce));
                    return ALAE_E_DEVICE;
                }
                const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                hipGraphDestroy(g);
                if (ie != hipSuccess) {
                    ex = nullptr;
                    set_error("instantiating the level batch failed: %s", hipGetErrorString(ie));
                    return ALAE_E_DEVICE;
                }
                ws->lg_sig[cur] = std::move(sig);
                ++graph_captures;
            }
            HIP_TRY(hipGraphLaunch(ex, s));
        } else {
            enqueue(cur, s);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(ws->evk1, s));
        HIP_TRY(hipMemcpyAsync(ws->h_ctl, ws->d_ctl, sizeof(LevelCtl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(ws->h_cnt, ws->d_cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        float kms = 0.f;
        HIP_TRY(hipEventElapsedTime(&kms, ws->evk0, ws->evk1));
        expand_ms += kms;
        ++launches;
        const LevelCtl &r = *ws->h_ctl;
        levels += r.ran;
        level_launches += r.ran;
        device_levels += r.ran;
        if (r.ran & 1u) cur ^= 1;
        nn = r.nn;
        nlw = r.nlw;
        depth = r.depth;
        peak_nodes = r.peak;
        max_depth = r.max_depth;
        if (trace)
            fprintf(stderr, "[alae] device levels to depth %d: %u levels, %llu+%llu nodes, stop %u; %.3f ms\n",
                    depth, r.ran, (unsigned long long)nn, (unsigned long long)nlw, r.stop, kms);
        if (r.stop == kStopOverflow) {
            ++retries;
            if ((st = grow_overflowed(*ws->h_cnt, r.snap, cur ^ 1)) != ALAE_OK) return st;
            *ws->h_cnt = r.snap;  // the counters the level found
            rerun = true;
        }
        return ALAE_OK;
    };
    while ((nn > 0 || nlw > 0) && depth < lmax) {
        peak_nodes = std::max<uint64_t>(peak_nodes, nn + nlw);
        if (nn + nlw <= split_below && (nn + nlw) * kSplitShrink <= peak_nodes) {
            // count and write the items (one host round trip), then decide
            Counters z = *ws->h_cnt;
            z.cnodes = z.centries = 0;
            z.overflow = 0;
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
            set_caps(cur);
            HIP_TRY(hipEventRecord(ws->evk0, s));
            k_split_nodes<<<(uint32_t)((nn + nlw + 255) / 256), 256, 0, s>>>(
                ws->nodes[cur], (uint32_t)nn, ws->lwide[cur], (uint32_t)nlw, (uint32_t)depth, ws->cnodes, caps,
                ws->d_cnt);
            double split_ms = 0.0;
            if ((st = timed(split_ms)) != ALAE_OK) return st;
            start_ms += split_ms;
            const uint64_t items = ws->h_cnt->cnodes;
            if (ws->h_cnt->overflow || items > kSplitChains || items == 0) {
                split_below = (nn + nlw) / 2;  // too many occurrences: again once the frontier has halved
            } else {
                const Counters before = *ws->h_cnt;
                for (;;) {
                    Counters z2 = before;
                    z2.overflow = 0;
                    HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z2, sizeof(Counters), hipMemcpyHostToDevice, s));
                    set_caps(cur);
                    const ChainQueues q{ws->gnodes, ws->gents, ws->wnodes, ws->wents, ws->hkeys, ws->hscores};
                    HIP_TRY(hipEventRecord(ws->evk0, s));
                    // the level kernels wrote these rows' hits at every occurrence already
                    k_chain_start<false><<<(uint32_t)((items + kStartBlock - 1) / kStartBlock), kStartBlock, 0, s>>>(
                        a, sub, ws->cnodes, ws->ents[cur], q, caps, ws->d_cnt, false, nullptr);
                    double ums = 0.0;
                    if ((st = timed(ums)) != ALAE_OK) return st;
                    start_ms += ums;
                    const Counters &c = *ws->h_cnt;
                    if (!c.overflow) break;
                    ++retries;
                    if ((st = grow_overflowed(c, before, cur)) != ALAE_OK) return st;
                }
                if (trace)
                    fprintf(stderr, "[alae] depth %d: %llu+%llu nodes -> %llu chains (frontier tail)\n", depth,
                            (unsigned long long)nn, (unsigned long long)nlw, (unsigned long long)items);
                tail_chains = items;
                tail_depth = (uint64_t)depth;
                nn = nlw = 0;
                break;
            }
        }
        if (level_batch != 0 && nn + nlw <= kDeviceFrontier) {
            // Device-driven levels: a batch of K level slots, each k_level_step and the
            // level's kernels with grids sized for a frontier of kDeviceFrontier nodes, then
            // one host round trip.  A level that overflowed is run again below by the host
            // path (its buffers grown); the tail split is taken at the top of the loop, and
            // a larger frontier by the host-driven loop.
            bool rerun = false;
            if ((st = run_level_batch(rerun)) != ALAE_OK) return st;
            if (!rerun) continue;
        }
        const int32_t d1 = depth + 1;
        const int nxt = cur ^ 1;
        const double t0 = expand_ms;
        // level expansion (lane kernel + wave kernel); per-level buffers restart,
        // hits and queues carry over
        const Counters before = *ws->h_cnt;
        for (;;) {
            Counters z = before;
            z.nodes = z.entries = z.lwnodes = z.cnodes = z.centries = 0;
            z.overflow = 0;
            z.stage_need = 0;
            z.tasks = 0;
            if ((st = grow(ws->tasks, ws->task_cap, (uint64_t)sigma * std::max<uint64_t>(nn, 1), false, 0, s)) !=
                ALAE_OK)
                return st;
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
            set_caps(nxt);
            LevelOut o;
            o.onodes = ws->nodes[nxt];
            o.owide = ws->lwide[nxt];
            o.oent = ws->ents[nxt];
            o.chains = ws->cnodes;
            o.cent = ws->cents;
            o.hkeys = ws->hkeys;
            o.hscores = ws->hscores;
            o.node_base = o.wide_base = o.ent_base = o.chain_base = o.cent_base = o.hit_base = 0;
            HIP_TRY(hipEventRecord(ws->evk0, s));
            if (nn > 0) {
                // node phase (child tasks), then one child row per lane
                k_level_tasks<false><<<(uint32_t)((nn + kTaskBlock - 1) / kTaskBlock), kTaskBlock, 0, s>>>(a, ws->nodes[cur], (uint32_t)nn,
                                                                          ws->tasks, caps, ws->d_cnt, nullptr);
                const uint64_t maxtasks = (uint64_t)sigma * nn;
                const uint32_t cblocks = (uint32_t)((maxtasks + kLevelBlock - 1) / kLevelBlock);
                if (level_stage == 2)
                    k_expand_children<2, false><<<cblocks, kLevelBlock, 0, s>>>(a, ws->ents[cur], ws->tasks, d1, o, caps,
                                                                         ws->d_cnt, nullptr);
                else if (level_stage == 8)
                    k_expand_children<8, false><<<cblocks, kLevelBlock, 0, s>>>(a, ws->ents[cur], ws->tasks, d1, o, caps,
                                                                         ws->d_cnt, nullptr);
                else
                    k_expand_children<4, false><<<cblocks, kLevelBlock, 0, s>>>(a, ws->ents[cur], ws->tasks, d1, o, caps,
                                                                         ws->d_cnt, nullptr);
            }
            HIP_TRY(hipEventRecord(ws->evkm, s));
            if (nlw > 0) {
                // one wave per node; as many as the CUs hold (rows just over a lane's limit are
                // common at the levels where the frontier widens, and each costs a few round trips)
                const uint32_t blocks = (uint32_t)std::max<uint64_t>(
                    1, std::min<uint64_t>({nlw, (uint64_t)cus * 16, stage_budget / srow}));
                if ((st = grow(ws->stage, ws->stage_cap, (uint64_t)blocks * srow, false, 0, s)) != ALAE_OK) return st;
                k_expand_level_wide<<<blocks, 64, 0, s>>>(a, ws->lwide[cur], (uint32_t)nlw, ws->ents[cur], d1, o,
                                                          caps, ws->d_cnt, ws->stage, nullptr);
            }
            // the chains this level makes, right behind it (one host round trip a level)
            HIP_TRY(hipEventRecord(ws->evks, s));
            {
                const uint64_t most = std::min<uint64_t>((uint64_t)sigma * (nn + nlw), caps.cnodes);
                if (most > 0) {
                    ChainQueues q{ws->gnodes, ws->gents, ws->wnodes, ws->wents, ws->hkeys, ws->hscores};
                    k_chain_start<false><<<(uint32_t)((most + kStartBlock - 1) / kStartBlock), kStartBlock, 0, s>>>(
                        a, sub, ws->cnodes, ws->cents, q, caps, ws->d_cnt, true, nullptr);
                }
            }
            double unit_ms = 0.0;
            if ((st = timed(unit_ms)) != ALAE_OK) return st;
            {
                float ems = 0.f, sms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ems, ws->evk0, ws->evks));
                HIP_TRY(hipEventElapsedTime(&sms, ws->evks, ws->evk1));
                expand_ms += ems;
                start_ms += sms;
            }
            ++level_launches;
            if (nn > 0) {  // the node and child phases alone (the trie-expansion kernels)
                float lms = 0.f;
                HIP_TRY(hipEventElapsedTime(&lms, ws->evk0, ws->evkm));
                lane_ms += lms;
                ++lane_launches;
            }
            const Counters &c = *ws->h_cnt;
            if (!c.overflow) break;
            ++retries;
            if ((st = grow_overflowed(c, before, nxt)) != ALAE_OK) return st;
        }
        const uint64_t nc = ws->h_cnt->cnodes;
        const double t1 = expand_ms;
        if (trace)
            fprintf(stderr,
                    "[alae] depth %d: %llu+%llu nodes -> %llu+%llu nodes, %llu entries, %llu chains "
                    "(general %llu, wide %llu); level %.3f ms, chains %.3f ms\n",
                    d1, (unsigned long long)nn, (unsigned long long)nlw, (unsigned long long)ws->h_cnt->nodes,
                    (unsigned long long)ws->h_cnt->lwnodes, (unsigned long long)ws->h_cnt->entries,
                    (unsigned long long)nc, (unsigned long long)ws->h_cnt->gnodes,
                    (unsigned long long)ws->h_cnt->wnodes, t1 - t0, start_ms);
        nn = ws->h_cnt->nodes;
        nlw = ws->h_cnt->lwnodes;
        cur = nxt;
        depth = d1;
        ++levels;
        if (nn || nlw || nc) max_depth = (uint64_t)d1;
    }

    const alae_mlp *model = opts ? opts->order_model : nullptr;
    const int order_queues = (opts && opts->order_queues) ? opts->order_queues : 2;
    // predicted log2(1 + work) at which a lane-queue chain joins the first wave pass
    const float part_thresh = (!opts || opts->partition_threshold <= 0.f) ? -3.0e38f : opts->partition_threshold;
    uint64_t partitioned = 0, leftover = 0;
    alae_trace *trace_out = opts ? opts->trace : nullptr;
    if (trace_out) trace_out->count = trace_out->total = 0;
    if (model && model->device != ws->device) {
        set_error("the ordering model lives on device %d, the search on device %d", model->device, ws->device);
        return ALAE_E_ARG;
    }
    // ---- chains ----------------------------------------------------------------
    // The lane walker (chains with gap states) and a first pass of the wave
    // walker (chains already too wide for a lane, plus lane-queue chains the
    // work predictor marks heavy) run concurrently on two streams; a second
    // wave pass then takes the chains the lane walker promoted.
    const uint64_t ng = ws->h_cnt->gnodes;
    const bool tracing = trace_out != nullptr;
    double order_ms = 0.0;
    HIP_TRY(hipEventRecord(ws->evk0, s));
    QueuePrep gq;
    if ((st = prepare_queue(ws->qb[0], a, ws->gnodes, ws->gents, ng, 0.f, model, (order_queues & 1) != 0, tracing,
                            s, gq)) != ALAE_OK)
        return st;
    uint64_t moved = 0;
    if (gq.pred && part_thresh > -1e30f && ng > 0) {
        // partition: heavy lane-queue chains go to the first wave pass
        QueueBufs &q = ws->qb[0];
        const uint64_t n1 = ng + 1;
        if ((st = grow(q.part, q.part_cap, 4 * n1, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(q.scratch, q.scratch_cap, scan_scratch_words(n1), false, 0, s)) != ALAE_OK) return st;
        uint32_t *heavy = q.part, *hpos = q.part + n1, *ent = q.part + 2 * n1, *epos = q.part + 3 * n1;
        k_partition_flags<<<(uint32_t)((n1 + 255) / 256), 256, 0, s>>>(gq.pred, ws->gnodes, (uint32_t)ng,
                                                                        part_thresh, heavy, ent);
        HIP_TRY(scan_exclusive_u32(heavy, hpos, n1, q.scratch, s));
        HIP_TRY(scan_exclusive_u32(ent, epos, n1, q.scratch, s));
        uint32_t tot[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(&tot[0], hpos + ng, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&tot[1], epos + ng, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (tot[0] > 0) {
            Counters c = *ws->h_cnt;
            if ((st = grow(ws->wnodes, ws->wnode_cap, c.wnodes + tot[0], true, c.wnodes, s)) != ALAE_OK) return st;
            if ((st = grow(ws->wents, ws->went_cap, c.wentries + tot[1], true, c.wentries, s)) != ALAE_OK) return st;
            k_partition_move<<<(uint32_t)((ng + 255) / 256), 256, 0, s>>>(a, ws->gnodes, ws->gents, (uint32_t)ng,
                                                                           heavy, hpos, epos, ws->wnodes, ws->wents,
                                                                           (uint32_t)c.wnodes, (uint32_t)c.wentries,
                                                                           ws->d_cnt);
            HIP_TRY(hipGetLastError());
            c.wnodes += tot[0];
            c.wentries += tot[1];
            *ws->h_cnt = c;
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, ws->h_cnt, sizeof(Counters), hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            moved = tot[0];
        }
    }
    // Wave-walker queue: items 0 .. nw1-1 are queued now; the lane walker
    // appends the chains it hands over.  A live pass on the second stream
    // takes items as they are published, concurrently with the lane walker.
    const uint64_t nw1 = ws->h_cnt->wnodes;
    QueuePrep wq;
    if ((st = prepare_queue(ws->qb[1], a, ws->wnodes, ws->wents, nw1, 1.f, model, (order_queues & 2) != 0, false, s,
                            wq)) != ALAE_OK)
        return st;
    if (model || tracing) {
        HIP_TRY(hipEventRecord(ws->evk1, s));
        HIP_TRY(hipEventSynchronize(ws->evk1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ws->evk0, ws->evk1));
        order_ms = ms;
    }
    const uint32_t live_blocks = (uint32_t)cus * wide_bpc;  // kWideWaves waves each
    // one query whose prefix-max keys fit 31 bits: the wave walkers' 32-bit scan
    const bool wide_fast = !multi && (int64_t)(std::max(1, a.smax) - a.ss) * (int64_t)m < (1ll << 30);
    if (ng > 0 || nw1 > 0) {
        const Counters before = *ws->h_cnt;
        for (;;) {
            Counters z = before;
            z.general_head = 0;
            z.wide_head = 0;
            z.gen_done = 0;
            z.gen_started = 0;
            z.missed = 0;
            z.t_gen0 = z.t_live0 = z.t_push0 = ~0ull;
            z.t_gen1 = z.t_live1 = 0;
            z.overflow = 0;
            if (tracing && ng > 0) {
                if ((st = grow(ws->wsrc, ws->wsrc_cap, ws->wnode_cap, false, 0, s)) != ALAE_OK) return st;
                k_fill_u32<<<(uint32_t)((ws->wnode_cap + 255) / 256), 256, 0, s>>>(ws->wsrc, 0xFFFFFFFFu,
                                                                                 ws->wnode_cap);
            }
            if (tracing) {
                if ((st = grow(ws->qb[1].twork, ws->qb[1].twork_cap, ws->wnode_cap, false, 0, s)) != ALAE_OK)
                    return st;
                k_zero_f32<<<(uint32_t)((ws->wnode_cap + 255) / 256), 256, 0, s>>>(ws->qb[1].twork, ws->wnode_cap);
            }
            if ((st = grow(ws->ready, ws->ready_cap, ws->wnode_cap, false, 0, s)) != ALAE_OK) return st;
            if ((st = grow(ws->missed, ws->missed_cap, live_blocks, false, 0, s)) != ALAE_OK) return st;
            k_fill_u32<<<(uint32_t)((nw1 + 255) / 256 + 1), 256, 0, s>>>(ws->ready, 1u, nw1);
            k_fill_u32<<<(uint32_t)((ws->wnode_cap - nw1 + 255) / 256 + 1), 256, 0, s>>>(ws->ready + nw1, 0u,
                                                                                      ws->wnode_cap - nw1);
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
            set_caps(cur);
            const uint32_t waves = (uint32_t)std::min<uint64_t>((ng + 63) / 64, max_waves);
            const uint32_t gblocks = (waves + 3) / 4;
            LiveQueue lq;
            lq.ready = ws->ready;
            lq.nstatic = (uint32_t)nw1;
            lq.gen_items = ng;
            lq.missed = ws->missed;
            lq.patience = 20000000;  // 200 ms of the 100 MHz clock without any progress
            HIP_TRY(hipEventRecord(ws->evk0, s));
            // the second stream waits for the set-up above, not for the lane walker
            HIP_TRY(hipEventRecord(ws->ev_fork, s));
            HIP_TRY(hipStreamWaitEvent(ws->s2, ws->ev_fork, 0));
            if (ng > 0)
                k_chain_general<<<gblocks, 256, 0, s>>>(a, ws->gnodes, (uint32_t)ng, ws->gents, ws->wnodes, ws->wents,
                                                        ws->hkeys, ws->hscores, caps, ws->d_cnt, gq.order, gq.twork,
                                                        tracing ? ws->wsrc : nullptr, ws->ready);
            HIP_TRY(hipGetLastError());
            // At most two wave-walker waves per SIMD run beside the lane walker: with more, walker
            // blocks dispatched first could leave a CU no room for a lane-walker wave (whose
            // pushes they wait for).  The rest start on the lane walker's stream once it ends and
            // take items from the same queue.
            const uint32_t live_during = std::min<uint32_t>(live_blocks, (uint32_t)cus * (8u / kWideWaves));
            const uint32_t live_after = live_blocks - live_during;
            auto wide_live = [&](uint32_t blocks, hipStream_t st2) {
                if (wide_fast)
                    k_chain_wide_lds<true><<<blocks, 64 * kWideWaves, 0, st2>>>(
                        a, ws->wnodes, 0, 0xFFFFFFFFu, ws->wents, ws->onodes, ws->oents, ws->hkeys, ws->hscores,
                        caps, ws->d_cnt, wq.order, tracing ? ws->qb[1].twork : nullptr, lq);
                else
                    k_chain_wide_lds<false><<<blocks, 64 * kWideWaves, 0, st2>>>(
                        a, ws->wnodes, 0, 0xFFFFFFFFu, ws->wents, ws->onodes, ws->oents, ws->hkeys, ws->hscores,
                        caps, ws->d_cnt, wq.order, tracing ? ws->qb[1].twork : nullptr, lq);
            };
            wide_live(live_during, ws->s2);
            HIP_TRY(hipGetLastError());
            if (live_after > 0) {
                wide_live(live_after, s);
                HIP_TRY(hipGetLastError());
            }
            HIP_TRY(hipEventRecord(ws->ev_join, ws->s2));
            HIP_TRY(hipStreamWaitEvent(s, ws->ev_join, 0));
            if ((st = timed(general_ms)) != ALAE_OK) return st;
            const Counters &c = *ws->h_cnt;
            if (!c.overflow) break;
            ++retries;
            if ((st = grow_overflowed(c, before, cur)) != ALAE_OK) return st;
        }
    }
    // items the live pass did not take: given-up claims, then the unclaimed tail
    double live_ms = 0.0;
    {
        const Counters c0 = *ws->h_cnt;
        if (c0.t_live0 != ~0ull && c0.t_live1 > c0.t_live0) live_ms = (double)(c0.t_live1 - c0.t_live0) * 1e-5;
        if (trace && (ng > 0 || nw1 > 0)) {
            const double t0 = (double)std::min(c0.t_gen0, c0.t_live0);
            fprintf(stderr,
                    "[alae] chains: lane walker %.3f-%.3f ms, live wave pass %.3f-%.3f ms, first push %.3f ms, "
                    "missed %llu, pushed %llu (static %llu)\n",
                    (c0.t_gen0 - t0) * 1e-5, (c0.t_gen1 - t0) * 1e-5, (c0.t_live0 - t0) * 1e-5,
                    (c0.t_live1 - t0) * 1e-5, c0.t_push0 == ~0ull ? -1.0 : (c0.t_push0 - t0) * 1e-5,
                    (unsigned long long)c0.missed, (unsigned long long)c0.wnodes, (unsigned long long)nw1);
        }
        const uint64_t made = c0.wnodes;
        const uint64_t head = std::min<uint64_t>(c0.wide_head, made);
        // given-up claims past the last pushed item name no item
        std::vector<uint32_t> miss(std::min<uint64_t>(c0.missed, live_blocks));
        if (!miss.empty()) {
            HIP_TRY(hipMemcpyAsync(miss.data(), ws->missed, miss.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        std::vector<uint32_t> lst;
        for (uint32_t v : miss)
            if (v < made) lst.push_back(v);
        for (uint64_t i = head; i < made; ++i) lst.push_back((uint32_t)i);
        const uint64_t nleft = lst.size();
        if (nleft > 0) {
            if ((st = grow(ws->left, ws->left_cap, nleft, false, 0, s)) != ALAE_OK) return st;
            HIP_TRY(hipMemcpyAsync(ws->left, lst.data(), nleft * sizeof(uint32_t), hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            const Counters before = *ws->h_cnt;
            const uint32_t blocks = (uint32_t)std::min<uint64_t>(nleft, (uint64_t)cus * (24u / kWideWaves));
            LiveQueue none;
            memset(&none, 0, sizeof(none));
            for (;;) {
                Counters z = before;
                z.wide_head = 0;
                z.overflow = 0;
                HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
                set_caps(cur);
                HIP_TRY(hipEventRecord(ws->evk0, s));
                if (wide_fast)
                    k_chain_wide_lds<true><<<blocks, 64 * kWideWaves, 0, s>>>(
                        a, ws->wnodes, 0, (uint32_t)nleft, ws->wents, ws->onodes, ws->oents, ws->hkeys, ws->hscores,
                        caps, ws->d_cnt, ws->left, tracing ? ws->qb[1].twork : nullptr, none);
                else
                    k_chain_wide_lds<false><<<blocks, 64 * kWideWaves, 0, s>>>(
                        a, ws->wnodes, 0, (uint32_t)nleft, ws->wents, ws->onodes, ws->oents, ws->hkeys, ws->hscores,
                        caps, ws->d_cnt, ws->left, tracing ? ws->qb[1].twork : nullptr, none);
                if ((st = timed(wide_ms)) != ALAE_OK) return st;
                const Counters &c = *ws->h_cnt;
                if (!c.overflow) break;
                ++retries;
                if ((st = grow_overflowed(c, before, cur)) != ALAE_OK) return st;
            }
        }
        leftover = nleft;
        if (tracing && made > 0) {
            QueueBufs &q = ws->qb[1];
            if ((st = grow(q.feat, q.feat_cap, made * ALAE_MLP_FEATURES, false, 0, s)) != ALAE_OK) return st;
            k_item_features<<<(uint32_t)((made + 255) / 256), 256, 0, s>>>(a, ws->wnodes, (uint32_t)made, ws->wents,
                                                                            1.f, q.feat);
            if (ng > 0)
                k_link_work<<<(uint32_t)((made + 255) / 256), 256, 0, s>>>(ws->wsrc, 0, (uint32_t)made, q.twork,
                                                                            ws->qb[0].twork, (uint32_t)ng);
            HIP_TRY(hipGetLastError());
            if ((st = record_trace(q, made, trace_out, s)) != ALAE_OK) return st;
        }
        if ((st = record_trace(ws->qb[0], ng, trace_out, s)) != ALAE_OK) return st;
    }
    partitioned = moved;
    // rows that outgrew LDS: one wave each, rows in global memory
    const uint64_t no = ws->h_cnt->onodes;
    if (no > 0) {
        const uint64_t budget_entries = ((8ull << 30) >> (2 * sh)) / sizeof(Entry);
        uint64_t waves = std::min<uint64_t>(no, (uint64_t)max_waves);
        waves = std::max<uint64_t>(1, std::min<uint64_t>(waves, budget_entries / (2 * wrow)));
        if (ws->wrow_cap != wrow || ws->rowbuf_cap < waves * 2 * wrow) {
            dev_free(ws->rowbuf);
            ws->rowbuf = nullptr;
            ws->rowbuf_cap = 0;
            const hipError_t e = dev_alloc(reinterpret_cast<void **>(&ws->rowbuf), waves * 2 * wrow * sizeof(Entry));
            if (e != hipSuccess) {
                hipGetLastError();
                alloc_error(waves * 2 * wrow * sizeof(Entry), e);
                return ALAE_E_NOMEM;
            }
            ws->rowbuf_cap = waves * 2 * wrow;
            ws->wrow_cap = wrow;
        }
        const Counters before = *ws->h_cnt;
        for (;;) {
            Counters z = before;
            z.overflow_head = 0;
            z.overflow = 0;
            HIP_TRY(hipMemcpyAsync(ws->d_cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, s));
            set_caps(cur);
            HIP_TRY(hipEventRecord(ws->evk0, s));
            k_chain_wide_global<<<(uint32_t)waves, 64, 0, s>>>(a, ws->onodes, (uint32_t)no, ws->oents, ws->rowbuf,
                                                               ws->hkeys, ws->hscores, caps, ws->d_cnt);
            if ((st = timed(wide_ms)) != ALAE_OK) return st;
            const Counters &c = *ws->h_cnt;
            if (!c.overflow) break;
            ++retries;
            if ((st = grow_overflowed(c, before, cur)) != ALAE_OK) return st;
        }
    }

    // ---- max-merge and sort --------------------------------------------------
    const uint64_t emitted = ws->h_cnt->hits;           // hit slots written, padding included
    const uint64_t padding = ws->h_cnt->hit_padding;    // unused reserved slots (sorted last)
    uint64_t unique = 0;
    float merge_ms = 0.f;
    HIP_TRY(hipEventRecord(ws->evk0, s));
    if (emitted > 0) {
        if ((st = grow_pair(ws->hkeys_alt, ws->hscores_alt, ws->alt_cap, emitted, 0, s)) != ALAE_OK) return st;
        uint64_t need = std::max(radix_scratch_words(emitted), scan_scratch_words(emitted + 1));
        if ((st = grow(ws->scratch, ws->scratch_cap, need, false, 0, s)) != ALAE_OK) return st;
        // sort on (query end, text end) packed into as few bits as the sizes need
        const int tb = std::max(1, bit_length(idx->n - 1));  // text ends are below n
        const int qb = std::max(1, bit_length(m - 1));
        int bits = qb + tb;
        if ((m - 1) == (1ull << qb) - 1 && (idx->n - 1) == (1ull << tb) - 1) ++bits;  // keep the padding key on top
        // scores fit below the key when smax * m does: one 64-bit record a hit
        const int sb = bit_length((uint64_t)std::max(1, a.smax) * m);
        const bool packed = bits + sb <= 64;
        if ((st = grow(ws->flags, ws->flags_cap, emitted + 1, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow(ws->pos, ws->pos_cap, emitted + 1, false, 0, s)) != ALAE_OK) return st;
        if ((st = grow_pair(ws->res_keys, ws->res_scores, ws->res_cap, emitted, 0, s)) != ALAE_OK) return st;
        const uint64_t valid = emitted - padding;
        bool in_alt = false;
        const uint32_t *count_at = ws->pos + valid;  // where the merge leaves the distinct count
        if (packed) {
            HIP_TRY(pack_sort_hits(ws->hkeys, ws->hscores, ws->hkeys_alt, emitted, tb, sb, bits, ws->scratch,
                                   &in_alt, s));
            const uint64_t *k = in_alt ? ws->hkeys_alt : ws->hkeys;
            HIP_TRY(max_merge_packed(k, valid, sb, tb, ws->res_keys, ws->res_scores, ws->pos, ws->scratch, s));
            count_at = ws->pos + merge_tile_count(valid);
        } else {
            HIP_TRY(repack_hit_keys(ws->hkeys, emitted, tb, bits, s));
            HIP_TRY(radix_sort_pairs(ws->hkeys, ws->hscores, ws->hkeys_alt, ws->hscores_alt, emitted, bits,
                                     ws->scratch, &in_alt, s));
            const uint64_t *k = in_alt ? ws->hkeys_alt : ws->hkeys;
            const uint32_t *v = in_alt ? ws->hscores_alt : ws->hscores;
            HIP_TRY(max_merge_sorted(k, v, valid, ws->res_keys, ws->res_scores, ws->flags, ws->pos, ws->scratch, s,
                                     tb));
        }
        uint32_t cnt32 = 0;
        HIP_TRY(hipEventRecord(ws->evk1, s));
        HIP_TRY(hipMemcpyAsync(&cnt32, count_at, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipEventElapsedTime(&merge_ms, ws->evk0, ws->evk1));
        unique = cnt32;
    }
    ws->res_count = unique;
    *hit_count = unique;
    ws->nseg = multi ? nseg : 1;
    if (multi) {
        // per-query ranges of the sorted result, then query-local columns
        if ((st = grow(ws->d_off, ws->off_cap, nseg + 1, false, 0, s)) != ALAE_OK) return st;
        k_batch_offsets<<<(uint32_t)((nseg + 1 + 255) / 256), 256, 0, s>>>(ws->res_keys, unique, a.segbeg,
                                                                           (uint32_t)nseg, ws->d_off);
        if (unique > 0)
            k_batch_localize<<<(uint32_t)((unique + 255) / 256), 256, 0, s>>>(ws->res_keys, unique, a.qord,
                                                                             a.segbeg);
        HIP_TRY(hipGetLastError());
        ws->h_off.resize(nseg + 1);
        HIP_TRY(hipMemcpyAsync(ws->h_off.data(), ws->d_off, (nseg + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (opts && opts->stats) {
        alae_stats *o = opts->stats;
        const Counters &c = *ws->h_cnt;
        o->nodes = c.st_nodes;
        o->entries = c.st_entries;
        o->entries_diag = c.st_diag;
        o->entries_gap2 = c.st_gap2;
        o->entries_gap3 = c.st_gap3;
        o->dominated = c.st_dominated;
        o->dominated_qgram = c.st_qdom;
        o->emitted = emitted - padding;
        o->hits = unique;
        o->levels = levels;
        o->retries = retries;
        o->max_depth = max_depth;
        o->occ_reads = c.st_occ_reads;
        o->sa_reads = c.st_sa_reads;
        o->text_reads = c.st_text_reads;
        o->frontier_bytes = c.st_frontier_bytes;
        o->level_launches = level_launches;
        o->level_ms = expand_ms;
        o->start_ms = start_ms;
        o->general_ms = general_ms;
        o->wide_ms = wide_ms;
        o->chain_steps = c.st_chain_steps + c.st_ngr_steps;
        o->wide_steps = c.st_wide_steps;
        o->promoted = c.st_promoted;
        o->dominated_gapped = c.st_dominated_gapped;
        o->chain_bytes = c.st_chain_bytes;
        o->merge_ms = merge_ms;
        o->partitioned = partitioned;
        o->order_ms = order_ms;
        o->level_lane_ms = lane_ms;
        o->level_lane_launches = lane_launches;
        o->tail_chains = tail_chains;
        o->tail_depth = tail_depth;
        o->leftover = leftover;
        o->reused = c.st_reused;
        o->replay_chains = c.st_replay;
        o->wide_entries = c.st_wide_entries;
        o->wide_max_steps = c.st_wide_max;
        o->wide_slowest_ms = (double)(c.st_wide_slow >> 38) * 1e-5;
        o->wide_slowest_start_ms = (double)((c.st_wide_slow >> 18) & ((1ull << 20) - 1)) * 1e-3;
        o->wide_slowest_rows = c.st_wide_slow & ((1ull << 18) - 1);
        o->live_ms = live_ms;
        o->device_levels = device_levels;
        o->graph_captures = graph_captures;
    }
    return ALAE_OK;
}

}  // namespace alae

// Launch-shape options: 0 (default) or a supported value.
static bool launch_shapes_ok(const alae_search_opts *o, const char *where) {
    if (!o) return true;
    const bool ok = (o->level_stage == 0 || o->level_stage == 2 || o->level_stage == 4 || o->level_stage == 8) &&
                    o->wide_blocks_per_cu >= 0 && o->wide_blocks_per_cu <= 8 && o->lane_waves_per_cu >= 0 &&
                    o->lane_waves_per_cu <= 16 && o->level_graph >= -64 && o->level_graph <= 64;
    if (!ok)
        set_error("%s: level_stage must be 0, 2, 4 or 8, wide_blocks_per_cu 0..8, lane_waves_per_cu 0..16, "
                  "level_graph -64..64",
                  where);
    return ok;
}

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
    HIP_TRY(hipEventCreate(&ws->evkm));
    HIP_TRY(hipEventCreate(&ws->evks));
    HIP_TRY(hipEventCreateWithFlags(&ws->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ws->ev_join, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&ws->s2, hipStreamNonBlocking));
    *out = ws.release();
    return ALAE_OK;
}

void alae_workspace_free(alae_workspace *ws) {
    if (!ws) return;
    ws_release(ws);
    delete ws;
}

}  // extern "C"

namespace alae {

alae_status region_workspace_create(int device, uint8_t *region, uint64_t bytes, alae_workspace **out) {
    const uint64_t head = (sizeof(Counters) + 255) & ~255ull;
    if (!region || bytes <= head) {
        set_error("fixed scratch region is missing or too small");
        return ALAE_E_ARG;
    }
    std::unique_ptr<alae_workspace> ws(new (std::nothrow) alae_workspace());
    if (!ws) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    ws->device = device;
    HIP_TRY(hipSetDevice(device));
    ws->d_cnt = reinterpret_cast<Counters *>(region);
    ws->h_cnt = new (std::nothrow) Counters();
    if (!ws->h_cnt) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    ws->region = FixedRegion{region + head, bytes - head, 0};
    HIP_TRY(hipEventCreate(&ws->ev0));
    HIP_TRY(hipEventCreate(&ws->ev1));
    HIP_TRY(hipEventCreate(&ws->evk0));
    HIP_TRY(hipEventCreate(&ws->evk1));
    HIP_TRY(hipEventCreate(&ws->evkm));
    HIP_TRY(hipEventCreate(&ws->evks));
    HIP_TRY(hipEventCreateWithFlags(&ws->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ws->ev_join, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&ws->s2, hipStreamNonBlocking));
    *out = ws.release();
    return ALAE_OK;
}

alae_status region_search(alae_workspace *ws, const alae_index *idx, const uint8_t *d_query, uint64_t m,
                          const alae_scoring *scoring, int32_t H, const alae_search_opts *opts, void *stream,
                          uint64_t *d_keys, int32_t *d_scores, uint64_t capacity, uint64_t *hit_count) {
    if (!launch_shapes_ok(opts, "alae_search_device_noalloc")) return ALAE_E_ARG;
    if (opts && (opts->order_model || opts->trace)) {
        set_error("the search without allocation takes no ordering model and no trace");
        return ALAE_E_ARG;
    }
    if (idx->device != ws->device) {
        set_error("index on device %d, scratch region on device %d", idx->device, ws->device);
        return ALAE_E_ARG;
    }
    {
        std::lock_guard<std::mutex> lock(idx->mu);
        if (!idx->on_device) {
            set_error("the index is not on the device yet (alae_index_upload, or any other search, puts it there)");
            return ALAE_E_ARG;
        }
    }
    // every buffer pointer starts empty: the region is handed out afresh
    {
        alae_workspace fresh;
        fresh.idx = idx;
        fresh.device = ws->device;
        fresh.d_cnt = ws->d_cnt;
        fresh.h_cnt = ws->h_cnt;
        fresh.ev0 = ws->ev0;
        fresh.ev1 = ws->ev1;
        fresh.evk0 = ws->evk0;
        fresh.evk1 = ws->evk1;
        fresh.evkm = ws->evkm;
        fresh.evks = ws->evks;
        fresh.ev_fork = ws->ev_fork;
        fresh.ev_join = ws->ev_join;
        fresh.s2 = ws->s2;
        fresh.region = FixedRegion{ws->region.base, ws->region.size, 0};
        *ws = fresh;
    }
    struct RegionScope {
        explicit RegionScope(FixedRegion *r) { t_region = r; }
        ~RegionScope() { t_region = nullptr; }
    } scope(&ws->region);
    HIP_TRY(hipSetDevice(ws->device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(ws->ev0, s));
    uint64_t cnt = 0;
    alae_status st = run_search(ws, d_query, m, nullptr, 1, scoring, H, opts, s, &cnt);
    if (st != ALAE_OK) return st;
    *hit_count = cnt;
    if (cnt > capacity) {
        set_error("the result holds %llu hits, more than the output capacity of %llu", (unsigned long long)cnt,
                  (unsigned long long)capacity);
        return ALAE_E_NOMEM;
    }
    if (cnt > 0) {
        HIP_TRY(hipMemcpyAsync(d_keys, ws->res_keys, cnt * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_scores, ws->res_scores, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipEventRecord(ws->ev1, s));
    HIP_TRY(hipEventSynchronize(ws->ev1));
    if (opts && opts->stats) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ws->ev0, ws->ev1);
        opts->stats->device_ms = ms;
    }
    return ALAE_OK;
}

}  // namespace alae

extern "C" {

alae_status alae_index_upload(const alae_index *index) {
    if (!index) {
        set_error("alae_index_upload: null index");
        return ALAE_E_ARG;
    }
    return ensure_device(index);
}

alae_status alae_search_device(alae_workspace *ws, const uint8_t *d_query_codes, size_t m,
                               const alae_scoring *scoring, int32_t H, const alae_search_opts *opts, void *stream,
                               size_t *hit_count) {
    if (!ws || !d_query_codes || !hit_count) {
        set_error("alae_search_device: null argument");
        return ALAE_E_ARG;
    }
    if (!launch_shapes_ok(opts, "alae_search_device")) return ALAE_E_ARG;
    HIP_TRY(hipSetDevice(ws->device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(ws->ev0, s));
    uint64_t cnt = 0;
    alae_status st = run_search(ws, d_query_codes, m, nullptr, 1, scoring, H, opts, s, &cnt);
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

alae_status alae_autotune(alae_workspace *ws, const uint8_t *d_query_codes, size_t m, const alae_scoring *scoring,
                          int32_t H, alae_search_opts *opts, int32_t reps, void *stream, alae_tune_report *report) {
    if (!ws || !d_query_codes || !opts || !report || reps < 1) {
        set_error("alae_autotune: null argument or reps < 1");
        return ALAE_E_ARG;
    }
    if (!launch_shapes_ok(opts, "alae_autotune")) return ALAE_E_ARG;
    alae_search_opts o = *opts;
    o.trace = nullptr;  // tracing would change what is timed
    if (!o.level_stage) o.level_stage = kStageDefault;
    if (!o.wide_blocks_per_cu) o.wide_blocks_per_cu = 3;
    if (!o.lane_waves_per_cu) o.lane_waves_per_cu = 8;
    memset(report, 0, sizeof(*report));
    size_t want = 0;
    bool have = false;
    // mean device time of `reps` searches with the shapes of c; every search must give the same hit count
    auto timed = [&](const alae_search_opts &c, double *ms) -> alae_status {
        alae_stats st;
        alae_search_opts r = c;
        r.stats = &st;
        double sum = 0.0;
        for (int i = 0; i < reps; ++i) {
            size_t cnt = 0;
            memset(&st, 0, sizeof(st));
            const alae_status e = alae_search_device(ws, d_query_codes, m, scoring, H, &r, stream, &cnt);
            if (e != ALAE_OK) return e;
            if (have && cnt != want) {
                set_error("alae_autotune: hit count changed with the launch shapes (%zu, %zu)", cnt, want);
                return ALAE_E_INTERNAL;
            }
            want = cnt;
            have = true;
            sum += st.device_ms;
        }
        *ms = sum / reps;
        if (report->trials < (int32_t)(sizeof(report->trial) / sizeof(report->trial[0]))) {
            alae_tune_trial &tr = report->trial[report->trials++];
            tr.level_stage = c.level_stage;
            tr.wide_blocks_per_cu = c.wide_blocks_per_cu;
            tr.lane_waves_per_cu = c.lane_waves_per_cu;
            tr.level_graph = c.level_graph;
            tr.ms = *ms;
        }
        return ALAE_OK;
    };
    double warm = 0.0;
    alae_status st = timed(o, &warm);  // warm-up: buffers grow to the query's needs
    if (st != ALAE_OK) return st;
    report->trials = 0;
    double best_ms = 0.0;
    if ((st = timed(o, &best_ms)) != ALAE_OK) return st;
    report->default_ms = best_ms;
    // coordinate descent over the four shapes; a change must win by 1%
    const int32_t wide_c[] = {2, 3, 4, 6}, lane_c[] = {4, 8, 12}, stage_c[] = {2, 4, 8}, graph_c[] = {0, 8};
    for (int pass = 0; pass < 4; ++pass) {
        const int32_t *cand = pass == 0 ? wide_c : pass == 1 ? lane_c : pass == 2 ? stage_c : graph_c;
        const int nc = pass == 0 ? 4 : pass == 3 ? 2 : 3;
        const int32_t start = pass == 0   ? o.wide_blocks_per_cu
                              : pass == 1 ? o.lane_waves_per_cu
                              : pass == 2 ? o.level_stage
                                          : o.level_graph;
        for (int i = 0; i < nc; ++i) {
            if (cand[i] == start) continue;  // timed already
            alae_search_opts c = o;
            int32_t &field = pass == 0   ? c.wide_blocks_per_cu
                             : pass == 1 ? c.lane_waves_per_cu
                             : pass == 2 ? c.level_stage
                                         : c.level_graph;
            field = cand[i];
            double ms = 0.0;
            if ((st = timed(c, &ms)) != ALAE_OK) return st;
            if (ms < 0.99 * best_ms) {
                best_ms = ms;
                o = c;
            }
        }
    }
    report->best_ms = best_ms;
    opts->level_stage = o.level_stage;
    opts->wide_blocks_per_cu = o.wide_blocks_per_cu;
    opts->lane_waves_per_cu = o.lane_waves_per_cu;
    opts->level_graph = o.level_graph;
    return ALAE_OK;
}

}  // extern "C"

namespace alae {

// Statistics of several searches added up (the deepest depths kept).
static void add_stats(alae_stats &to, const alae_stats &x) {
#define ALAE_ADD(f) to.f += x.f
    ALAE_ADD(nodes);
    ALAE_ADD(entries);
    ALAE_ADD(entries_diag);
    ALAE_ADD(entries_gap2);
    ALAE_ADD(entries_gap3);
    ALAE_ADD(dominated);
    ALAE_ADD(emitted);
    ALAE_ADD(hits);
    ALAE_ADD(levels);
    ALAE_ADD(retries);
    ALAE_ADD(occ_reads);
    ALAE_ADD(sa_reads);
    ALAE_ADD(text_reads);
    ALAE_ADD(frontier_bytes);
    ALAE_ADD(level_launches);
    ALAE_ADD(level_ms);
    ALAE_ADD(start_ms);
    ALAE_ADD(general_ms);
    ALAE_ADD(wide_ms);
    ALAE_ADD(chain_steps);
    ALAE_ADD(wide_steps);
    ALAE_ADD(promoted);
    ALAE_ADD(dominated_gapped);
    ALAE_ADD(chain_bytes);
    ALAE_ADD(merge_ms);
    ALAE_ADD(reused);
    ALAE_ADD(replay_chains);
    ALAE_ADD(partitioned);
    ALAE_ADD(leftover);
    ALAE_ADD(order_ms);
    ALAE_ADD(level_lane_ms);
    ALAE_ADD(level_lane_launches);
    ALAE_ADD(tail_chains);
    ALAE_ADD(wide_entries);
    ALAE_ADD(dominated_qgram);
    ALAE_ADD(live_ms);
    ALAE_ADD(device_levels);
    ALAE_ADD(graph_captures);
#undef ALAE_ADD
    to.max_depth = std::max(to.max_depth, x.max_depth);
    to.tail_depth = std::max(to.tail_depth, x.tail_depth);
    to.wide_max_steps = std::max(to.wide_max_steps, x.wide_max_steps);
    if (x.wide_slowest_ms > to.wide_slowest_ms) {
        to.wide_slowest_ms = x.wide_slowest_ms;
        to.wide_slowest_rows = x.wide_slowest_rows;
        to.wide_slowest_start_ms = x.wide_slowest_start_ms;
    }
}

constexpr uint64_t kBatchColumns = 1ull << 19;

}  // namespace alae

extern "C" {

alae_status alae_search_device_batch(alae_workspace *ws, const uint8_t *d_query_codes, const size_t *lens, size_t k,
                                     const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                                     void *stream, size_t *hit_count) {
    if (!launch_shapes_ok(opts, "alae_search_device_batch")) return ALAE_E_ARG;
    if (!ws || !d_query_codes || !lens || !hit_count || k == 0) {
        set_error("alae_search_device_batch: null argument or empty batch");
        return ALAE_E_ARG;
    }
    std::vector<uint64_t> seg;
    uint64_t m = 0;
    for (size_t i = 0; i < k; ++i) {
        seg.push_back((uint64_t)lens[i]);
        m += lens[i];
    }
    // groups of consecutive queries of at most `budget` columns share one traversal: the
    // frontier of a traversal grows with the columns it serves
    const uint64_t budget = (opts && opts->batch_columns) ? opts->batch_columns : kBatchColumns;
    std::vector<uint64_t> gfirst;  // first query of every group
    {
        uint64_t cols = 0;
        for (uint64_t i = 0; i < k; ++i) {
            if (i == 0 || (cols > 0 && cols + seg[i] > budget)) {
                gfirst.push_back(i);
                cols = 0;
            }
            cols += seg[i];
        }
        gfirst.push_back(k);
    }
    HIP_TRY(hipSetDevice(ws->device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(ws->ev0, s));
    uint64_t cnt = 0;
    alae_status st;
    const size_t ngroups = gfirst.size() - 1;
    if (ngroups == 1) {
        st = run_search(ws, d_query_codes, m, seg.data(), (uint64_t)k, scoring, H, opts, s, &cnt);
        if (st != ALAE_OK) return st;
        if (k == 1) {  // a batch of one is a plain search
            ws->h_off.assign({0, cnt});
        }
    } else {
        // every group's result is appended to the accumulated result, in query order
        alae_stats total;
        memset(&total, 0, sizeof(total));
        alae_stats one;
        if (opts && opts->trace) {
            set_error("alae_search_device_batch: a trace needs the batch in one traversal (raise batch_columns)");
            return ALAE_E_ARG;
        }
        alae_search_opts o = opts ? *opts : alae_search_opts{};
        if (!opts) {
            o.use_domination = o.use_score_filter = o.use_qprefix = 1;
        }
        o.stats = &one;
        std::vector<uint64_t> off;
        off.reserve(k + 1);
        uint64_t col0 = 0;
        for (size_t g = 0; g < ngroups; ++g) {
            const uint64_t q0 = gfirst[g], q1 = gfirst[g + 1];
            uint64_t mg = 0;
            for (uint64_t i = q0; i < q1; ++i) mg += seg[i];
            memset(&one, 0, sizeof(one));
            uint64_t cg = 0;
            st = run_search(ws, d_query_codes + col0, mg, seg.data() + q0, q1 - q0, scoring, H, &o, s, &cg);
            if (st != ALAE_OK) return st;
            if (q1 - q0 == 1) ws->h_off.assign({0, cg});
            if ((st = grow_pair(ws->acc_keys, ws->acc_scores, ws->acc_cap, cnt + cg, cnt, s)) != ALAE_OK) return st;
            if (cg > 0) {
                HIP_TRY(hipMemcpyAsync(ws->acc_keys + cnt, ws->res_keys, cg * sizeof(uint64_t),
                                       hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipMemcpyAsync(ws->acc_scores + cnt, ws->res_scores, cg * sizeof(uint32_t),
                                       hipMemcpyDeviceToDevice, s));
            }
            for (uint64_t i = 0; i < q1 - q0; ++i) off.push_back(cnt + ws->h_off[i]);
            cnt += cg;
            col0 += mg;
            add_stats(total, one);
        }
        off.push_back(cnt);
        HIP_TRY(hipStreamSynchronize(s));
        std::swap(ws->res_keys, ws->acc_keys);
        std::swap(ws->res_scores, ws->acc_scores);
        std::swap(ws->res_cap, ws->acc_cap);
        ws->res_count = cnt;
        ws->h_off = off;
        ws->nseg = k;
        if (opts && opts->stats) *opts->stats = total;
    }
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

alae_status alae_workspace_batch_offsets(const alae_workspace *ws, size_t *offsets, size_t k) {
    if (!ws || !offsets) {
        set_error("alae_workspace_batch_offsets: null argument");
        return ALAE_E_ARG;
    }
    if (ws->h_off.size() != k + 1 || ws->nseg != k) {
        set_error("alae_workspace_batch_offsets: the last search on this workspace was not a batch of %zu queries",
                  k);
        return ALAE_E_ARG;
    }
    for (size_t i = 0; i <= k; ++i) offsets[i] = (size_t)ws->h_off[i];
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
    HIP_TRY(hipMemcpyAsync(d_keys, ws->res_keys, ws->res_count * sizeof(uint64_t), hipMemcpyDefault, s));
    HIP_TRY(hipMemcpyAsync(d_scores, ws->res_scores, ws->res_count * sizeof(int32_t), hipMemcpyDefault, s));
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
    if (!launch_shapes_ok(opts, "alae_search")) return ALAE_E_ARG;
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
    {
        Scheme sch;
        alae_status vs = check_scoring(scoring, index->sigma, H, sch);
        if (vs != ALAE_OK) return vs;
    }
    // concatenate the non-empty queries (an empty query has no hits)
    std::vector<uint8_t> codes;
    std::vector<size_t> seg, which;
    for (size_t i = 0; i < k; ++i) {
        if (lens[i] == 0) continue;
        if (!queries[i]) {
            set_error("alae_search_batch: query %zu is NULL", i);
            return ALAE_E_ARG;
        }
        const size_t at = codes.size();
        try {
            codes.resize(at + lens[i]);
        } catch (const std::bad_alloc &) {
            set_error("out of host memory");
            return ALAE_E_NOMEM;
        }
        if (!encode(queries[i], lens[i], index->alphabet, codes.data() + at)) {
            set_error("alae_search_batch: query %zu holds a character outside the alphabet", i);
            return ALAE_E_ALPHABET;
        }
        seg.push_back(lens[i]);
        which.push_back(i);
    }
    auto empty_hits = [](alae_hits &h) -> bool {
        h.count = 0;
        h.query_end = (uint32_t *)malloc(sizeof(uint32_t));
        h.text_end = (uint64_t *)malloc(sizeof(uint64_t));
        h.score = (int32_t *)malloc(sizeof(int32_t));
        return h.query_end && h.text_end && h.score;
    };
    auto fail = [&](alae_status st) {
        for (size_t j = 0; j < k; ++j) alae_hits_free(&outs[j]);
        return st;
    };
    alae_workspace *ws = nullptr;
    alae_status st = ALAE_OK;
    alae_hits all;
    memset(&all, 0, sizeof(all));
    std::vector<size_t> off;
    if (!seg.empty()) {
        if ((st = alae_workspace_create(index, &ws)) != ALAE_OK) return st;
        std::unique_ptr<alae_workspace, void (*)(alae_workspace *)> guard(ws, alae_workspace_free);
        if ((st = grow(ws->d_query, ws->q_cap, codes.size(), false, 0, nullptr)) != ALAE_OK) return st;
        HIP_TRY(hipMemcpy(ws->d_query, codes.data(), codes.size(), hipMemcpyHostToDevice));
        size_t cnt = 0;
        if ((st = alae_search_device_batch(ws, ws->d_query, seg.data(), seg.size(), scoring, H, opts, nullptr,
                                           &cnt)) != ALAE_OK)
            return st;
        off.resize(seg.size() + 1);
        if ((st = alae_workspace_batch_offsets(ws, off.data(), seg.size())) != ALAE_OK) return st;
        if ((st = download_hits(ws, nullptr, &all)) != ALAE_OK) return st;
    }
    std::unique_ptr<alae_hits, void (*)(alae_hits *)> all_guard(&all, alae_hits_free);
    std::vector<bool> done(k, false);
    for (size_t g = 0; g < which.size(); ++g) {
        alae_hits &h = outs[which[g]];
        const size_t b = off[g], e = off[g + 1], n = e - b;
        const size_t alloc = n ? n : 1;
        h.count = n;
        h.query_end = (uint32_t *)malloc(alloc * sizeof(uint32_t));
        h.text_end = (uint64_t *)malloc(alloc * sizeof(uint64_t));
        h.score = (int32_t *)malloc(alloc * sizeof(int32_t));
        if (!h.query_end || !h.text_end || !h.score) {
            set_error("out of host memory");
            return fail(ALAE_E_NOMEM);
        }
        if (n) {
            memcpy(h.query_end, all.query_end + b, n * sizeof(uint32_t));
            memcpy(h.text_end, all.text_end + b, n * sizeof(uint64_t));
            memcpy(h.score, all.score + b, n * sizeof(int32_t));
        }
        done[which[g]] = true;
    }
    for (size_t i = 0; i < k; ++i) {
        if (done[i]) continue;
        if (!empty_hits(outs[i])) {
            set_error("out of host memory");
            return fail(ALAE_E_NOMEM);
        }
    }
    return ALAE_OK;
}

}  // extern "C"
