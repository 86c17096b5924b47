// FM-index of the reversed text built on the GPU (Section 5: the suffix array
// of T^-1 $ with the positions of T kept; Section 2.3: BWT, C and occ).  The
// arrays are the same as those of the host build (index_build.cpp); only the
// way the suffix array is found differs.
//
// Suffix array by prefix doubling (Manber and Myers 1993) over the library's
// own LSD radix sort.  S' is T^-1 with every code shifted up by one and the
// terminator 0 at the end.  Round 0 sorts every suffix by its first `per`
// symbols packed into one 64-bit key (zeros past the end; the terminator is
// unique and smallest, so a suffix that reaches it within `per` symbols is
// already told apart).  Afterwards each suffix i has a rank: the position of
// the first suffix of its group (suffixes with the same first h symbols).  A
// round takes only the suffixes whose group still holds several, and sorts
// them by (rank[i], rank[i + h]), which orders them by their first 2h symbols;
// groups keep their places in the array, so the sorted suffixes go back to
// the same positions.  A tied suffix never reaches the terminator within h
// symbols, so i + h is always inside S'.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "alae_internal.h"
#include "device_algos.h"

namespace alae {

namespace {

#define GPU_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            hipGetLastError();                                                                   \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
            return ALAE_E_DEVICE;                                                                \
        }                                                                                        \
    } while (0)

constexpr uint32_t kTB = 256;

inline uint32_t grid_for(uint64_t n) { return (uint32_t)((n + kTB - 1) / kTB); }

// Round 0 keys: suffix i of S' (length N = n + 1) packed as `per` symbols of
// `bits` bits, the first symbol highest: '$' (and past the end) 0, a record
// separator 1, character c as c + 2.
__global__ void k_sa_init(const uint8_t *text, uint64_t n, int bits, int per, uint64_t *keys, uint32_t *vals) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    uint64_t key = 0;
    for (int k = 0; k < per; ++k) {
        const uint64_t p = i + (uint64_t)k;
        uint32_t sym = 0u;
        if (p < n) {
            const uint32_t x = text[n - 1 - p];
            sym = x == kSepCode ? 1u : x + 2u;
        }
        key = (key << bits) | sym;
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
}

// flags[p] = 1 where a new group starts (key differs from the one before);
// flags[cnt] = 1 closes the last group.
__global__ void k_group_flags(const uint64_t *keys, uint64_t cnt, uint32_t *flags) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > cnt) return;
    flags[p] = (p == 0 || p == cnt || keys[p] != keys[p - 1]) ? 1u : 0u;
}

// gstart[g] = array position of the first element of group g.  gidx is the
// exclusive scan of flags; pos maps an element to its position in the suffix
// array (nullptr: the element's own index).
__global__ void k_group_starts(const uint32_t *flags, const uint32_t *gidx, const uint32_t *pos, uint64_t cnt,
                               uint32_t *gstart) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= cnt || !flags[p]) return;
    gstart[gidx[p]] = pos ? pos[p] : (uint32_t)p;
}

// rank[suffix] = start of its group; tied[p] = 1 when the group holds more
// than one element (tied[cnt] = 0 for the compaction scan).
__global__ void k_set_ranks(const uint32_t *flags, const uint32_t *gidx, const uint32_t *gstart,
                            const uint32_t *suffix, uint64_t cnt, uint32_t *rank, uint32_t *tied) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > cnt) return;
    if (p == cnt) {
        tied[p] = 0;
        return;
    }
    const uint32_t g = gidx[p] + flags[p] - 1;
    rank[suffix[p]] = gstart[g];
    tied[p] = (flags[p] && flags[p + 1]) ? 0u : 1u;
}

// out[tpos[p]] = position of element p, for the tied elements.
__global__ void k_compact_tied(const uint32_t *tied, const uint32_t *tpos, const uint32_t *pos, uint64_t cnt,
                               uint32_t *out) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= cnt || !tied[p]) return;
    out[tpos[p]] = pos ? pos[p] : (uint32_t)p;
}

// Keys of a doubling round for the tied positions U: (rank[i] << B) | rank[i + h].
__global__ void k_round_keys(const uint32_t *U, uint64_t cnt, const uint32_t *sa, const uint32_t *rank, uint64_t h,
                             int B, uint64_t *keys, uint32_t *vals) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt) return;
    const uint32_t i = sa[U[k]];
    keys[k] = ((uint64_t)rank[i] << B) | (uint64_t)rank[(uint64_t)i + h];
    vals[k] = i;
}

__global__ void k_put_back(const uint32_t *U, const uint32_t *vals, uint64_t cnt, uint32_t *sa) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cnt) sa[U[k]] = vals[k];
}

// Row h of the index: the text end of its occurrence and the character that
// follows it in T (Section 5, searches (2) and (3)); 0xFF marks the
// terminator, whose row is recorded.
__global__ void k_rows(const uint32_t *sa, const uint8_t *text, uint64_t n, uint32_t *sa_end, uint8_t *bwt,
                       uint64_t *dollar_row) {
    const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h > n) return;
    const uint64_t p = sa[h];
    sa_end[h] = p == n ? kNoPos : (uint32_t)(n - 1 - p);
    if (p == 0) {
        bwt[h] = 0xFF;
        *dollar_row = h;
    } else {
        bwt[h] = text[n - p];
    }
}

// Per occ block: count of every code (the terminator and separators are not counted).
// counts[c * nblocks + b].
__global__ void k_block_counts(const uint8_t *bwt, uint64_t N, int per_block, int sigma, uint64_t nblocks,
                               uint32_t *counts) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    uint32_t c[20];
    for (int k = 0; k < sigma; ++k) c[k] = 0;
    const uint64_t lo = b * (uint64_t)per_block;
    for (int k = 0; k < per_block; ++k) {
        const uint64_t h = lo + (uint64_t)k;
        if (h >= N) break;
        const uint8_t x = bwt[h];
        for (int q = 0; q < sigma; ++q) c[q] += (x == q) ? 1u : 0u;
    }
    for (int k = 0; k < sigma; ++k) counts[(uint64_t)k * nblocks + b] = c[k];
}

// Occ blocks: counts before the block (prefix[c * nblocks + b]), then the
// block's characters (DNA: 2-bit codes, the terminator as 0; protein: bytes,
// 0xFF for the terminator and for rows past the end).
__global__ void k_write_blocks(const uint8_t *bwt, uint64_t N, int sigma, bool packed, uint64_t nblocks,
                               const uint32_t *prefix, uint8_t *occ) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    if (packed) {
        DnaOccBlock blk;
        for (int c = 0; c < 4; ++c) blk.cnt[c] = prefix[(uint64_t)c * nblocks + b];
        for (int w = 0; w < 12; ++w) blk.bits[w] = 0;
        const uint64_t lo = b * (uint64_t)kDnaBlockChars;
        for (int k = 0; k < kDnaBlockChars; ++k) {
            const uint64_t h = lo + (uint64_t)k;
            if (h >= N) break;
            const uint8_t x = bwt[h];
            const uint32_t code = x == 0xFF ? 0u : x;
            blk.bits[k / 16] |= code << (2 * (k % 16));
        }
        reinterpret_cast<DnaOccBlock *>(occ)[b] = blk;
    } else {
        GenOccBlock blk;
        for (int c = 0; c < 20; ++c) blk.cnt[c] = c < sigma ? prefix[(uint64_t)c * nblocks + b] : 0u;
        const uint64_t lo = b * (uint64_t)kGenBlockChars;
        for (int k = 0; k < kGenBlockChars; ++k) {
            const uint64_t h = lo + (uint64_t)k;
            blk.ch[k] = h < N ? bwt[h] : (uint8_t)0xFF;
        }
        reinterpret_cast<GenOccBlock *>(occ)[b] = blk;
    }
}

int bit_len(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Device buffers of one build, released on every path out.
struct Bufs {
    std::vector<void *> ptrs;
    template <typename T>
    hipError_t get(T **p, uint64_t count) {
        *p = nullptr;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(p), std::max<uint64_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    void release(void *p) {
        for (auto &q : ptrs)
            if (q == p) {
                hipFree(q);
                q = nullptr;
            }
    }
    ~Bufs() {
        for (void *p : ptrs)
            if (p) hipFree(p);
    }
};

}  // namespace

bool device_present(int device) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        hipGetLastError();
        return false;
    }
    return device >= 0 && device < ndev;
}

// Build sa_end, occ, C and the terminator row of `idx` (whose text, n, sigma
// and device are set) on its GPU; the device copies stay resident (the index
// is marked as uploaded) and the host arrays are filled from them.
alae_status build_index_on_device(alae_index *idx) {
    const uint64_t n = idx->n;
    const uint64_t N = n + 1;
    const int sigma = idx->sigma;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || idx->device < 0 || idx->device >= ndev) {
        hipGetLastError();
        set_error("no HIP device %d for the index build", idx->device);
        return ALAE_E_DEVICE;
    }
    GPU_TRY(hipSetDevice(idx->device));
    hipStream_t s = nullptr;
    Bufs b;
    // the text with readable slack on both sides: it stays as the index's device text
    uint8_t *text_alloc = nullptr;
    GPU_TRY(hipMalloc(&text_alloc, n + 2 * 64));
    struct TextGuard {
        uint8_t **p;
        ~TextGuard() {
            if (*p) hipFree(*p);
        }
    } text_guard{&text_alloc};
    uint8_t *d_text = text_alloc + 64;
    GPU_TRY(hipMemsetAsync(text_alloc, 0, n + 2 * 64, s));
    GPU_TRY(hipMemcpyAsync(d_text, idx->text.data(), n, hipMemcpyHostToDevice, s));

    const bool packed = idx->occ_packed;
    const int bits = sigma == 4 ? 3 : 5;  // symbols 0 .. sigma + 1
    const int per = 63 / bits;
    const int B = std::max(1, bit_len(N));  // ranks are below N
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt, *scratch, *sa, *rank, *flags, *gidx, *gstart, *U, *U2;
    // N + 1 keys each: a key buffer later holds two arrays of N + 1 words
    GPU_TRY(b.get(&keys, N + 1));
    GPU_TRY(b.get(&keys_alt, N + 1));
    GPU_TRY(b.get(&vals, N));
    GPU_TRY(b.get(&vals_alt, N));
    GPU_TRY(b.get(&scratch, std::max(radix_scratch_words(N), scan_scratch_words(N + 1))));
    GPU_TRY(b.get(&rank, N));
    GPU_TRY(b.get(&flags, N + 1));
    GPU_TRY(b.get(&gidx, N + 1));
    GPU_TRY(b.get(&gstart, N));

    // round 0: every suffix by its first `per` symbols
    k_sa_init<<<grid_for(N), kTB, 0, s>>>(d_text, n, bits, per, keys, vals);
    GPU_TRY(hipGetLastError());
    bool alt = false;
    GPU_TRY(radix_sort_pairs(keys, vals, keys_alt, vals_alt, N, bits * per, scratch, &alt, s));
    uint64_t *ks = alt ? keys_alt : keys;
    sa = alt ? vals_alt : vals;  // the suffix array, refined in place from here on
    uint32_t *tmp_vals = alt ? vals : vals_alt;
    uint64_t *tmp_keys = alt ? keys : keys_alt;
    k_group_flags<<<grid_for(N + 1), kTB, 0, s>>>(ks, N, flags);
    GPU_TRY(scan_exclusive_u32(flags, gidx, N + 1, scratch, s));
    k_group_starts<<<grid_for(N), kTB, 0, s>>>(flags, gidx, nullptr, N, gstart);
    // tied flags and their scan: N + 1 words each, in the key buffer the sort left free
    uint32_t *tied = reinterpret_cast<uint32_t *>(tmp_keys);
    uint32_t *tpos = reinterpret_cast<uint32_t *>(tmp_keys) + (N + 1);
    k_set_ranks<<<grid_for(N + 1), kTB, 0, s>>>(flags, gidx, gstart, sa, N, rank, tied);
    GPU_TRY(scan_exclusive_u32(tied, tpos, N + 1, scratch, s));
    uint32_t cnt32 = 0;
    GPU_TRY(hipMemcpyAsync(&cnt32, tpos + N, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    GPU_TRY(hipStreamSynchronize(s));
    uint64_t cnt = cnt32;
    GPU_TRY(b.get(&U, std::max<uint64_t>(cnt, 1)));
    GPU_TRY(b.get(&U2, std::max<uint64_t>(cnt, 1)));
    k_compact_tied<<<grid_for(N), kTB, 0, s>>>(tied, tpos, nullptr, N, U);
    GPU_TRY(hipGetLastError());
    // the round buffers: tied suffixes only (the first round's arrays are free now)
    uint64_t *rk = ks, *rk_alt = tmp_keys;
    uint32_t *rv = tmp_vals;
    uint32_t *rv_alt = gstart;  // free from here on: the rounds keep their group starts in rgs
    uint32_t *rgs = nullptr;
    GPU_TRY(b.get(&rgs, std::max<uint64_t>(cnt, 1)));
    uint64_t h = (uint64_t)per;
    int rounds = 0;
    while (cnt > 0) {
        if (++rounds > 64) {
            set_error("suffix array rounds did not converge (internal error)");
            return ALAE_E_INTERNAL;
        }
        k_round_keys<<<grid_for(cnt), kTB, 0, s>>>(U, cnt, sa, rank, h, B, rk, rv);
        GPU_TRY(hipGetLastError());
        bool a2 = false;
        GPU_TRY(radix_sort_pairs(rk, rv, rk_alt, rv_alt, cnt, 2 * B, scratch, &a2, s));
        uint64_t *sk = a2 ? rk_alt : rk;
        uint32_t *sv = a2 ? rv_alt : rv;
        k_put_back<<<grid_for(cnt), kTB, 0, s>>>(U, sv, cnt, sa);
        k_group_flags<<<grid_for(cnt + 1), kTB, 0, s>>>(sk, cnt, flags);
        GPU_TRY(scan_exclusive_u32(flags, gidx, cnt + 1, scratch, s));
        k_group_starts<<<grid_for(cnt), kTB, 0, s>>>(flags, gidx, U, cnt, rgs);
        // tied / tpos live in the half of the key buffer the sort did not leave its result in
        uint32_t *t_tied = reinterpret_cast<uint32_t *>(a2 ? rk : rk_alt);
        uint32_t *t_pos = t_tied + (cnt + 1);
        k_set_ranks<<<grid_for(cnt + 1), kTB, 0, s>>>(flags, gidx, rgs, sv, cnt, rank, t_tied);
        GPU_TRY(scan_exclusive_u32(t_tied, t_pos, cnt + 1, scratch, s));
        GPU_TRY(hipMemcpyAsync(&cnt32, t_pos + cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        GPU_TRY(hipStreamSynchronize(s));
        const uint64_t next = cnt32;
        k_compact_tied<<<grid_for(cnt), kTB, 0, s>>>(t_tied, t_pos, U, cnt, U2);
        GPU_TRY(hipGetLastError());
        std::swap(U, U2);
        cnt = next;
        h *= 2;
    }
    // the round arrays are no longer needed
    b.release(U);
    b.release(U2);
    b.release(rgs);
    b.release(flags);
    b.release(gidx);
    b.release(gstart);
    b.release(rank);

    // rows: SA of text ends and BWT
    uint32_t *d_sa_end = nullptr;
    GPU_TRY(hipMalloc(&d_sa_end, N * sizeof(uint32_t)));
    struct SaGuard {
        uint32_t **p;
        ~SaGuard() {
            if (*p) hipFree(*p);
        }
    } sa_guard{&d_sa_end};
    uint8_t *bwt = reinterpret_cast<uint8_t *>(tmp_vals);  // N bytes fit in N words
    uint64_t *d_dollar = reinterpret_cast<uint64_t *>(scratch);
    k_rows<<<grid_for(N), kTB, 0, s>>>(sa, d_text, n, d_sa_end, bwt, d_dollar);
    GPU_TRY(hipGetLastError());
    uint64_t dollar_row = 0;
    GPU_TRY(hipMemcpyAsync(&dollar_row, d_dollar, sizeof(uint64_t), hipMemcpyDeviceToHost, s));

    // occ blocks: per-block counts, a scan per code, then the blocks
    const int per_block = packed ? kDnaBlockChars : kGenBlockChars;
    const uint64_t nblocks = (N + per_block - 1) / per_block;
    const uint64_t occ_bytes = nblocks * (packed ? sizeof(DnaOccBlock) : sizeof(GenOccBlock));
    uint32_t *counts = nullptr, *prefix = nullptr;
    GPU_TRY(b.get(&counts, (uint64_t)sigma * nblocks));
    GPU_TRY(b.get(&prefix, (uint64_t)sigma * nblocks));
    uint8_t *d_occ = nullptr;
    GPU_TRY(hipMalloc(&d_occ, occ_bytes));
    struct OccGuard {
        uint8_t **p;
        ~OccGuard() {
            if (*p) hipFree(*p);
        }
    } occ_guard{&d_occ};
    k_block_counts<<<grid_for(nblocks), kTB, 0, s>>>(bwt, N, per_block, sigma, nblocks, counts);
    GPU_TRY(hipGetLastError());
    for (int c = 0; c < sigma; ++c)
        GPU_TRY(scan_exclusive_u32(counts + (uint64_t)c * nblocks, prefix + (uint64_t)c * nblocks, nblocks, scratch + 2,
                                   s));
    k_write_blocks<<<grid_for(nblocks), kTB, 0, s>>>(bwt, N, sigma, packed, nblocks, prefix, d_occ);
    GPU_TRY(hipGetLastError());
    // C from the code totals
    std::vector<uint32_t> last_pre(sigma), last_cnt(sigma);
    for (int c = 0; c < sigma; ++c) {
        GPU_TRY(hipMemcpyAsync(&last_pre[c], prefix + (uint64_t)c * nblocks + nblocks - 1, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        GPU_TRY(hipMemcpyAsync(&last_cnt[c], counts + (uint64_t)c * nblocks + nblocks - 1, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
    }
    // host copies of the arrays
    try {
        idx->sa_end.resize(N);
        idx->occ.resize(occ_bytes);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory for the index arrays (n=%llu)", (unsigned long long)n);
        return ALAE_E_NOMEM;
    }
    GPU_TRY(hipMemcpyAsync(idx->sa_end.data(), d_sa_end, N * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    GPU_TRY(hipMemcpyAsync(idx->occ.data(), d_occ, occ_bytes, hipMemcpyDeviceToHost, s));
    GPU_TRY(hipStreamSynchronize(s));
    uint64_t acc = 1 + idx->nsep;  // the rows of '$' and of the separators come first
    for (int c = 0; c < sigma; ++c) {
        idx->C[c] = acc;
        acc += (uint64_t)last_pre[c] + last_cnt[c];
    }
    idx->C[sigma] = acc;
    if (acc != N) {
        set_error("index build: code totals add up to %llu, not %llu (internal error)", (unsigned long long)acc,
                  (unsigned long long)N);
        return ALAE_E_INTERNAL;
    }
    idx->nblocks = nblocks;
    idx->dollar_row = dollar_row;
    // the device copies become the index's resident arrays
    {
        std::lock_guard<std::mutex> lock(idx->mu);
        idx->d_text_alloc = text_alloc;
        idx->d_text = d_text;
        idx->d_sa = d_sa_end;
        idx->d_occ = d_occ;
        idx->on_device = true;
    }
    text_alloc = nullptr;
    d_sa_end = nullptr;
    d_occ = nullptr;
    return ALAE_OK;
}

}  // namespace alae
