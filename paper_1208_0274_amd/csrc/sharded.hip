// Text-sharded index (for texts beyond one suffix array's 32-bit reach, or
// larger than the device memory kept for one index).  Shard s owns the text
// ends [s*L, min(n, (s+1)*L)) and indexes the text from `overlap` characters
// before its first owned end.  By Theorem 1 (Equation 1) an alignment that
// scores at least H spans at most L_max text characters, so when
// overlap >= L_max - 1 every hit with an owned end is found in the shard with
// the same score as in the whole text; the shards' hits are disjoint and their
// union is the whole text's hit set.  Each shard is searched on the device,
// its owned hits get global 64-bit text ends, and the union is sorted by
// (query end, text end) with the library's radix sort, all on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "alae_internal.h"
#include "device_algos.h"

struct alae_sharded {
    uint64_t n = 0;
    int alphabet = 0;
    int device = 0;
    uint64_t shard_len = 0, overlap = 0;
    uint32_t max_resident = 0;
    std::vector<alae_index *> shards;
    std::vector<uint64_t> first;  // first text position each shard indexes
    std::vector<uint64_t> own_lo; // first owned text end of each shard
};

namespace alae {
namespace {

#define SH_TRY(expr)                                                                             \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            hipGetLastError();                                                                   \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
            return ALAE_E_DEVICE;                                                                \
        }                                                                                        \
    } while (0)

// Owned hits of one shard: flag[i] = 1 when the hit's text end (local + first)
// is at least own_lo (the shard's result ends are all below its owned range's end).
__global__ void k_owned_flags(const uint64_t *keys, uint64_t cnt, uint64_t min_local, uint32_t *flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > cnt) return;
    flags[i] = (i < cnt && (keys[i] & 0xFFFFFFFFull) >= min_local) ? 1u : 0u;
}

// Append owned hits at base + pos[i]: key (query end << tbits) | global text end.
__global__ void k_owned_append(const uint64_t *keys, const int32_t *scores, uint64_t cnt, const uint32_t *flags,
                               const uint32_t *pos, uint64_t first, int tbits, uint64_t base, uint64_t *okeys,
                               uint32_t *oscores) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt || !flags[i]) return;
    const uint64_t k = keys[i];
    const uint64_t t = (k & 0xFFFFFFFFull) + first;
    okeys[base + pos[i]] = ((k >> 32) << tbits) | t;
    oscores[base + pos[i]] = (uint32_t)scores[i];
}

template <typename T>
hipError_t ensure(T *&p, uint64_t &cap, uint64_t need, bool keep, uint64_t keep_n) {
    if (need <= cap && p) return hipSuccess;
    uint64_t nc = cap ? cap : 1024;
    while (nc < need) nc *= 2;
    T *q = nullptr;
    hipError_t e = hipMalloc(&q, nc * sizeof(T));
    if (e != hipSuccess) return e;
    if (keep && p && keep_n) {
        e = hipMemcpy(q, p, keep_n * sizeof(T), hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
            hipFree(q);
            return e;
        }
    }
    if (p) hipFree(p);
    p = q;
    cap = nc;
    return hipSuccess;
}

struct DevBufs {
    uint64_t *keys = nullptr, *keys_alt = nullptr;
    uint32_t *scores = nullptr, *scores_alt = nullptr, *flags = nullptr, *pos = nullptr, *scratch = nullptr;
    uint64_t kcap = 0, kacap = 0, scap = 0, sacap = 0, fcap = 0, pcap = 0, xcap = 0;
    uint8_t *query = nullptr;
    uint64_t qcap = 0;
    ~DevBufs() {
        hipFree(keys);
        hipFree(keys_alt);
        hipFree(scores);
        hipFree(scores_alt);
        hipFree(flags);
        hipFree(pos);
        hipFree(scratch);
        hipFree(query);
    }
};

int bits_of(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

}  // namespace
}  // namespace alae

using namespace alae;

extern "C" {

alae_status alae_sharded_build(const uint8_t *codes, uint64_t n, alae_alphabet alphabet, uint64_t shard_len,
                               uint64_t overlap, uint32_t max_resident, const alae_index_opts *opts,
                               alae_sharded **out) {
    if (!codes || !out || n == 0 || shard_len == 0) {
        set_error("alae_sharded_build: null argument, empty text or zero shard length");
        return ALAE_E_ARG;
    }
    if (shard_len + overlap >= 0x7FFFFFFEull) {
        set_error("alae_sharded_build: a shard of %llu + %llu characters exceeds one index",
                  (unsigned long long)shard_len, (unsigned long long)overlap);
        return ALAE_E_TOO_LONG;
    }
    if (n >= (1ull << 36)) {
        set_error("alae_sharded_build: texts of 2^36 characters or more are not supported");
        return ALAE_E_TOO_LONG;
    }
    std::unique_ptr<alae_sharded> sh(new (std::nothrow) alae_sharded());
    if (!sh) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    sh->n = n;
    sh->alphabet = alphabet;
    sh->device = opts ? opts->device : 0;
    sh->shard_len = shard_len;
    sh->overlap = overlap;
    sh->max_resident = max_resident;
    auto cleanup = [&]() {
        for (alae_index *x : sh->shards) alae_index_free(x);
        sh->shards.clear();
    };
    for (uint64_t lo = 0; lo < n; lo += shard_len) {
        const uint64_t first = lo > overlap ? lo - overlap : 0;
        const uint64_t end = std::min(n, lo + shard_len);
        alae_index *x = nullptr;
        const alae_status st = alae_index_build_codes(codes + first, end - first, alphabet, opts, &x);
        if (st != ALAE_OK) {
            cleanup();
            return st;
        }
        sh->shards.push_back(x);
        sh->first.push_back(first);
        sh->own_lo.push_back(lo);
        // an index built on the GPU stays there; beyond the residency limit it goes back to the host
        if (max_resident && sh->shards.size() > max_resident) release_device(x);
    }
    *out = sh.release();
    return ALAE_OK;
}

void alae_sharded_free(alae_sharded *sh) {
    if (!sh) return;
    for (alae_index *x : sh->shards) alae_index_free(x);
    delete sh;
}

alae_status alae_sharded_search(const alae_sharded *sh, const char *query, size_t m, const alae_scoring *scoring,
                                int32_t H, const alae_search_opts *opts, alae_hits *out) {
    if (!sh || !query || !out || m == 0 || !scoring) {
        set_error("alae_sharded_search: null argument or empty query");
        return ALAE_E_ARG;
    }
    // Theorem 1: every hit's alignment spans at most L_max text characters
    int64_t smax = scoring->sa;
    if (scoring->use_matrix && scoring->matrix) {
        const int sigma = alphabet_sigma(sh->alphabet);
        smax = scoring->matrix[0];
        for (int k = 0; k < sigma * sigma; ++k) smax = std::max<int64_t>(smax, scoring->matrix[k]);
    }
    if (scoring->ss >= 0 || smax <= 0 || H < 1) {
        set_error("alae_sharded_search: scoring outside the model of Section 2.1");
        return ALAE_E_SCORING;
    }
    const int64_t num = (int64_t)H - (smax * (int64_t)m + scoring->sg);
    int64_t q = num / scoring->ss;
    if ((num % scoring->ss != 0) && ((num < 0) != (scoring->ss < 0))) q -= 1;
    const uint64_t lmax = (uint64_t)std::max<int64_t>((int64_t)m, (int64_t)m + q);
    if (sh->shards.size() > 1 && lmax > sh->overlap + 1) {
        set_error("alae_sharded_search: L_max = %llu of this query exceeds the shard overlap %llu + 1",
                  (unsigned long long)lmax, (unsigned long long)sh->overlap);
        return ALAE_E_TOO_LONG;
    }
    std::vector<uint8_t> codes(m);
    if (!encode(query, m, sh->alphabet, codes.data())) {
        set_error("alae_sharded_search: query holds a character outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    SH_TRY(hipSetDevice(sh->device));
    DevBufs b;
    SH_TRY(ensure(b.query, b.qcap, m, false, 0));
    SH_TRY(hipMemcpy(b.query, codes.data(), m, hipMemcpyHostToDevice));
    const int tbits = std::max(1, bits_of(sh->n - 1));
    const int qbits = std::max(1, bits_of(m - 1));
    if (qbits + tbits > 64) {
        set_error("alae_sharded_search: query and text too long for one 64-bit hit key");
        return ALAE_E_TOO_LONG;
    }
    uint64_t total = 0;
    alae_stats agg;
    memset(&agg, 0, sizeof(agg));
    for (size_t s = 0; s < sh->shards.size(); ++s) {
        alae_index *x = sh->shards[s];
        alae_workspace *ws = nullptr;
        alae_status st = alae_workspace_create(x, &ws);  // puts the shard on the device
        if (st != ALAE_OK) return st;
        std::unique_ptr<alae_workspace, void (*)(alae_workspace *)> guard(ws, alae_workspace_free);
        alae_stats one;
        alae_search_opts o = opts ? *opts : alae_search_opts{};
        if (!opts) o.use_domination = o.use_score_filter = o.use_qprefix = 1;
        o.stats = &one;
        memset(&one, 0, sizeof(one));
        size_t cnt = 0;
        if ((st = alae_search_device(ws, b.query, m, scoring, H, &o, nullptr, &cnt)) != ALAE_OK) return st;
        if (opts && opts->stats) {
            agg.entries += one.entries;
            agg.nodes += one.nodes;
            agg.emitted += one.emitted;
            agg.device_ms += one.device_ms;
            agg.levels += one.levels;
            agg.max_depth = std::max(agg.max_depth, one.max_depth);
        }
        if (cnt > 0) {
            const uint64_t *dk = nullptr;
            const int32_t *ds = nullptr;
            size_t c2 = 0;
            if ((st = alae_workspace_result(ws, &dk, &ds, &c2)) != ALAE_OK) return st;
            SH_TRY(ensure(b.flags, b.fcap, cnt + 1, false, 0));
            SH_TRY(ensure(b.pos, b.pcap, cnt + 1, false, 0));
            SH_TRY(ensure(b.scratch, b.xcap, scan_scratch_words(cnt + 1), false, 0));
            const uint64_t min_local = sh->own_lo[s] - sh->first[s];
            const uint32_t g = (uint32_t)((cnt + 1 + 255) / 256);
            k_owned_flags<<<g, 256>>>(dk, cnt, min_local, b.flags);
            SH_TRY(hipGetLastError());
            SH_TRY(scan_exclusive_u32(b.flags, b.pos, cnt + 1, b.scratch, nullptr));
            uint32_t owned = 0;
            SH_TRY(hipMemcpy(&owned, b.pos + cnt, sizeof(uint32_t), hipMemcpyDeviceToHost));
            SH_TRY(ensure(b.keys, b.kcap, total + owned, true, total));
            SH_TRY(ensure(b.scores, b.scap, total + owned, true, total));
            k_owned_append<<<g, 256>>>(dk, ds, cnt, b.flags, b.pos, sh->first[s], tbits, total, b.keys, b.scores);
            SH_TRY(hipGetLastError());
            SH_TRY(hipDeviceSynchronize());
            total += owned;
        }
        guard.reset();
        if (sh->max_resident && s + 1 > sh->max_resident) release_device(x);  // stream shards through HBM
    }
    if (opts && opts->stats) {
        agg.hits = total;
        *opts->stats = agg;
    }
    // union of the shards' owned hits, sorted by (query end, text end)
    bool alt = false;
    if (total > 1) {
        SH_TRY(ensure(b.keys_alt, b.kacap, total, false, 0));
        SH_TRY(ensure(b.scores_alt, b.sacap, total, false, 0));
        SH_TRY(ensure(b.scratch, b.xcap, radix_scratch_words(total), false, 0));
        SH_TRY(radix_sort_pairs(b.keys, b.scores, b.keys_alt, b.scores_alt, total, qbits + tbits, b.scratch, &alt,
                                nullptr));
    }
    alae_hits h;
    memset(&h, 0, sizeof(h));
    const size_t alloc = total ? total : 1;
    h.count = total;
    h.query_end = (uint32_t *)malloc(alloc * sizeof(uint32_t));
    h.text_end = (uint64_t *)malloc(alloc * sizeof(uint64_t));
    h.score = (int32_t *)malloc(alloc * sizeof(int32_t));
    std::vector<uint64_t> keys;
    try {
        keys.resize(total);
    } catch (const std::bad_alloc &) {
        alae_hits_free(&h);
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    if (!h.query_end || !h.text_end || !h.score) {
        alae_hits_free(&h);
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    if (total) {
        if (hipMemcpy(keys.data(), alt ? b.keys_alt : b.keys, total * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(h.score, alt ? b.scores_alt : b.scores, total * sizeof(int32_t), hipMemcpyDeviceToHost) !=
                hipSuccess) {
            hipGetLastError();
            alae_hits_free(&h);
            set_error("copying hits to the host failed");
            return ALAE_E_DEVICE;
        }
        const uint64_t tmask = (1ull << tbits) - 1;
        for (uint64_t i = 0; i < total; ++i) {
            h.query_end[i] = (uint32_t)(keys[i] >> tbits);
            h.text_end[i] = keys[i] & tmask;
        }
    }
    *out = h;
    return ALAE_OK;
}

}  // extern "C"
