// Device primitives: exclusive scan, stable LSD radix sort, max-merge of hits.
// Written for wave64 (gfx950): ballots are 64-bit and a 256-thread block holds
// four waves.
#include <hip/hip_runtime.h>

#include "device_algos.h"

namespace alae {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // elements per block
constexpr int kWaves = kThreads / 64;

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of the 256 per-thread totals of a block; returns the prefix
// for this thread and writes the block total to *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void __launch_bounds__(kThreads) scan_tiles(const uint32_t *in, uint32_t *out, uint64_t n,
                                                       uint32_t *tile_sums) {
    const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        uint64_t i = base + k;
        v[k] = i < n ? in[i] : 0u;
        sum += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, &total);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) scan_add(uint32_t *out, uint64_t n, const uint32_t *tile_prefix) {
    const uint32_t add = tile_prefix[blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        uint64_t i = base + k;
        if (i < n) out[i] += add;
    }
}

// LSD radix sort with 11-bit digits (2048 bins): a block ranks a tile of
// 256 x ITEMS keys; ranks within a wave come from ballots, and only the bins a
// round touches are updated (by one leader lane per bin and wave).
constexpr int kDigit = 11;
constexpr int kBins = 1 << kDigit;
// Keys a thread takes per pass: 64 (tiles of 16384 keys), or 256 (tiles of
// 65536) for key-only sorts (packed hit records) of at least kBigSort keys,
// where a larger tile means a quarter of the per-tile histogram entries to
// write, scan and read back and still two or more blocks per CU.
constexpr int kSortItems = 64;
constexpr int kSortItemsBig = 256;
constexpr uint64_t kBigSort = 1ull << 25;
constexpr int kSortTile = kThreads * kSortItems;  // the smallest tile (sizes the scratch)

// Lanes of a wave holding the same digit: the peers mask (ballot per digit
// bit) and this lane's rank among them.
__device__ inline uint64_t digit_peers(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kDigit; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

// Per-block digit counts, one LDS atomic per key (grouping a wave's equal
// digits with ballots first was slower: the ballots form a chain of dependent
// instructions per key, while same-address LDS atomics are rare enough).
template <int ITEMS>
__global__ void __launch_bounds__(kThreads) radix_hist(const uint64_t *keys, uint64_t n, int shift, uint32_t *hist,
                                                       uint32_t nblocks) {
    __shared__ uint32_t cnt[kBins];
    for (int b = threadIdx.x; b < kBins; b += kThreads) cnt[b] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * ITEMS);
    constexpr int kBatch = 16;  // loads issued together
    for (int r0 = 0; r0 < ITEMS; r0 += kBatch) {
        uint64_t kk[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const uint64_t i = base + (uint64_t)(r0 + j) * kThreads + threadIdx.x;
            kk[j] = i < n ? keys[i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const uint64_t i = base + (uint64_t)(r0 + j) * kThreads + threadIdx.x;
            const bool valid = i < n;
            const uint32_t d = (uint32_t)(kk[j] >> shift) & (kBins - 1);
            if (valid) atomicAdd(&cnt[d], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kThreads) hist[(uint64_t)b * nblocks + blockIdx.x] = cnt[b];
}

// Stable scatter: elements of a tile are ranked in index order (round, wave,
// lane); offs holds the exclusive scan of the digit-major histogram.  VALS:
// 32-bit values move with the keys.
template <bool VALS, int ITEMS>
__global__ void __launch_bounds__(kThreads) radix_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                          uint32_t *vout, uint64_t n, int shift,
                                                          const uint32_t *offs, uint32_t nblocks) {
    __shared__ uint32_t run[kBins];
    __shared__ uint32_t wcnt[kWaves][kBins];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    for (int b = tid; b < kBins; b += kThreads) {
        run[b] = offs[(uint64_t)b * nblocks + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcnt[w][b] = 0;
    }
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * ITEMS);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t k_next = base + tid < n ? kin[base + tid] : 0ull;  // the next round's element, loaded early
    uint32_t v_next = (VALS && base + tid < n) ? vin[base + tid] : 0u;
    for (int r = 0; r < ITEMS; ++r) {
        const uint64_t i = base + (uint64_t)r * kThreads + tid;
        const bool valid = i < n;
        const uint64_t k = k_next;
        const uint32_t v = v_next;
        if (r + 1 < ITEMS) {
            const uint64_t i2 = i + kThreads;
            k_next = i2 < n ? kin[i2] : 0ull;
            if (VALS) v_next = i2 < n ? vin[i2] : 0u;
        }
        const uint32_t d = (uint32_t)(k >> shift) & (kBins - 1);
        const uint64_t peers = digit_peers(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        const uint32_t same = (uint32_t)__popcll(peers);
        const bool leader = valid && rank == 0;
        if (leader) wcnt[wave][d] = same;
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = k;
            if (VALS) vout[pos] = v;
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&run[d], same);
            wcnt[wave][d] = 0;
        }
        __syncthreads();
    }
}

__global__ void merge_flags(const uint64_t *keys, uint64_t n, uint32_t *flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
    if (i == n) flags[i] = 0u;
}

__global__ void merge_write(const uint64_t *keys, const uint32_t *scores, uint64_t n, const uint32_t *flags,
                            const uint32_t *pos, uint64_t *out_keys, uint32_t *out_scores, int low_bits) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint64_t key = keys[i];
    int32_t best = (int32_t)scores[i];
    for (uint64_t j = i + 1; j < n && keys[j] == key; ++j) {
        int32_t s = (int32_t)scores[j];
        best = s > best ? s : best;
    }
    // packed keys (high part << low_bits | low part) go back to (high << 32) | low
    const uint64_t out = low_bits ? ((key >> low_bits) << 32) | (key & ((1ull << low_bits) - 1)) : key;
    out_keys[pos[i]] = out;
    out_scores[pos[i]] = (uint32_t)best;
}

// Hit records as one word: ((query end << low_bits | text end) << sb) | score,
// the padding key going to `pad` (above every real record); the block also
// counts the digits of the first radix pass (bits sb .. sb+10) of its tile,
// so that pass needs no histogram pass of its own.
template <int ITEMS>
__global__ void __launch_bounds__(kThreads) pack_records_hist(uint64_t *keys, const uint32_t *scores, uint64_t n,
                                                              int low_bits, int sb, uint64_t pad, uint32_t *hist,
                                                              uint32_t nblocks) {
    __shared__ uint32_t cnt[kBins];
    for (int b = threadIdx.x; b < kBins; b += kThreads) cnt[b] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * ITEMS);
    constexpr int kBatch = 16;
    for (int r0 = 0; r0 < ITEMS; r0 += kBatch) {
        uint64_t kk[kBatch];
        uint32_t ss[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const uint64_t i = base + (uint64_t)(r0 + j) * kThreads + threadIdx.x;
            kk[j] = i < n ? keys[i] : 0ull;
            ss[j] = i < n ? scores[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const uint64_t i = base + (uint64_t)(r0 + j) * kThreads + threadIdx.x;
            const bool valid = i < n;
            const uint64_t k = kk[j];
            const uint64_t rec =
                k == ~0ull ? pad : ((((k >> 32) << low_bits) | (k & 0xFFFFFFFFull)) << sb) | (uint64_t)ss[j];
            if (valid) keys[i] = rec;
            const uint32_t d = (uint32_t)(rec >> sb) & (kBins - 1);
            if (valid) atomicAdd(&cnt[d], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kThreads) hist[(uint64_t)b * nblocks + blockIdx.x] = cnt[b];
}

// Max-merge of packed records in two passes over tiles of kTile records
// (kItems consecutive records a thread): count the records that start a new
// key per tile, then (after a scan of the tile counts) write one record per
// key at its place.  A group's largest score is found by reading on from its
// first record.
// The tile's records go through LDS: loaded with coalesced reads, then each
// thread takes kItems consecutive ones.
__device__ inline void load_tile(const uint64_t *recs, uint64_t n, uint64_t tile, uint64_t *s_rec) {
    for (int k = threadIdx.x; k < kTile; k += kThreads) {
        const uint64_t i = tile + k;
        s_rec[k] = i < n ? recs[i] : 0ull;
    }
    __syncthreads();
}

__device__ inline uint32_t group_starts(const uint64_t *recs, const uint64_t *s_rec, uint64_t n, int sb,
                                        uint64_t tile, bool (&st)[kItems]) {
    const int k0 = threadIdx.x * kItems;
    const uint64_t first = tile + k0;
    uint64_t prev = ~0ull;
    if (k0 > 0)
        prev = s_rec[k0 - 1] >> sb;
    else if (first > 0 && first <= n)
        prev = recs[first - 1] >> sb;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t i = first + k;
        const uint64_t key = s_rec[k0 + k] >> sb;
        st[k] = i < n && (i == 0 || key != prev);
        c += st[k] ? 1u : 0u;
        prev = key;
    }
    return c;
}

__global__ void __launch_bounds__(kThreads) merge_count(const uint64_t *recs, uint64_t n, int sb,
                                                        uint32_t *tile_counts) {
    __shared__ uint64_t s_rec[kTile];
    const uint64_t tile = (uint64_t)blockIdx.x * kTile;
    load_tile(recs, n, tile, s_rec);
    bool st[kItems];
    const uint32_t c = group_starts(recs, s_rec, n, sb, tile, st);
    uint32_t total;
    block_exclusive_scan(c, &total);
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = total;
    if (blockIdx.x == 0 && threadIdx.x == 0) tile_counts[gridDim.x] = 0u;  // the scan leaves the total there
}

// One output record per key that starts in this tile, with the largest score
// of its group (read on past the tile's end when the group continues);
// written through LDS so that the tile's outputs leave as one coalesced run.
__global__ void __launch_bounds__(kThreads) merge_emit(const uint64_t *recs, uint64_t n, int sb, int low_bits,
                                                       const uint32_t *tile_prefix, uint64_t *out_keys,
                                                       uint32_t *out_scores) {
    __shared__ uint64_t s_rec[kTile];  // the tile's records, then its output keys
    __shared__ uint32_t s_score[kTile];
    const uint64_t tile = (uint64_t)blockIdx.x * kTile;
    load_tile(recs, n, tile, s_rec);
    bool st[kItems];
    const uint32_t c = group_starts(recs, s_rec, n, sb, tile, st);
    uint32_t total;
    uint32_t pos = block_exclusive_scan(c, &total);
    const uint64_t smask = (1ull << sb) - 1;
    const int k0 = threadIdx.x * kItems;
    uint64_t okey[kItems];
    uint32_t oscore[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        okey[k] = 0;
        oscore[k] = 0;
        if (!st[k]) continue;
        const uint64_t key = s_rec[k0 + k] >> sb;
        uint64_t best = s_rec[k0 + k] & smask;
        int j = k0 + k + 1;
        for (; j < kTile && tile + j < n && (s_rec[j] >> sb) == key; ++j) {
            const uint64_t s = s_rec[j] & smask;
            best = s > best ? s : best;
        }
        if (j == kTile)  // the group may go on in the next tile
            for (uint64_t g = tile + kTile; g < n && (recs[g] >> sb) == key; ++g) {
                const uint64_t s = recs[g] & smask;
                best = s > best ? s : best;
            }
        okey[k] = ((key >> low_bits) << 32) | (key & ((1ull << low_bits) - 1));
        oscore[k] = (uint32_t)best;
    }
    __syncthreads();  // every group has been read: the record tile takes the outputs
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (!st[k]) continue;
        s_rec[pos] = okey[k];
        s_score[pos] = oscore[k];
        ++pos;
    }
    __syncthreads();
    const uint64_t out = tile_prefix[blockIdx.x];
    for (uint32_t k = threadIdx.x; k < total; k += kThreads) {
        out_keys[out + k] = s_rec[k];
        out_scores[out + k] = s_score[k];
    }
}

__global__ void repack_keys(uint64_t *keys, uint64_t n, int low_bits, uint64_t pad) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    keys[i] = k == ~0ull ? pad : ((k >> 32) << low_bits) | (k & 0xFFFFFFFFull);
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

const uint32_t kZero = 0;

}  // namespace

uint64_t scan_scratch_words(uint64_t n) {
    uint64_t words = 0;
    while (n > 1) {
        n = ceil_div(n, kTile);
        words += n + 1;
    }
    return words + 2;
}

hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t tiles = ceil_div(n, kTile);
    uint32_t *sums = tmp;
    scan_tiles<<<(uint32_t)tiles, kThreads, 0, s>>>(in, out, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || tiles == 1) return e;
    e = scan_exclusive_u32(sums, sums, tiles, tmp + tiles + 1, s);
    if (e != hipSuccess) return e;
    scan_add<<<(uint32_t)tiles, kThreads, 0, s>>>(out, n, sums);
    return hipGetLastError();
}

uint64_t radix_scratch_words(uint64_t n) {
    const uint64_t blocks = ceil_div(n ? n : 1, kSortTile);
    const uint64_t hist = (uint64_t)kBins * blocks;
    return hist + scan_scratch_words(hist);
}

static bool big_sort(uint64_t n) { return n >= kBigSort; }
static uint32_t sort_blocks(uint64_t n) {
    return (uint32_t)ceil_div(n, (uint64_t)kThreads * (big_sort(n) ? kSortItemsBig : kSortItems));
}

// Key-value sorts (query seeds, and hits that do not fit one word) keep the
// 64-key tiles at every size.
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n,
                            int bits, uint32_t *scratch, bool *result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n <= 1 || bits <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)ceil_div(n, kSortTile);
    uint32_t *hist = scratch;
    uint32_t *tmp = scratch + (uint64_t)kBins * blocks;
    uint64_t *kin = keys, *kout = keys_alt;
    uint32_t *vin = vals, *vout = vals_alt;
    bool alt = false;
    for (int shift = 0; shift < bits; shift += kDigit) {
        radix_hist<kSortItems><<<blocks, kThreads, 0, s>>>(kin, n, shift, hist, blocks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_exclusive_u32(hist, hist, (uint64_t)kBins * blocks, tmp, s);
        if (e != hipSuccess) return e;
        radix_scatter<true, kSortItems><<<blocks, kThreads, 0, s>>>(kin, vin, kout, vout, n, shift, hist, blocks);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(kin, kout);
        std::swap(vin, vout);
        alt = !alt;
    }
    *result_in_alt = alt;
    return hipSuccess;
}

// first_hist: the histogram of the first pass is already in the scratch.
static hipError_t radix_sort_keys_impl(uint64_t *keys, uint64_t *keys_alt, uint64_t n, int lo_bit, int bits,
                                       uint32_t *scratch, bool *result_in_alt, hipStream_t s, bool first_hist) {
    *result_in_alt = false;
    if (n <= 1 || bits <= 0) return hipSuccess;
    const bool big = big_sort(n);
    const uint32_t blocks = sort_blocks(n);
    uint32_t *hist = scratch;
    uint32_t *tmp = scratch + (uint64_t)kBins * blocks;
    uint64_t *kin = keys, *kout = keys_alt;
    bool alt = false;
    for (int shift = lo_bit; shift < lo_bit + bits; shift += kDigit) {
        if (!(first_hist && shift == lo_bit)) {
            if (big)
                radix_hist<kSortItemsBig><<<blocks, kThreads, 0, s>>>(kin, n, shift, hist, blocks);
            else
                radix_hist<kSortItems><<<blocks, kThreads, 0, s>>>(kin, n, shift, hist, blocks);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_exclusive_u32(hist, hist, (uint64_t)kBins * blocks, tmp, s);
        if (e != hipSuccess) return e;
        if (big)
            radix_scatter<false, kSortItemsBig><<<blocks, kThreads, 0, s>>>(kin, nullptr, kout, nullptr, n, shift,
                                                                            hist, blocks);
        else
            radix_scatter<false, kSortItems><<<blocks, kThreads, 0, s>>>(kin, nullptr, kout, nullptr, n, shift, hist,
                                                                         blocks);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(kin, kout);
        alt = !alt;
    }
    *result_in_alt = alt;
    return hipSuccess;
}

hipError_t radix_sort_keys(uint64_t *keys, uint64_t *keys_alt, uint64_t n, int lo_bit, int bits, uint32_t *scratch,
                           bool *result_in_alt, hipStream_t s) {
    return radix_sort_keys_impl(keys, keys_alt, n, lo_bit, bits, scratch, result_in_alt, s, false);
}

hipError_t pack_sort_hits(uint64_t *keys, const uint32_t *scores, uint64_t *keys_alt, uint64_t n, int low_bits,
                          int sb, int total_bits, uint32_t *scratch, bool *result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n == 0) return hipSuccess;
    const int all = total_bits + sb;
    const uint64_t pad = all >= 64 ? ~0ull : ((1ull << all) - 1);
    const uint32_t blocks = sort_blocks(n);  // the tiles of radix_sort_keys_impl's first pass
    if (big_sort(n))
        pack_records_hist<kSortItemsBig><<<blocks, kThreads, 0, s>>>(keys, scores, n, low_bits, sb, pad, scratch,
                                                                      blocks);
    else
        pack_records_hist<kSortItems><<<blocks, kThreads, 0, s>>>(keys, scores, n, low_bits, sb, pad, scratch,
                                                                   blocks);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return radix_sort_keys_impl(keys, keys_alt, n, sb, total_bits, scratch, result_in_alt, s, true);
}

hipError_t max_merge_packed(const uint64_t *recs, uint64_t n, int sb, int low_bits, uint64_t *out_keys,
                            uint32_t *out_scores, uint32_t *tiles, uint32_t *tmp, hipStream_t s) {
    const uint64_t nt = ceil_div(n, kTile);
    if (n == 0) return hipMemcpyAsync(tiles, &kZero, sizeof(uint32_t), hipMemcpyHostToDevice, s);
    merge_count<<<(uint32_t)nt, kThreads, 0, s>>>(recs, n, sb, tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive_u32(tiles, tiles, nt + 1, tmp, s);  // tiles[nt]: the distinct count
    if (e != hipSuccess) return e;
    merge_emit<<<(uint32_t)nt, kThreads, 0, s>>>(recs, n, sb, low_bits, tiles, out_keys, out_scores);
    return hipGetLastError();
}

uint64_t merge_tile_count(uint64_t n) { return ceil_div(n, kTile); }

hipError_t repack_hit_keys(uint64_t *keys, uint64_t n, int low_bits, int total_bits, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t pad = total_bits >= 64 ? ~0ull : ((1ull << total_bits) - 1);
    repack_keys<<<(uint32_t)ceil_div(n, 256), 256, 0, s>>>(keys, n, low_bits, pad);
    return hipGetLastError();
}

hipError_t max_merge_sorted(const uint64_t *keys, const uint32_t *scores, uint64_t n, uint64_t *out_keys,
                            uint32_t *out_scores, uint32_t *flags, uint32_t *pos, uint32_t *tmp,
                            hipStream_t s, int low_bits) {
    const uint32_t threads = 256;
    const uint32_t grid = (uint32_t)ceil_div(n + 1, threads);
    merge_flags<<<grid, threads, 0, s>>>(keys, n, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive_u32(flags, pos, n + 1, tmp, s);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    merge_write<<<(uint32_t)ceil_div(n, threads), threads, 0, s>>>(keys, scores, n, flags, pos, out_keys,
                                                                   out_scores, low_bits);
    return hipGetLastError();
}

}  // namespace alae
