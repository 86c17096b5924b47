// Host-callable device primitives written for this library: exclusive scan,
// LSD radix sort of (64-bit key, 32-bit value) pairs, and the max-merge of
// sorted hit records.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace alae {

// Scratch needed by scan_exclusive_u32 for n elements (in uint32 words).
uint64_t scan_scratch_words(uint64_t n);
// out[i] = sum of in[0..i-1]; in and out may alias.  tmp holds scan_scratch_words(n) words.
hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s);

// Scratch (uint32 words) for radix_sort_pairs on n elements.
uint64_t radix_scratch_words(uint64_t n);
// Stable LSD radix sort by the low `bits` bits of the keys, 11 bits per pass.
// (keys, vals) and (keys_alt, vals_alt) are ping-pong buffers of n elements;
// on return *result_in_alt says which pair holds the sorted data.
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n,
                            int bits, uint32_t *scratch, bool *result_in_alt, hipStream_t s);

// Stable LSD radix sort of bare 64-bit keys by bits [lo_bit, lo_bit + bits),
// 11 bits per pass; scratch as for radix_sort_pairs.
hipError_t radix_sort_keys(uint64_t *keys, uint64_t *keys_alt, uint64_t n, int lo_bit, int bits, uint32_t *scratch,
                           bool *result_in_alt, hipStream_t s);

// Hit keys (query end << 32) | text end become (query end << low_bits) | text
// end, and the padding key ~0 becomes 2^total_bits - 1 (above every real key),
// so that the sort reads total_bits bits only.
hipError_t repack_hit_keys(uint64_t *keys, uint64_t n, int low_bits, int total_bits, hipStream_t s);
// The same key with the score below it in one word when total_bits + sb <= 64:
// ((query end << low_bits | text end) << sb) | score, the padding record
// 2^(total_bits + sb) - 1; then sorted by bits [sb, sb + total_bits) (the
// packing kernel counts the first pass's digits).  Scratch as for
// radix_sort_pairs; *result_in_alt says whether keys_alt holds the result.
hipError_t pack_sort_hits(uint64_t *keys, const uint32_t *scores, uint64_t *keys_alt, uint64_t n, int low_bits,
                          int sb, int total_bits, uint32_t *scratch, bool *result_in_alt, hipStream_t s);

// Given hit records sorted by key, keep one record per key with the largest
// score (Algorithm 1's "keep the larger score").  flags/pos hold n+1 words
// each, tmp scan_scratch_words(n+1); pos[n] receives the distinct count.
// low_bits > 0: the keys are repacked and are written back in the unpacked form.
hipError_t max_merge_sorted(const uint64_t *keys, const uint32_t *scores, uint64_t n, uint64_t *out_keys,
                            uint32_t *out_scores, uint32_t *flags, uint32_t *pos, uint32_t *tmp,
                            hipStream_t s, int low_bits = 0);
// The same for records packed by pack_sort_hits: tiles holds
// merge_tile_count(n) + 1 words and receives the distinct count at index
// merge_tile_count(n); tmp scan_scratch_words(merge_tile_count(n) + 1).
hipError_t max_merge_packed(const uint64_t *recs, uint64_t n, int sb, int low_bits, uint64_t *out_keys,
                            uint32_t *out_scores, uint32_t *tiles, uint32_t *tmp, hipStream_t s);
uint64_t merge_tile_count(uint64_t n);

}  // namespace alae
