// Internal declarations shared by the host and device translation units of libalae.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "alae.h"

namespace alae {

// Occurrence blocks of the BWT (Section 2.3, backward search; Section 5).
// DNA: 64 bytes cover 192 BWT characters: the counts of each character in all
// earlier blocks, then 2-bit codes (character k of the block sits in word k/16
// at bit 2*(k%16)).  The terminator is stored as code 0 and corrected for by
// the dollar row.
constexpr int kDnaBlockChars = 192;
struct DnaOccBlock {
    uint32_t cnt[4];
    uint32_t bits[12];
};
static_assert(sizeof(DnaOccBlock) == 64, "DNA occ block must be one 64-byte granule");

// Protein (sigma <= 20): 128 bytes cover 48 BWT characters, one byte each;
// the terminator is 0xFF.
constexpr int kGenBlockChars = 48;
struct GenOccBlock {
    uint32_t cnt[20];
    uint8_t ch[48];
};
static_assert(sizeof(GenOccBlock) == 128, "protein occ block must be 128 bytes");

constexpr uint32_t kNoPos = 0xFFFFFFFFu;
// Code of the record separator in the text of a multi-record index (Section
// 2.2 concatenates the database's sequences into one text; the separator keeps
// every alignment inside one record).  Never a character of a query.
constexpr uint8_t kSepCode = 0xFE;

void set_error(const char *fmt, ...);
int alphabet_sigma(int alphabet);
// Map characters to codes; returns false on a character outside the alphabet.
bool encode(const char *s, size_t len, int alphabet, uint8_t *out);

}  // namespace alae

struct alae_index {
    uint64_t n = 0;
    int sigma = 0;
    int alphabet = 0;
    int device = 0;
    std::vector<uint8_t> text;     // codes, n
    std::vector<uint32_t> sa_end;  // n+1: 0-based text end of each BWT row, row of '$' = kNoPos
    std::vector<uint8_t> occ;      // occurrence blocks
    uint64_t nblocks = 0;
    uint64_t C[21] = {0};
    uint64_t dollar_row = 0;
    // multi-record texts: separators (kSepCode) between records, record starts
    uint64_t nsep = 0;
    std::vector<uint64_t> rec_start;
    // occ blocks: packed DNA (2-bit, DnaOccBlock) or one byte a character (GenOccBlock,
    // protein and every text with separators)
    bool occ_packed = true;

    // Device copy, created on first use.
    mutable std::mutex mu;
    mutable bool on_device = false;
    mutable uint8_t *d_text = nullptr;        // first character (inside d_text_alloc)
    mutable uint8_t *d_text_alloc = nullptr;  // text with readable slack on both sides
    mutable uint32_t *d_sa = nullptr;
    mutable uint8_t *d_occ = nullptr;
    mutable uint64_t *d_C = nullptr;
};

namespace alae {
// A fixed block of device memory that a search cuts all its buffers from
// (callers that cannot allocate): base, size in bytes, bytes handed out.
struct FixedRegion {
    uint8_t *base;
    uint64_t size;
    uint64_t used;
};
// A workspace bound to `bytes` bytes of device memory at `region` on `device`
// (its counters take the first few kilobytes); creates its stream and events.
alae_status region_workspace_create(int device, uint8_t *region, uint64_t bytes, alae_workspace **out);
// One search of a device-resident query on such a workspace, the sorted
// result copied to the caller's d_keys / d_scores (capacity records).
// *hit_count gets the result size, also when it exceeds capacity
// (ALAE_E_NOMEM).  `stream` is a hipStream_t.
alae_status region_search(alae_workspace *ws, const alae_index *idx, const uint8_t *d_query, uint64_t m,
                          const alae_scoring *scoring, int32_t H, const alae_search_opts *opts, void *stream,
                          uint64_t *d_keys, int32_t *d_scores, uint64_t capacity, uint64_t *hit_count);
// Free the buffers a workspace has grown (they grow again on the next search).
void workspace_trim(alae_workspace *ws);
// True when HIP device `device` exists.
bool device_present(int device);
// Build the suffix array, BWT, occ blocks and C of `idx` (text, n, sigma and
// device set) on its GPU; the device arrays stay resident and the host
// arrays are filled from them.
alae_status build_index_on_device(alae_index *idx);
// Host-side occ(c, i): number of c in BWT[0..i] (i may be -1).
uint64_t host_occ(const alae_index *idx, int c, int64_t i);
// Upload the index to its device (idempotent, thread-safe).
alae_status ensure_device(const alae_index *idx);
void release_device(const alae_index *idx);
}  // namespace alae
