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
// Host-side occ(c, i): number of c in BWT[0..i] (i may be -1).
uint64_t host_occ(const alae_index *idx, int c, int64_t i);
// Upload the index to its device (idempotent, thread-safe).
alae_status ensure_device(const alae_index *idx);
void release_device(const alae_index *idx);
}  // namespace alae
