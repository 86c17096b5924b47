// Host-side construction of the FM-index of the reversed text (Section 5).
//
// The text T (codes 0..sigma-1) is reversed and terminated: S = T^-1 $, with
// S[k] = T[n-1-k] for k < n and S[n] = $ (smallest).  Its suffix array is
// built with induced sorting (SA-IS, Nong, Zhang and Chan 2009).  For BWT row
// h the index keeps
//   sa_end[h] = n-1-SA[h]  -- the 0-based text position where the occurrence
//                             of the row's trie node ends (Section 5, search
//                             (2)); the terminator row holds kNoPos;
//   BWT[h]    = S[SA[h]-1] -- the text character right after that end, i.e.
//                             the character that extends the trie node by one
//                             (Section 5, search (3)); '$' when SA[h] = 0.
// C[c] = 1 + #(text characters < c).  Backward search appends a character c
// to the right of X:  [l, r] -> [C[c] + occ(c, l-1), C[c] + occ(c, r) - 1].
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <new>

#include "alae_internal.h"

namespace alae {

namespace {
thread_local std::string g_error;

// Induced sorting of the suffixes of s[0..n-1], where s[n-1] is the unique
// smallest symbol.  K is the alphabet size.  SA receives n positions.
template <typename Sym>
void induced_sort(const Sym *s, int32_t *SA, int32_t n, int32_t K) {
    if (n == 1) {
        SA[0] = 0;
        return;
    }
    std::vector<uint8_t> stype(n);  // 1: S-type suffix, 0: L-type
    stype[n - 1] = 1;
    for (int32_t i = n - 2; i >= 0; --i)
        stype[i] = (s[i] < s[i + 1] || (s[i] == s[i + 1] && stype[i + 1])) ? 1 : 0;
    auto lms = [&](int32_t i) { return i > 0 && stype[i] && !stype[i - 1]; };

    std::vector<int32_t> bucket(K);
    auto heads_or_tails = [&](bool tails) {
        std::fill(bucket.begin(), bucket.end(), 0);
        for (int32_t i = 0; i < n; ++i) bucket[s[i]]++;
        int32_t acc = 0;
        for (int32_t c = 0; c < K; ++c) {
            acc += bucket[c];
            bucket[c] = tails ? acc : acc - bucket[c];
        }
    };
    auto induce_ls = [&]() {
        heads_or_tails(false);
        for (int32_t i = 0; i < n; ++i) {
            int32_t p = SA[i] - 1;
            if (SA[i] > 0 && !stype[p]) SA[bucket[s[p]]++] = p;
        }
        heads_or_tails(true);
        for (int32_t i = n - 1; i >= 0; --i) {
            int32_t p = SA[i] - 1;
            if (SA[i] > 0 && stype[p]) SA[--bucket[s[p]]] = p;
        }
    };

    // 1. sort the LMS substrings by one round of induction
    heads_or_tails(true);
    std::fill(SA, SA + n, -1);
    for (int32_t i = 1; i < n; ++i)
        if (lms(i)) SA[--bucket[s[i]]] = i;
    induce_ls();

    // 2. gather the sorted LMS positions and name equal LMS substrings alike
    int32_t n1 = 0;
    for (int32_t i = 0; i < n; ++i)
        if (lms(SA[i])) SA[n1++] = SA[i];
    std::fill(SA + n1, SA + n, -1);
    int32_t names = 0, prev = -1;
    for (int32_t i = 0; i < n1; ++i) {
        int32_t pos = SA[i];
        bool differs = false;
        for (int32_t d = 0; d < n; ++d) {
            if (prev < 0 || s[pos + d] != s[prev + d] || stype[pos + d] != stype[prev + d]) {
                differs = true;
                break;
            }
            if (d > 0 && (lms(pos + d) || lms(prev + d))) break;
        }
        if (differs) {
            ++names;
            prev = pos;
        }
        SA[n1 + pos / 2] = names - 1;
    }
    for (int32_t i = n - 1, j = n - 1; i >= n1; --i)
        if (SA[i] >= 0) SA[j--] = SA[i];

    // 3. order the LMS suffixes (recursively if names repeat)
    int32_t *sa1 = SA;
    int32_t *s1 = SA + n - n1;
    if (names < n1) {
        induced_sort<int32_t>(s1, sa1, n1, names);
    } else {
        for (int32_t i = 0; i < n1; ++i) sa1[s1[i]] = i;
    }

    // 4. place the sorted LMS suffixes at their bucket tails and induce the rest
    heads_or_tails(true);
    for (int32_t i = 1, j = 0; i < n; ++i)
        if (lms(i)) s1[j++] = i;
    for (int32_t i = 0; i < n1; ++i) sa1[i] = s1[sa1[i]];
    std::fill(SA + n1, SA + n, -1);
    for (int32_t i = n1 - 1; i >= 0; --i) {
        int32_t p = SA[i];
        SA[i] = -1;
        SA[--bucket[s[p]]] = p;
    }
    induce_ls();
}

const char kDna[] = "ACGT";
const char kProtein[] = "ARNDCQEGHILKMFPSTWYV";

}  // namespace

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
}

const char *last_error_text() { return g_error.c_str(); }

int alphabet_sigma(int alphabet) { return alphabet == ALAE_DNA ? 4 : (alphabet == ALAE_PROTEIN ? 20 : 0); }

bool encode(const char *s, size_t len, int alphabet, uint8_t *out) {
    static uint8_t lut[2][256];
    static std::once_flag once;
    std::call_once(once, [] {
        memset(lut, 0xFF, sizeof(lut));
        for (int i = 0; i < 4; ++i) {
            lut[0][(uint8_t)kDna[i]] = (uint8_t)i;
            lut[0][(uint8_t)(kDna[i] + 32)] = (uint8_t)i;
        }
        for (int i = 0; i < 20; ++i) {
            lut[1][(uint8_t)kProtein[i]] = (uint8_t)i;
            lut[1][(uint8_t)(kProtein[i] + 32)] = (uint8_t)i;
        }
    });
    const uint8_t *t = lut[alphabet == ALAE_PROTEIN ? 1 : 0];
    for (size_t i = 0; i < len; ++i) {
        uint8_t c = t[(uint8_t)s[i]];
        if (c == 0xFF) return false;
        out[i] = c;
    }
    return true;
}

uint64_t host_occ(const alae_index *idx, int c, int64_t i) {
    if (i < 0) return 0;
    if (idx->occ_packed) {
        const DnaOccBlock *b = reinterpret_cast<const DnaOccBlock *>(idx->occ.data()) + i / kDnaBlockChars;
        int off = (int)(i % kDnaBlockChars);
        uint64_t cnt = b->cnt[c];
        for (int k = 0; k <= off; ++k) {
            int code = (b->bits[k / 16] >> (2 * (k % 16))) & 3;
            cnt += (code == c);
        }
        // the terminator is stored as code 0; block counts already leave it out
        const uint64_t bstart = (uint64_t)(i / kDnaBlockChars) * kDnaBlockChars;
        if (c == 0 && idx->dollar_row >= bstart && idx->dollar_row <= (uint64_t)i) cnt -= 1;
        return cnt;
    }
    const GenOccBlock *b = reinterpret_cast<const GenOccBlock *>(idx->occ.data()) + i / kGenBlockChars;
    int off = (int)(i % kGenBlockChars);
    uint64_t cnt = b->cnt[c];
    for (int k = 0; k <= off; ++k) cnt += (b->ch[k] == c);
    return cnt;
}

static alae_status build_from_codes(std::unique_ptr<alae_index> &idx) {
    const uint64_t n = idx->n;
    const int sigma = idx->sigma;
    const uint8_t *t = idx->text.data();
    const int64_t N = (int64_t)n + 1;

    // S = reversed text + terminator: '$' = 0, a record separator 1, characters 2..sigma+1.
    std::vector<uint8_t> S;
    std::vector<int32_t> SA;
    try {
        S.resize(N);
        SA.resize(N);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory building the suffix array (n=%llu)", (unsigned long long)n);
        return ALAE_E_NOMEM;
    }
    for (uint64_t k = 0; k < n; ++k) {
        const uint8_t x = t[n - 1 - k];
        S[k] = x == kSepCode ? 1 : (uint8_t)(x + 2);
    }
    S[n] = 0;
    induced_sort<uint8_t>(S.data(), SA.data(), (int32_t)N, sigma + 2);

    // C[c] = 1 + separators + characters below c (the rows of '$' and of the
    // separators come first)
    uint64_t counts[21] = {0};
    for (uint64_t i = 0; i < n; ++i)
        if (t[i] != kSepCode) counts[t[i]]++;
    uint64_t acc = 1 + idx->nsep;
    for (int c = 0; c < sigma; ++c) {
        idx->C[c] = acc;
        acc += counts[c];
    }
    idx->C[sigma] = acc;
    idx->occ_packed = sigma == 4 && idx->nsep == 0;

    idx->sa_end.resize(N);
    std::vector<uint8_t> bwt(N);
    for (int64_t h = 0; h < N; ++h) {
        int32_t p = SA[h];
        idx->sa_end[h] = (p == (int32_t)n) ? kNoPos : (uint32_t)(n - 1 - (uint64_t)p);
        if (p == 0) {
            bwt[h] = 0xFF;
            idx->dollar_row = (uint64_t)h;
        } else {
            bwt[h] = S[p - 1] == 1 ? kSepCode : (uint8_t)(S[p - 1] - 2);
        }
    }
    SA.clear();
    SA.shrink_to_fit();
    S.clear();
    S.shrink_to_fit();

    if (idx->occ_packed) {
        idx->nblocks = (uint64_t)(N + kDnaBlockChars - 1) / kDnaBlockChars;
        idx->occ.assign(idx->nblocks * sizeof(DnaOccBlock), 0);
        DnaOccBlock *blk = reinterpret_cast<DnaOccBlock *>(idx->occ.data());
        uint32_t run[4] = {0, 0, 0, 0};
        for (uint64_t b = 0; b < idx->nblocks; ++b) {
            for (int c = 0; c < 4; ++c) blk[b].cnt[c] = run[c];
            for (int k = 0; k < kDnaBlockChars; ++k) {
                uint64_t h = b * kDnaBlockChars + k;
                if (h >= (uint64_t)N) break;
                uint8_t c = bwt[h];
                uint32_t code = (c == 0xFF) ? 0u : c;
                blk[b].bits[k / 16] |= code << (2 * (k % 16));
                if (c != 0xFF) run[c]++;
            }
        }
    } else {
        idx->nblocks = (uint64_t)(N + kGenBlockChars - 1) / kGenBlockChars;
        idx->occ.assign(idx->nblocks * sizeof(GenOccBlock), 0);
        GenOccBlock *blk = reinterpret_cast<GenOccBlock *>(idx->occ.data());
        uint32_t run[20] = {0};
        for (uint64_t b = 0; b < idx->nblocks; ++b) {
            for (int c = 0; c < 20; ++c) blk[b].cnt[c] = run[c];
            for (int k = 0; k < kGenBlockChars; ++k) {
                uint64_t h = b * kGenBlockChars + k;
                uint8_t c = (h < (uint64_t)N) ? bwt[h] : 0xFF;
                blk[b].ch[k] = c;
                if (h < (uint64_t)N && c < 20) run[c]++;
            }
        }
    }
    return ALAE_OK;
}

}  // namespace alae

using namespace alae;

extern "C" {

const char *alae_last_error(void) { return alae::last_error_text(); }

const char *alae_version(void) { return "alae-mi355x 0.1 (gfx950)"; }

}  // extern "C"

namespace alae {

// The index of idx->text (codes, separators included; n, sigma, alphabet, nsep
// and rec_start set) by the builder the options pick.
static alae_status build_index(std::unique_ptr<alae_index> &idx, const alae_index_opts *opts, alae_index **out) {
    const uint64_t n = idx->n;
    idx->device = opts ? opts->device : 0;
    // builder: 1 = host, 2 = GPU, 0 = the GPU for texts of 2^22 characters or more when one is present
    const int builder = opts ? opts->builder : 0;
    if (builder < 0 || builder > 2) {
        set_error("alae_index_build: builder must be 0, 1 or 2 (got %d)", builder);
        return ALAE_E_ARG;
    }
    const bool on_gpu = builder == 2 || (builder == 0 && n >= (1ull << 22) && device_present(idx->device));
    idx->occ_packed = idx->sigma == 4 && idx->nsep == 0;
    alae_status st;
    try {
        st = on_gpu ? build_index_on_device(idx.get()) : build_from_codes(idx);
    } catch (const std::bad_alloc &) {
        set_error("alae_index_build: out of host memory");
        return ALAE_E_NOMEM;
    }
    if (st != ALAE_OK) return st;
    *out = idx.release();
    return ALAE_OK;
}

}  // namespace alae

extern "C" {

alae_status alae_index_build_codes(const uint8_t *codes, size_t n, alae_alphabet alphabet,
                                   const alae_index_opts *opts, alae_index **out) {
    if (!codes || !out || n == 0) {
        set_error("alae_index_build: null argument or empty text");
        return ALAE_E_ARG;
    }
    int sigma = alphabet_sigma(alphabet);
    if (!sigma) {
        set_error("alae_index_build: unknown alphabet %d", (int)alphabet);
        return ALAE_E_ARG;
    }
    if (n >= 0x7FFFFFFEull) {
        set_error("alae_index_build: text of %zu characters exceeds the 32-bit suffix array", n);
        return ALAE_E_TOO_LONG;
    }
    for (size_t i = 0; i < n; ++i) {
        if (codes[i] >= sigma) {
            set_error("alae_index_build: code %u at %zu outside the alphabet", codes[i], i);
            return ALAE_E_ALPHABET;
        }
    }
    std::unique_ptr<alae_index> idx;
    try {
        idx.reset(new alae_index());
        idx->text.assign(codes, codes + n);
        idx->rec_start.assign(1, 0);
    } catch (const std::bad_alloc &) {
        set_error("alae_index_build: out of host memory");
        return ALAE_E_NOMEM;
    }
    idx->n = n;
    idx->sigma = sigma;
    idx->alphabet = alphabet;
    return build_index(idx, opts, out);
}

alae_status alae_index_build_records(const uint8_t *codes, const size_t *lens, size_t k, alae_alphabet alphabet,
                                     const alae_index_opts *opts, alae_index **out) {
    if (!codes || !lens || !out || k == 0) {
        set_error("alae_index_build_records: null argument or no record");
        return ALAE_E_ARG;
    }
    const int sigma = alphabet_sigma(alphabet);
    if (!sigma) {
        set_error("alae_index_build_records: unknown alphabet %d", (int)alphabet);
        return ALAE_E_ARG;
    }
    uint64_t total = 0;
    for (size_t r = 0; r < k; ++r) {
        if (lens[r] == 0) {
            set_error("alae_index_build_records: record %zu is empty", r);
            return ALAE_E_ARG;
        }
        total += lens[r];
    }
    const uint64_t n = total + (k - 1);
    if (n >= 0x7FFFFFFEull) {
        set_error("alae_index_build_records: %llu characters with separators exceed the 32-bit suffix array",
                  (unsigned long long)n);
        return ALAE_E_TOO_LONG;
    }
    for (uint64_t i = 0; i < total; ++i) {
        if (codes[i] >= sigma) {
            set_error("alae_index_build_records: code %u at %llu outside the alphabet", codes[i],
                      (unsigned long long)i);
            return ALAE_E_ALPHABET;
        }
    }
    std::unique_ptr<alae_index> idx;
    try {
        idx.reset(new alae_index());
        idx->text.resize(n);
        idx->rec_start.resize(k);
    } catch (const std::bad_alloc &) {
        set_error("alae_index_build_records: out of host memory");
        return ALAE_E_NOMEM;
    }
    uint64_t at = 0, src = 0;
    for (size_t r = 0; r < k; ++r) {
        if (r > 0) idx->text[at++] = kSepCode;
        idx->rec_start[r] = at;
        memcpy(idx->text.data() + at, codes + src, lens[r]);
        at += lens[r];
        src += lens[r];
    }
    idx->n = n;
    idx->sigma = sigma;
    idx->alphabet = alphabet;
    idx->nsep = k - 1;
    return build_index(idx, opts, out);
}

alae_status alae_index_record_of(const alae_index *index, uint64_t text_pos, uint64_t *record, uint64_t *offset) {
    if (!index || !record || !offset) {
        set_error("alae_index_record_of: null argument");
        return ALAE_E_ARG;
    }
    if (text_pos >= index->n || index->text[text_pos] == kSepCode) {
        set_error("alae_index_record_of: position %llu is not a character of a record",
                  (unsigned long long)text_pos);
        return ALAE_E_ARG;
    }
    const auto &rs = index->rec_start;
    const size_t r = (size_t)(std::upper_bound(rs.begin(), rs.end(), text_pos) - rs.begin()) - 1;
    *record = r;
    *offset = text_pos - rs[r];
    return ALAE_OK;
}

alae_status alae_index_build(const char *text, size_t n, alae_alphabet alphabet, const alae_index_opts *opts,
                             alae_index **out) {
    if (!text || !out || n == 0) {
        set_error("alae_index_build: null argument or empty text");
        return ALAE_E_ARG;
    }
    if (!alphabet_sigma(alphabet)) {
        set_error("alae_index_build: unknown alphabet %d", (int)alphabet);
        return ALAE_E_ARG;
    }
    std::vector<uint8_t> codes;
    try {
        codes.resize(n);
    } catch (const std::bad_alloc &) {
        set_error("alae_index_build: out of host memory");
        return ALAE_E_NOMEM;
    }
    if (!encode(text, n, alphabet, codes.data())) {
        set_error("alae_index_build: character outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    return alae_index_build_codes(codes.data(), n, alphabet, opts, out);
}

void alae_index_free(alae_index *index) {
    if (!index) return;
    release_device(index);
    delete index;
}

alae_status alae_index_get_info(const alae_index *index, alae_index_info *out) {
    if (!index || !out) {
        set_error("alae_index_get_info: null argument");
        return ALAE_E_ARG;
    }
    memset(out, 0, sizeof(*out));
    out->n = index->n;
    out->sigma = index->sigma;
    out->alphabet = index->alphabet;
    for (int c = 0; c <= index->sigma; ++c) out->C[c] = index->C[c];
    out->dollar_row = index->dollar_row;
    out->records = index->rec_start.size();
    out->host_bytes = index->text.size() + index->sa_end.size() * 4 + index->occ.size();
    out->device_bytes = index->on_device ? out->host_bytes : 0;
    return ALAE_OK;
}

alae_status alae_index_copy_sa(const alae_index *index, uint32_t *sa_end) {
    if (!index || !sa_end) {
        set_error("alae_index_copy_sa: null argument");
        return ALAE_E_ARG;
    }
    memcpy(sa_end, index->sa_end.data(), index->sa_end.size() * sizeof(uint32_t));
    return ALAE_OK;
}

alae_status alae_index_copy_bwt(const alae_index *index, uint8_t *bwt) {
    if (!index || !bwt) {
        set_error("alae_index_copy_bwt: null argument");
        return ALAE_E_ARG;
    }
    const uint64_t N = index->n + 1;
    for (uint64_t h = 0; h < N; ++h) {
        if (h == index->dollar_row) {
            bwt[h] = 0xFF;
            continue;
        }
        if (index->occ_packed) {
            const DnaOccBlock *b = reinterpret_cast<const DnaOccBlock *>(index->occ.data()) + h / kDnaBlockChars;
            int k = (int)(h % kDnaBlockChars);
            bwt[h] = (uint8_t)((b->bits[k / 16] >> (2 * (k % 16))) & 3);
        } else {
            const GenOccBlock *b = reinterpret_cast<const GenOccBlock *>(index->occ.data()) + h / kGenBlockChars;
            bwt[h] = b->ch[h % kGenBlockChars];
        }
    }
    return ALAE_OK;
}

alae_status alae_index_range(const alae_index *index, const uint8_t *pattern, size_t len, uint64_t *lo,
                             uint64_t *hi) {
    if (!index || !lo || !hi || (len && !pattern)) {
        set_error("alae_index_range: null argument");
        return ALAE_E_ARG;
    }
    int64_t l = 0, r = (int64_t)index->n;  // root: every row
    for (size_t k = 0; k < len; ++k) {
        int c = pattern[k];
        if (c >= index->sigma) {
            set_error("alae_index_range: code outside the alphabet");
            return ALAE_E_ALPHABET;
        }
        l = (int64_t)index->C[c] + (int64_t)host_occ(index, c, l - 1);
        r = (int64_t)index->C[c] + (int64_t)host_occ(index, c, r) - 1;
        if (l > r) break;
    }
    *lo = (uint64_t)l;
    *hi = (uint64_t)r;
    if (l > r) {  // empty: report lo = hi + 1
        *lo = (uint64_t)(r + 1);
    }
    return ALAE_OK;
}

// ---- persistence -----------------------------------------------------------
static const char kMagic[8] = {'A', 'L', 'A', 'E', 'I', 'D', 'X', '2'};

alae_status alae_index_save(const alae_index *index, const char *path) {
    if (!index || !path) {
        set_error("alae_index_save: null argument");
        return ALAE_E_ARG;
    }
    std::ofstream f(path, std::ios::binary | std::ios::trunc);
    if (!f) {
        set_error("alae_index_save: cannot open %s", path);
        return ALAE_E_IO;
    }
    uint64_t hdr[9] = {index->n, (uint64_t)index->sigma, (uint64_t)index->alphabet, index->nblocks,
                       index->dollar_row, (uint64_t)index->occ.size(), index->nsep,
                       (uint64_t)index->rec_start.size(), (uint64_t)(index->occ_packed ? 1 : 0)};
    f.write(kMagic, 8);
    f.write(reinterpret_cast<const char *>(hdr), sizeof(hdr));
    f.write(reinterpret_cast<const char *>(index->C), sizeof(index->C));
    f.write(reinterpret_cast<const char *>(index->rec_start.data()),
            (std::streamsize)(index->rec_start.size() * sizeof(uint64_t)));
    f.write(reinterpret_cast<const char *>(index->text.data()), (std::streamsize)index->text.size());
    f.write(reinterpret_cast<const char *>(index->sa_end.data()), (std::streamsize)(index->sa_end.size() * 4));
    f.write(reinterpret_cast<const char *>(index->occ.data()), (std::streamsize)index->occ.size());
    if (!f) {
        set_error("alae_index_save: write failed for %s", path);
        return ALAE_E_IO;
    }
    return ALAE_OK;
}

alae_status alae_index_load(const char *path, const alae_index_opts *opts, alae_index **out) {
    if (!path || !out) {
        set_error("alae_index_load: null argument");
        return ALAE_E_ARG;
    }
    std::ifstream f(path, std::ios::binary);
    if (!f) {
        set_error("alae_index_load: cannot open %s", path);
        return ALAE_E_IO;
    }
    char magic[8];
    uint64_t hdr[9];
    f.read(magic, 8);
    f.read(reinterpret_cast<char *>(hdr), sizeof(hdr));
    if (!f || memcmp(magic, kMagic, 8) != 0) {
        set_error("alae_index_load: %s is not an index image of this version", path);
        return ALAE_E_IO;
    }
    std::unique_ptr<alae_index> idx;
    try {
        idx.reset(new alae_index());
        idx->n = hdr[0];
        idx->sigma = (int)hdr[1];
        idx->alphabet = (int)hdr[2];
        idx->nblocks = hdr[3];
        idx->dollar_row = hdr[4];
        idx->nsep = hdr[6];
        idx->occ_packed = hdr[8] != 0;
        if (alphabet_sigma(idx->alphabet) != idx->sigma || idx->n == 0 || idx->n >= 0x7FFFFFFEull ||
            hdr[7] != idx->nsep + 1 || (idx->occ_packed && (idx->sigma != 4 || idx->nsep != 0))) {
            set_error("alae_index_load: corrupt header in %s", path);
            return ALAE_E_IO;
        }
        f.read(reinterpret_cast<char *>(idx->C), sizeof(idx->C));
        idx->rec_start.resize(hdr[7]);
        f.read(reinterpret_cast<char *>(idx->rec_start.data()), (std::streamsize)(hdr[7] * sizeof(uint64_t)));
        idx->text.resize(idx->n);
        idx->sa_end.resize(idx->n + 1);
        idx->occ.resize(hdr[5]);
    } catch (const std::bad_alloc &) {
        set_error("alae_index_load: out of host memory");
        return ALAE_E_NOMEM;
    }
    f.read(reinterpret_cast<char *>(idx->text.data()), (std::streamsize)idx->text.size());
    f.read(reinterpret_cast<char *>(idx->sa_end.data()), (std::streamsize)(idx->sa_end.size() * 4));
    f.read(reinterpret_cast<char *>(idx->occ.data()), (std::streamsize)idx->occ.size());
    if (!f) {
        set_error("alae_index_load: truncated file %s", path);
        return ALAE_E_IO;
    }
    idx->device = opts ? opts->device : 0;
    *out = idx.release();
    return ALAE_OK;
}

}  // extern "C"
