// Alignment starts (the paper's A(i,j).pos, Section 2.1 and Table 1) and
// transcripts for reported cells.
//
// For a hit (query end j, text end t, score S = A(t,j)) the start reported is
// the one of the optimal alignment with the largest text start x, and among
// those the largest query start y.  It is found by a local (Smith-Waterman,
// Gotoh) DP over a window T[t-W+1..t] x P[j-V+1..j] in which every state
// carries the start of its best alignment: value and start are packed into
// one 64-bit key (value high, start code i*V+k low), so the maximum of the
// keys is the best value with the latest start.  The zero floor of a cell is
// the empty alignment, whose key carries the start just after the cell (it
// wins ties at value 0: dropping a prefix of score 0 gives a later start).
// The window holds the wanted alignment once the DP reaches S at (t, j) and V
// covers the query span of every alignment starting at or after the found x:
// an alignment of text span r and score S has query span at most
// r + (s_max r + s_g - S) / |s_s| (a gap run pays for the extra query
// characters); otherwise W and V grow.  Windows stop at the start of the text
// and of the hit's record.
//
// The transcript is one optimal alignment from that start to (t, j): a global
// DP over the rectangle anchored at the start pair (an optimal alignment
// begins with an aligned pair, a leading gap only costs) keeps H, E and F of
// every cell, and one lane traces back from (t, j) by equality with the
// recurrences.  Ops: 'M' text and query character aligned, 'D' a text
// character against a gap, 'I' a query character against a gap.
//
// One wave (64 lanes) per cell; rows in order, 64 columns at a time; the
// query-gap state F of a row is an exclusive prefix maximum of
// H0(k') - s_s k' over the row (exact because s_g <= 0: opening a gap right
// after a gap never beats extending it), carried from one 64-column chunk to
// the next.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "alae_internal.h"

namespace alae {
namespace {

#define TB_TRY(expr)                                                                             \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            hipGetLastError();                                                                   \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
            return ALAE_E_DEVICE;                                                                \
        }                                                                                        \
    } while (0)

constexpr int64_t kNegKey = -(1ll << 61);       // a state that does not exist (window DP)
constexpr int32_t kNeg32 = -(1 << 29);          // the same in the rectangle DP
constexpr uint64_t kMaxCells = 1ull << 30;       // window cells of one hit (start codes fit 31 bits)
constexpr uint64_t kTraceBudget = 1ull << 31;    // bytes of rectangle matrices per launch

struct Scores {
    int8_t s[20 * 20];  // [text code][query code]
    int32_t sg, ss;
};

__device__ inline int64_t add_val(int64_t key, int64_t d) { return key + (d << 32); }

__device__ inline int64_t shfl_up64(int64_t v, int d) {
    const uint32_t lo = __shfl_up((uint32_t)(uint64_t)v, d, 64);
    const uint32_t hi = __shfl_up((uint32_t)((uint64_t)v >> 32), d, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int64_t shfl64(int64_t v, int src) {
    const uint32_t lo = __shfl((uint32_t)(uint64_t)v, src, 64);
    const uint32_t hi = __shfl((uint32_t)((uint64_t)v >> 32), src, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

struct LocateJob {
    uint64_t t;       // text end
    uint32_t j;       // query end
    uint32_t W, V;    // window rows (text) and columns (query)
};

// Window DP of one hit per wave.  rows: 4 * V keys per job at row_off[job]
// (H and E of the previous and of the current row).  out[job] = key of (t, j).
__global__ void __launch_bounds__(64) k_locate(const uint8_t *text, const uint8_t *query, Scores sc,
                                               const LocateJob *jobs, uint32_t njobs, const uint64_t *row_off,
                                               int64_t *rows, int64_t *out) {
    const uint32_t job = blockIdx.x;
    if (job >= njobs) return;
    const int lane = threadIdx.x;
    const LocateJob jb = jobs[job];
    const uint32_t W = jb.W, V = jb.V;
    int64_t *Hp = rows + row_off[job], *Ep = Hp + V, *Hc = Ep + V, *Ec = Hc + V;
    const uint64_t x0 = jb.t + 1 - W;  // text position of window row 0
    const uint32_t y0 = jb.j + 1 - V;  // query position of window column 0
    const int64_t open = (int64_t)sc.sg + sc.ss;
    int64_t last = kNegKey;
    for (uint32_t i = 0; i < W; ++i) {
        const uint32_t tc = text[x0 + i];
        int64_t carry_max = kNegKey;  // prefix max of H0 - s_s k over the earlier chunks of the row
        int64_t diag_carry = 0;       // H of the row above at the column before this chunk
        for (uint32_t c0 = 0; c0 < V; c0 += 64) {
            const uint32_t k = c0 + lane;
            const bool in = k < V;
            int64_t hup, eup;
            if (i == 0) {
                hup = (int64_t)(k + 1);  // the floor of (-1, k): value 0, start (0, k+1)
                eup = kNegKey;
            } else {
                hup = in ? Hp[k] : kNegKey;
                eup = in ? Ep[k] : kNegKey;
            }
            int64_t hd = shfl_up64(hup, 1);  // H(i-1, k-1)
            if (lane == 0) hd = c0 == 0 ? (int64_t)((uint64_t)i * V) : diag_carry;  // floor of (i-1, -1)
            diag_carry = shfl64(hup, 63);
            const uint32_t pc = in ? query[y0 + k] : 0u;
            const int64_t D = add_val(hd, sc.s[tc * 20 + pc]);
            int64_t E = add_val(eup, sc.ss);
            const int64_t Eo = add_val(hup, open);
            if (Eo > E) E = Eo;
            int64_t H0 = (int64_t)((uint64_t)(i + 1) * V + k + 1);  // the floor of (i, k)
            if (D > H0) H0 = D;
            if (E > H0) H0 = E;
            // F(i,k) = s_g + s_s k + max_{k'<k} (H0(i,k') - s_s k')
            int64_t incl = in ? add_val(H0, -(int64_t)sc.ss * (int64_t)k) : kNegKey;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int64_t o = shfl_up64(incl, d);
                if (lane >= d && o > incl) incl = o;
            }
            int64_t excl = shfl_up64(incl, 1);
            if (lane == 0) excl = kNegKey;
            if (carry_max > excl) excl = carry_max;
            const int64_t top = shfl64(incl, 63);
            if (top > carry_max) carry_max = top;
            int64_t H = H0;
            if (excl > kNegKey / 2) {
                const int64_t F = add_val(excl, (int64_t)sc.sg + (int64_t)sc.ss * (int64_t)k);
                if (F > H) H = F;
            }
            if (in) {
                Hc[k] = H;
                Ec[k] = E;
                if (i == W - 1 && k == V - 1) last = H;
            }
        }
        int64_t *t1 = Hp;
        Hp = Hc;
        Hc = t1;
        t1 = Ep;
        Ep = Ec;
        Ec = t1;
    }
    if (lane == (int)((V - 1) & 63)) out[job] = last;
}

struct TraceJob {
    uint64_t x;      // text start
    uint32_t y;      // query start
    uint32_t R, Q;   // rectangle rows (text) and columns (query)
};

// Global DP anchored at the start pair; M3 holds H, E, F of every cell
// (3 * R * Q int32 at mat_off[job]).  Lane 0 then traces back from the last
// cell, writing ops in reverse at ops_off[job] (at most R + Q of them).
__global__ void __launch_bounds__(64) k_trace(const uint8_t *text, const uint8_t *query, Scores sc,
                                              const TraceJob *jobs, uint32_t njobs, const uint64_t *mat_off,
                                              int32_t *mats, const uint64_t *ops_off, char *ops, uint32_t *ops_len,
                                              int32_t *end_value) {
    const uint32_t job = blockIdx.x;
    if (job >= njobs) return;
    const int lane = threadIdx.x;
    const TraceJob jb = jobs[job];
    const uint32_t R = jb.R, Q = jb.Q;
    const uint64_t RQ = (uint64_t)R * Q;
    int32_t *Hm = mats + mat_off[job], *Em = Hm + RQ, *Fm = Em + RQ;
    const int32_t open = sc.sg + sc.ss;
    auto live = [](int32_t v) { return v > kNeg32 / 2; };
    for (uint32_t i = 0; i < R; ++i) {
        const uint32_t tc = text[jb.x + i];
        int32_t carry_max = kNeg32, diag_carry = kNeg32;
        for (uint32_t c0 = 0; c0 < Q; c0 += 64) {
            const uint32_t k = c0 + lane;
            const bool in = k < Q;
            const int32_t hup = (i == 0 || !in) ? kNeg32 : Hm[(uint64_t)(i - 1) * Q + k];
            const int32_t eup = (i == 0 || !in) ? kNeg32 : Em[(uint64_t)(i - 1) * Q + k];
            int32_t hd = __shfl_up(hup, 1, 64);
            if (lane == 0) hd = c0 == 0 ? (i == 0 ? 0 : kNeg32) : diag_carry;  // only the start pair opens
            diag_carry = __shfl(hup, 63, 64);
            const uint32_t pc = in ? query[jb.y + k] : 0u;
            const int32_t D = live(hd) ? hd + sc.s[tc * 20 + pc] : kNeg32;
            const int32_t Ex = live(eup) ? eup + sc.ss : kNeg32;
            const int32_t Eo = live(hup) ? hup + open : kNeg32;
            const int32_t E = Ex > Eo ? Ex : Eo;
            const int32_t H0 = D > E ? D : E;
            int32_t incl = (in && live(H0)) ? H0 - sc.ss * (int32_t)k : kNeg32;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int32_t o = __shfl_up(incl, d, 64);
                if (lane >= d && o > incl) incl = o;
            }
            int32_t excl = __shfl_up(incl, 1, 64);
            if (lane == 0) excl = kNeg32;
            if (carry_max > excl) excl = carry_max;
            const int32_t top = __shfl(incl, 63, 64);
            if (top > carry_max) carry_max = top;
            const int32_t F = live(excl) ? excl + sc.sg + sc.ss * (int32_t)k : kNeg32;
            if (in) {
                const uint64_t at = (uint64_t)i * Q + k;
                Hm[at] = H0 > F ? H0 : F;
                Em[at] = E;
                Fm[at] = F;
            }
        }
        __syncthreads();
    }
    if (lane != 0) return;
    __threadfence_block();
    // traceback from (R-1, Q-1) in state H
    char *o = ops + ops_off[job];
    uint32_t n = 0;
    int64_t i = (int64_t)R - 1, k = (int64_t)Q - 1;
    int state = 0;  // 0: H, 1: E (text character against a gap), 2: F (query character against a gap)
    const uint32_t maxops = R + Q;
    bool ok = true;
    end_value[job] = Hm[RQ - 1];
    while (i >= 0 && k >= 0 && n < maxops) {
        const uint64_t at = (uint64_t)i * Q + k;
        if (state == 0) {
            const int32_t h = Hm[at];
            const int32_t s = sc.s[text[jb.x + i] * 20 + query[jb.y + k]];
            if (i == 0 && k == 0) {
                ok = h == s;
                o[n++] = 'M';
                break;
            }
            if (i > 0 && k > 0 && live(Hm[at - Q - 1]) && Hm[at - Q - 1] + s == h) {
                o[n++] = 'M';
                --i;
                --k;
            } else if (Em[at] == h) {
                state = 1;
            } else if (Fm[at] == h) {
                state = 2;
            } else {
                ok = false;
                break;
            }
        } else if (state == 1) {
            const int32_t e = Em[at];
            o[n++] = 'D';
            if (i == 0) {
                ok = false;
                break;
            }
            state = (live(Em[at - Q]) && Em[at - Q] + sc.ss == e) ? 1 : 0;
            if (state == 0 && Hm[at - Q] + open != e) {
                ok = false;
                break;
            }
            --i;
        } else {
            const int32_t f = Fm[at];
            o[n++] = 'I';
            if (k == 0) {
                ok = false;
                break;
            }
            state = (live(Fm[at - 1]) && Fm[at - 1] + sc.ss == f) ? 2 : 0;
            if (state == 0 && Hm[at - 1] + open != f) {
                ok = false;
                break;
            }
            --k;
        }
    }
    ops_len[job] = ok ? n : 0xFFFFFFFFu;
}

template <typename T>
hipError_t dev_buf(T *&p, uint64_t &cap, uint64_t need) {
    if (need <= cap && p) return hipSuccess;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(&p, std::max<uint64_t>(need, 1) * sizeof(T));
    if (e == hipSuccess) cap = std::max<uint64_t>(need, 1);
    return e;
}

struct TbBufs {
    LocateJob *ljobs = nullptr;
    TraceJob *tjobs = nullptr;
    uint64_t *off = nullptr, *off2 = nullptr;
    int64_t *rows = nullptr, *keys = nullptr;
    int32_t *mats = nullptr, *endv = nullptr;
    char *ops = nullptr;
    uint32_t *lens = nullptr;
    uint8_t *query = nullptr;
    uint64_t c_lj = 0, c_tj = 0, c_off = 0, c_off2 = 0, c_rows = 0, c_keys = 0, c_mats = 0, c_endv = 0, c_ops = 0,
             c_lens = 0, c_q = 0;
    ~TbBufs() {
        hipFree(ljobs);
        hipFree(tjobs);
        hipFree(off);
        hipFree(off2);
        hipFree(rows);
        hipFree(keys);
        hipFree(mats);
        hipFree(endv);
        hipFree(ops);
        hipFree(lens);
        hipFree(query);
    }
};

int64_t extra_query_span(int64_t r, int32_t smax, int32_t sg, int32_t ss, int32_t S) {
    const int64_t num = (int64_t)smax * r + sg - S;
    return num > 0 ? num / (-(int64_t)ss) : 0;
}

}  // namespace
}  // namespace alae

using namespace alae;

extern "C" {

alae_status alae_traceback(const alae_index *index, const char *query, size_t m, const alae_scoring *scoring,
                           const uint32_t *query_ends, const uint64_t *text_ends, const int32_t *scores, size_t k,
                           alae_alignments *out) {
    if (!index || !query || !scoring || !out || m == 0 || (k && (!query_ends || !text_ends || !scores))) {
        set_error("alae_traceback: null argument or empty query");
        return ALAE_E_ARG;
    }
    memset(out, 0, sizeof(*out));
    const int sigma = index->sigma;
    if (scoring->ss >= 0 || scoring->sg > 0 || (scoring->use_matrix && !scoring->matrix) ||
        (!scoring->use_matrix && (scoring->sa <= 0 || scoring->sb >= 0))) {
        set_error("alae_traceback: scoring outside the model of Section 2.1");
        return ALAE_E_SCORING;
    }
    Scores sc;
    memset(&sc, 0, sizeof(sc));
    sc.sg = scoring->sg;
    sc.ss = scoring->ss;
    int32_t smax = -128;
    for (int a = 0; a < sigma; ++a)
        for (int b = 0; b < sigma; ++b) {
            const int v = scoring->use_matrix ? scoring->matrix[a * sigma + b] : (a == b ? scoring->sa : scoring->sb);
            sc.s[a * 20 + b] = (int8_t)v;
            smax = std::max(smax, v);
        }
    std::vector<uint8_t> codes(m);
    if (!encode(query, m, index->alphabet, codes.data())) {
        set_error("alae_traceback: query holds a character outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    alae_status st = ensure_device(index);
    if (st != ALAE_OK) return st;
    TB_TRY(hipSetDevice(index->device));
    TbBufs b;
    TB_TRY(dev_buf(b.query, b.c_q, m));
    TB_TRY(hipMemcpy(b.query, codes.data(), m, hipMemcpyHostToDevice));
    std::unique_ptr<alae_alignment[]> aln(new (std::nothrow) alae_alignment[k ? k : 1]);
    if (!aln) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    // windows: start small, grow until they provably hold the wanted alignment
    std::vector<uint64_t> xmin(k);
    std::vector<uint32_t> W(k), V(k);
    std::vector<size_t> pending;
    for (size_t h = 0; h < k; ++h) {
        alae_alignment &a = aln[h];
        memset(&a, 0, sizeof(a));
        a.score = scores[h];
        const uint64_t t = text_ends[h];
        const uint32_t j = query_ends[h];
        if (t >= index->n || j >= m || scores[h] < 1 || index->text[t] == kSepCode) {
            a.status = ALAE_E_ARG;
            continue;
        }
        const auto &rs = index->rec_start;
        xmin[h] = rs.empty() ? 0 : rs[(size_t)(std::upper_bound(rs.begin(), rs.end(), t) - rs.begin()) - 1];
        const uint64_t wmax = t - xmin[h] + 1;
        const uint64_t w0 = std::min<uint64_t>(wmax, 2ull * ((uint64_t)scores[h] / (uint64_t)smax) + 32);
        W[h] = (uint32_t)w0;
        V[h] = (uint32_t)std::min<uint64_t>((uint64_t)j + 1,
                                            w0 + extra_query_span((int64_t)w0, smax, sc.sg, sc.ss, scores[h]) + 1);
        pending.push_back(h);
    }
    while (!pending.empty()) {
        std::vector<size_t> now;
        std::vector<LocateJob> jobs;
        std::vector<uint64_t> offs;
        uint64_t rows = 0;
        for (size_t h : pending) {
            if ((uint64_t)W[h] * V[h] > kMaxCells) {
                aln[h].status = ALAE_E_TOO_LONG;
                continue;
            }
            now.push_back(h);
            jobs.push_back(LocateJob{text_ends[h], query_ends[h], W[h], V[h]});
            offs.push_back(rows);
            rows += 4ull * V[h];
        }
        pending.clear();
        if (now.empty()) break;
        TB_TRY(dev_buf(b.ljobs, b.c_lj, jobs.size()));
        TB_TRY(dev_buf(b.off, b.c_off, offs.size()));
        TB_TRY(dev_buf(b.rows, b.c_rows, rows));
        TB_TRY(dev_buf(b.keys, b.c_keys, jobs.size()));
        TB_TRY(hipMemcpy(b.ljobs, jobs.data(), jobs.size() * sizeof(LocateJob), hipMemcpyHostToDevice));
        TB_TRY(hipMemcpy(b.off, offs.data(), offs.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
        k_locate<<<(uint32_t)jobs.size(), 64>>>(index->d_text, b.query, sc, b.ljobs, (uint32_t)jobs.size(), b.off,
                                               b.rows, b.keys);
        TB_TRY(hipGetLastError());
        std::vector<int64_t> keys(jobs.size());
        TB_TRY(hipMemcpy(keys.data(), b.keys, keys.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        for (size_t q = 0; q < now.size(); ++q) {
            const size_t h = now[q];
            const int64_t key = keys[q];
            const int32_t value = (int32_t)(key >> 32);
            const uint32_t code = (uint32_t)(key & 0xFFFFFFFFll);
            const uint64_t t = text_ends[h];
            const uint32_t j = query_ends[h];
            const uint64_t wmax = t - xmin[h] + 1;
            const int32_t S = scores[h];
            if (value > S) {  // the cell scores more than the given score: not this hit
                aln[h].status = ALAE_E_ARG;
                continue;
            }
            if (value == S) {
                const uint64_t i = code / V[h], kk = code % V[h];
                const uint64_t x = t + 1 - W[h] + i;
                const uint32_t y = (uint32_t)(j + 1 - V[h] + kk);
                const int64_t r = (int64_t)(t - x + 1);
                const uint64_t need = (uint64_t)r + extra_query_span(r, smax, sc.sg, sc.ss, S);
                if (V[h] == j + 1 || V[h] >= need) {
                    aln[h].text_start = x;
                    aln[h].query_start = y;
                    aln[h].status = ALAE_OK;
                    continue;
                }
                V[h] = (uint32_t)std::min<uint64_t>((uint64_t)j + 1, need);
                pending.push_back(h);
                continue;
            }
            if (W[h] == wmax && V[h] == j + 1) {  // the whole text and query prefix: no alignment reaches S
                aln[h].status = ALAE_E_ARG;
                continue;
            }
            W[h] = (uint32_t)std::min<uint64_t>(wmax, 2ull * W[h]);
            V[h] = (uint32_t)std::min<uint64_t>(
                (uint64_t)j + 1, std::max<uint64_t>(2ull * V[h], (uint64_t)W[h] +
                                                                     extra_query_span(W[h], smax, sc.sg, sc.ss, S)));
            pending.push_back(h);
        }
    }
    // transcripts, in launches of at most kTraceBudget bytes of matrices
    std::vector<size_t> ready;
    for (size_t h = 0; h < k; ++h)
        if (aln[h].status == ALAE_OK) ready.push_back(h);
    std::vector<std::vector<char>> ops_of(k);
    for (size_t p = 0; p < ready.size();) {
        std::vector<TraceJob> jobs;
        std::vector<uint64_t> moff, ooff;
        std::vector<size_t> which;
        uint64_t mats = 0, nops = 0;
        for (; p < ready.size(); ++p) {
            const size_t h = ready[p];
            const uint64_t R = text_ends[h] - aln[h].text_start + 1, Q = query_ends[h] - aln[h].query_start + 1;
            const uint64_t bytes = 12ull * R * Q;
            if (bytes > kTraceBudget) {  // the start stands; the transcript does not fit
                aln[h].status = ALAE_E_TOO_LONG;
                continue;
            }
            if (!jobs.empty() && 4ull * (mats + 3 * R * Q) > kTraceBudget) break;
            jobs.push_back(TraceJob{aln[h].text_start, aln[h].query_start, (uint32_t)R, (uint32_t)Q});
            moff.push_back(mats);
            ooff.push_back(nops);
            which.push_back(h);
            mats += 3 * R * Q;
            nops += R + Q;
        }
        if (jobs.empty()) continue;
        TB_TRY(dev_buf(b.tjobs, b.c_tj, jobs.size()));
        TB_TRY(dev_buf(b.off, b.c_off, jobs.size()));
        TB_TRY(dev_buf(b.off2, b.c_off2, jobs.size()));
        TB_TRY(dev_buf(b.mats, b.c_mats, mats));
        TB_TRY(dev_buf(b.ops, b.c_ops, nops));
        TB_TRY(dev_buf(b.lens, b.c_lens, jobs.size()));
        TB_TRY(dev_buf(b.endv, b.c_endv, jobs.size()));
        TB_TRY(hipMemcpy(b.tjobs, jobs.data(), jobs.size() * sizeof(TraceJob), hipMemcpyHostToDevice));
        TB_TRY(hipMemcpy(b.off, moff.data(), moff.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
        TB_TRY(hipMemcpy(b.off2, ooff.data(), ooff.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
        k_trace<<<(uint32_t)jobs.size(), 64>>>(index->d_text, b.query, sc, b.tjobs, (uint32_t)jobs.size(), b.off,
                                              b.mats, b.off2, b.ops, b.lens, b.endv);
        TB_TRY(hipGetLastError());
        std::vector<char> hops(nops);
        std::vector<uint32_t> lens(jobs.size());
        std::vector<int32_t> endv(jobs.size());
        TB_TRY(hipMemcpy(hops.data(), b.ops, nops, hipMemcpyDeviceToHost));
        TB_TRY(hipMemcpy(lens.data(), b.lens, lens.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
        TB_TRY(hipMemcpy(endv.data(), b.endv, endv.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (size_t q = 0; q < jobs.size(); ++q) {
            const size_t h = which[q];
            if (lens[q] == 0xFFFFFFFFu || endv[q] != aln[h].score) {
                set_error("alae_traceback: the transcript of hit %zu does not reach its score (internal error)", h);
                return ALAE_E_INTERNAL;
            }
            ops_of[h].assign(hops.begin() + (ptrdiff_t)ooff[q], hops.begin() + (ptrdiff_t)(ooff[q] + lens[q]));
            std::reverse(ops_of[h].begin(), ops_of[h].end());
        }
    }
    uint64_t total = 0;
    for (size_t h = 0; h < k; ++h) total += ops_of[h].size();
    char *all = (char *)malloc(total ? total : 1);
    if (!all) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    uint64_t at = 0;
    for (size_t h = 0; h < k; ++h) {
        aln[h].ops_offset = at;
        aln[h].ops_len = (uint32_t)ops_of[h].size();
        if (!ops_of[h].empty()) memcpy(all + at, ops_of[h].data(), ops_of[h].size());
        at += ops_of[h].size();
    }
    out->aln = aln.release();
    out->count = k;
    out->ops = all;
    out->ops_count = total;
    return ALAE_OK;
}

void alae_alignments_free(alae_alignments *a) {
    if (!a) return;
    delete[] a->aln;
    free(a->ops);
    memset(a, 0, sizeof(*a));
}

}  // extern "C"
