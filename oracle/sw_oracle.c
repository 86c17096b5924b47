/*
 * Plain CPU oracle for the local-alignment problem with affine gaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU search path.
 *
 * What it computes (Section 2.1, "Local alignment problem", and Algorithm 1
 * BASIC, which initialises every A(i,j) to 0, keeps the maximum and returns
 * the entries that reach H):
 *
 *     A(i,j) = max(0, max over x <= i, y <= j of sim(T[x..i], P[y..j]))
 *
 * where sim is the best global alignment score under the scoring scheme of
 * Section 2.1: a substitution score per aligned column and a gap of r
 * characters costing sg + r*ss (sg <= 0, ss < 0).  The output is every
 * (j, i, A(i,j)) with A(i,j) >= H.
 *
 * Algorithm: the textbook Smith-Waterman recurrence with Gotoh's three
 * states, row by row over the text with O(m) memory and 64-bit scores.
 * E is the state "text character aligned with a gap" (the paper's G_a),
 * F the state "query character aligned with a gap" (the paper's G_b):
 *
 *     E(i,j) = max(E(i-1,j) + ss, H(i-1,j) + sg + ss)
 *     F(i,j) = max(F(i,j-1) + ss, H(i,j-1) + sg + ss)
 *     H(i,j) = max(0, H(i-1,j-1) + s(T[i],P[j]), E(i,j), F(i,j))
 *
 * Parallelism (optional): the text is cut into chunks and each chunk is
 * recomputed from an all-zero row placed L_max rows before it.  This is exact
 * because, by Theorem 1 (Equation 1), an alignment that scores at least H
 * spans at most L_max = max(m, m + floor((H - (smax*m + sg)) / ss)) text
 * characters, so the best alignment of every reported cell starts inside the
 * recomputed rows.  A single thread uses no chunking at all.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NEG_INF (INT64_MIN / 4)

typedef struct {
    int64_t *qend;  /* j, 0-based query end   */
    int64_t *tend;  /* i, 0-based text end    */
    int64_t *score; /* A(i,j)                 */
    int64_t count;
    int64_t cap;
    int64_t cells;  /* DP cells evaluated     */
} oracle_hits;

static int hits_push(oracle_hits *h, int64_t j, int64_t i, int64_t s) {
    if (h->count == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        int64_t *a = (int64_t *)realloc(h->qend, (size_t)nc * sizeof(int64_t));
        if (!a) return -1;
        h->qend = a;
        a = (int64_t *)realloc(h->tend, (size_t)nc * sizeof(int64_t));
        if (!a) return -1;
        h->tend = a;
        a = (int64_t *)realloc(h->score, (size_t)nc * sizeof(int64_t));
        if (!a) return -1;
        h->score = a;
        h->cap = nc;
    }
    h->qend[h->count] = j;
    h->tend[h->count] = i;
    h->score[h->count] = s;
    h->count++;
    return 0;
}

static inline int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* Rows [row_begin, row_end) of the text, starting from a zero row above
 * row_begin; cells in rows >= row_emit that reach H are appended. */
static int sw_rows(const uint8_t *T, int64_t row_begin, int64_t row_emit, int64_t row_end,
                   const uint8_t *P, int64_t m, const int32_t *sub, int32_t sigma,
                   int64_t sg, int64_t ss, int64_t H, oracle_hits *out) {
    int64_t *Hprev = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    int64_t *Eprev = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    if (!Hprev || !Eprev) {
        free(Hprev);
        free(Eprev);
        return -1;
    }
    for (int64_t j = 0; j <= m; j++) {
        Hprev[j] = 0;
        Eprev[j] = ORACLE_NEG_INF;
    }
    const int64_t open_ext = sg + ss;
    for (int64_t i = row_begin; i < row_end; i++) {
        const int32_t *srow = sub + (size_t)T[i] * (size_t)sigma;
        int64_t Hleft = 0;              /* H(i, 0)           */
        int64_t F = ORACLE_NEG_INF;     /* F(i, 0)           */
        int64_t Hdiag = Hprev[0];       /* H(i-1, 0) = 0     */
        for (int64_t j = 1; j <= m; j++) {
            int64_t E = max2(Eprev[j] + ss, Hprev[j] + open_ext);
            F = max2(F + ss, Hleft + open_ext);
            int64_t h = Hdiag + (int64_t)srow[P[j - 1]];
            h = max2(h, E);
            h = max2(h, F);
            h = max2(h, 0);
            Hdiag = Hprev[j];
            Hprev[j] = h;
            Eprev[j] = E;
            Hleft = h;
            if (h >= H && i >= row_emit) {
                if (hits_push(out, j - 1, i, h)) {
                    free(Hprev);
                    free(Eprev);
                    return -1;
                }
            }
        }
    }
    out->cells += (row_end - row_begin) * m;
    free(Hprev);
    free(Eprev);
    return 0;
}

/* Equation 1 (Theorem 1), with the largest substitution score in place of s_a. */
int64_t oracle_lmax(int64_t m, int64_t smax, int64_t sg, int64_t ss, int64_t H) {
    /* floor((H - (smax*m + sg)) / ss) with ss < 0 */
    int64_t num = H - (smax * m + sg);
    int64_t q = num / ss;
    if ((num % ss != 0) && ((num < 0) != (ss < 0))) q -= 1;
    int64_t v = m + q;
    return v > m ? v : m;
}

typedef struct {
    const uint8_t *T;
    const uint8_t *P;
    const int32_t *sub;
    int64_t m, sg, ss, H;
    int32_t sigma;
    int64_t row_begin, row_emit, row_end;
    oracle_hits out;
    int rc;
} chunk_job;

static void *chunk_main(void *arg) {
    chunk_job *c = (chunk_job *)arg;
    c->rc = sw_rows(c->T, c->row_begin, c->row_emit, c->row_end, c->P, c->m, c->sub, c->sigma,
                    c->sg, c->ss, c->H, &c->out);
    return NULL;
}

/*
 * Hits (j, i, A(i,j)) with A >= H and text end i in [t_lo, t_hi), in
 * increasing (i, j) order.  sub is a sigma x sigma row-major table indexed
 * [text char][query char].  nthreads <= 1 runs one plain pass from row 0.
 * Returns 0 on success, -1 on allocation failure, -2 on bad arguments.
 */
int oracle_sw_hits(const uint8_t *T, int64_t n, const uint8_t *P, int64_t m,
                   const int32_t *sub, int32_t sigma, int32_t sg, int32_t ss, int32_t H,
                   int64_t t_lo, int64_t t_hi, int32_t nthreads, oracle_hits *out) {
    memset(out, 0, sizeof(*out));
    if (n < 0 || m <= 0 || sigma <= 0 || ss >= 0 || sg > 0 || H < 1) return -2;
    if (t_lo < 0) t_lo = 0;
    if (t_hi > n) t_hi = n;
    if (t_hi <= t_lo) return 0;
    for (int64_t i = 0; i < n; i++)
        if (T[i] >= sigma) return -2;
    for (int64_t j = 0; j < m; j++)
        if (P[j] >= sigma) return -2;

    if (nthreads <= 1) {
        return sw_rows(T, 0, t_lo, t_hi, P, m, sub, sigma, sg, ss, H, out);
    }
    int64_t smax = sub[0];
    for (int64_t k = 0; k < (int64_t)sigma * sigma; k++)
        if (sub[k] > smax) smax = sub[k];
    int64_t lmax = oracle_lmax(m, smax, sg, ss, H);

    int64_t span = t_hi - t_lo;
    int64_t nchunks = nthreads;
    if (nchunks > span) nchunks = span;
    chunk_job *jobs = (chunk_job *)calloc((size_t)nchunks, sizeof(chunk_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nchunks, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -1;
    }
    for (int64_t c = 0; c < nchunks; c++) {
        int64_t lo = t_lo + span * c / nchunks;
        int64_t hi = t_lo + span * (c + 1) / nchunks;
        int64_t start = lo - lmax;
        if (start < 0) start = 0;
        jobs[c] = (chunk_job){T, P, sub, m, sg, ss, H, sigma, start, lo, hi, {0}, 0};
        pthread_create(&th[c], NULL, chunk_main, &jobs[c]);
    }
    int rc = 0;
    for (int64_t c = 0; c < nchunks; c++) {
        pthread_join(th[c], NULL);
        if (jobs[c].rc) rc = jobs[c].rc;
    }
    if (rc == 0) {
        for (int64_t c = 0; c < nchunks && rc == 0; c++) {
            for (int64_t k = 0; k < jobs[c].out.count; k++) {
                if (hits_push(out, jobs[c].out.qend[k], jobs[c].out.tend[k], jobs[c].out.score[k])) {
                    rc = -1;
                    break;
                }
            }
            out->cells += jobs[c].out.cells;
        }
    }
    for (int64_t c = 0; c < nchunks; c++) {
        free(jobs[c].out.qend);
        free(jobs[c].out.tend);
        free(jobs[c].out.score);
    }
    free(jobs);
    free(th);
    return rc;
}

/* The full (n+1) x (m+1) matrix H of the recurrence above, row-major, for
 * small inputs (tests compare it cell by cell against exhaustive search). */
int oracle_sw_matrix(const uint8_t *T, int64_t n, const uint8_t *P, int64_t m,
                     const int32_t *sub, int32_t sigma, int32_t sg, int32_t ss, int64_t *Hout) {
    if (n < 0 || m < 0 || ss >= 0 || sg > 0) return -2;
    int64_t *Eprev = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    if (!Eprev) return -1;
    for (int64_t j = 0; j <= m; j++) {
        Hout[j] = 0;
        Eprev[j] = ORACLE_NEG_INF;
    }
    const int64_t open_ext = (int64_t)sg + ss;
    for (int64_t i = 1; i <= n; i++) {
        int64_t *row = Hout + i * (m + 1);
        const int64_t *up = Hout + (i - 1) * (m + 1);
        row[0] = 0;
        int64_t F = ORACLE_NEG_INF;
        for (int64_t j = 1; j <= m; j++) {
            int64_t E = max2(Eprev[j] + ss, up[j] + open_ext);
            F = max2(F + ss, row[j - 1] + open_ext);
            int64_t h = up[j - 1] + (int64_t)sub[(size_t)T[i - 1] * sigma + P[j - 1]];
            h = max2(h, E);
            h = max2(h, F);
            h = max2(h, 0);
            row[j] = h;
            Eprev[j] = E;
        }
    }
    free(Eprev);
    return 0;
}

/* G[a*(p_len+1) + b] = sim(T[t_len-a .. t_len-1], P[p_len-b .. p_len-1]): the best
 * global alignment score of the last a text and last b query characters
 * (Section 2.1: substitution scores, a maximal gap run of r characters costs
 * sg + r*ss), for every a <= t_len, b <= p_len.  Textbook Gotoh over the
 * reversed strings, with the state that ends in a text gap (E), a query gap
 * (F) or an aligned pair. */
int oracle_global_suffix(const uint8_t *T, int64_t t_len, const uint8_t *P, int64_t p_len, const int32_t *sub,
                         int32_t sigma, int32_t sg, int32_t ss, int64_t *G) {
    if (t_len < 0 || p_len < 0 || ss >= 0 || sg > 0) return -2;
    const int64_t w = p_len + 1;
    int64_t *E = (int64_t *)malloc((size_t)(t_len + 1) * (size_t)w * sizeof(int64_t));
    int64_t *F = (int64_t *)malloc((size_t)(t_len + 1) * (size_t)w * sizeof(int64_t));
    if (!E || !F) {
        free(E);
        free(F);
        return -1;
    }
    for (int64_t a = 0; a <= t_len; a++) {
        for (int64_t b = 0; b <= p_len; b++) {
            const int64_t at = a * w + b;
            if (a == 0 && b == 0) {
                G[at] = 0;
                E[at] = F[at] = ORACLE_NEG_INF;
                continue;
            }
            int64_t e = ORACLE_NEG_INF, f = ORACLE_NEG_INF, m = ORACLE_NEG_INF;
            if (a > 0) e = max2(E[at - w] + ss, G[at - w] + sg + ss);
            if (b > 0) f = max2(F[at - 1] + ss, G[at - 1] + sg + ss);
            if (a > 0 && b > 0)
                m = G[at - w - 1] + sub[(size_t)T[t_len - a] * sigma + P[p_len - b]];
            E[at] = e;
            F[at] = f;
            G[at] = max2(m, max2(e, f));
        }
    }
    free(E);
    free(F);
    return 0;
}

void oracle_hits_free(oracle_hits *h) {
    free(h->qend);
    free(h->tend);
    free(h->score);
    memset(h, 0, sizeof(*h));
}
