/*
 * alae.h -- C ABI of the MI355X exact local-alignment search library (libalae.so).
 *
 * Problem (Section 2.1, "Local alignment problem"; Algorithm 1): for a text T
 * of n characters, a query P of m characters, a scoring scheme
 * <s_a, s_b, s_g, s_s> and a threshold H, report every pair (query end j,
 * text end i) whose best local alignment score
 *
 *     A(i,j) = max(0, max over x <= i, y <= j of sim(T[x..i], P[y..j]))
 *
 * reaches H, together with A(i,j).  sim is the best global alignment score:
 * a substitution score per aligned column and a gap of r characters costing
 * s_g + r*s_s (Section 2.1).
 *
 * Method (Sections 2.2-5): the text's suffix trie is walked through an
 * FM-index of the reversed text (Section 5); each trie node X carries the
 * sparse row of M_X/G_a (Section 2.2) that survives the zero floor, the length
 * filter (Theorem 1), the score filter (Theorem 2), q-prefix seeding
 * (Theorem 3) and the domination test (Section 3.2); hits are spread to every
 * occurrence and the maximum per (j, i) is kept (Algorithm 1).
 *
 * Conventions for every entry point:
 *  - Indices are 0-based and inclusive: query_end in [0, m), text_end in [0, n).
 *  - Results are sorted ascending by (query_end, text_end), one record per pair.
 *  - Every call returns an alae_status; on error nothing is written to the
 *    caller's outputs and alae_last_error() describes the failure.
 *  - Input buffers stay owned by the caller and are copied; they may be freed
 *    as soon as the call returns.
 *  - An index is immutable after it is built or loaded and may be shared by
 *    threads; a workspace or a server must be used by one thread at a time.
 *  - No C++ exception crosses this interface.
 */
#ifndef ALAE_H
#define ALAE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ALAE_OK = 0,
    ALAE_E_ARG = 1,        /* null pointer, zero length, bad option value            */
    ALAE_E_ALPHABET = 2,   /* a character outside the alphabet                        */
    ALAE_E_SCORING = 3,    /* scoring scheme outside the model of Section 2.1         */
    ALAE_E_TOO_LONG = 4,   /* n or m beyond the library's 32-bit index limits         */
    ALAE_E_NOMEM = 5,      /* host or device allocation failed                        */
    ALAE_E_DEVICE = 6,     /* no usable GPU, or a HIP runtime error                   */
    ALAE_E_ADMISSION = 7,  /* a serving request does not fit the memory budget        */
    ALAE_E_INTERNAL = 8,   /* an internal consistency check failed                    */
    ALAE_E_IO = 9,         /* index file could not be read or written                 */
    ALAE_E_NOT_FOUND = 10  /* unknown request id                                      */
} alae_status;

typedef enum {
    ALAE_DNA = 0,     /* A C G T (case-insensitive)                         -> codes 0..3  */
    ALAE_PROTEIN = 1  /* A R N D C Q E G H I L K M F P S T W Y V (case-ins.) -> codes 0..19 */
} alae_alphabet;

/*
 * Scoring scheme (Section 2.1).  With use_matrix == 0 an identical pair
 * scores sa (> 0) and any other pair sb (< 0).  With use_matrix != 0,
 * matrix points to sigma*sigma int8 scores, row-major, [text char][query
 * char]; it must be symmetric with a positive diagonal.  A gap of r
 * characters costs sg + r*ss with sg <= 0 and ss < 0 (Theorem 1 divides by
 * ss).  Example: the paper's default <1,-3,-5,-2> is
 * {0, 1, -3, NULL, -5, -2}.
 */
typedef struct {
    int32_t use_matrix;
    int32_t sa;
    int32_t sb;
    const int8_t *matrix;
    int32_t sg;
    int32_t ss;
} alae_scoring;

/* A result set.  Arrays are allocated by the library; release with alae_hits_free. */
typedef struct {
    uint32_t *query_end;
    uint64_t *text_end;
    int32_t *score;
    size_t count;
} alae_hits;

/* Counters of one search (all optional to read). */
typedef struct {
    uint64_t nodes;          /* trie nodes whose row was computed                      */
    uint64_t entries;        /* DP entries computed (live entries of all rows)         */
    uint64_t entries_diag;   /* entries fed only by the diagonal (no-gap region, Eq. 3) */
    uint64_t entries_gap2;   /* entries with two contributing predecessors             */
    uint64_t entries_gap3;   /* entries with three contributing predecessors           */
    uint64_t dominated;      /* states removed by the domination test (Section 3.2)    */
    uint64_t emitted;        /* hit records emitted before the max-merge               */
    uint64_t hits;           /* distinct (query end, text end) pairs reported          */
    uint64_t levels;         /* trie depths visited                                    */
    uint64_t retries;        /* launches run again with larger buffers after an overflow */
    uint64_t max_depth;      /* deepest trie node with a live entry                    */
    double device_ms;        /* device time of the search (events around the work)      */
    /* traffic and time per kernel family (roofline accounting) */
    uint64_t occ_reads;      /* occurrence-block reads of the level kernels (64-byte granules) */
    uint64_t sa_reads;       /* suffix-array reads locating new chains                     */
    uint64_t text_reads;     /* text granules read by the chain walkers                     */
    uint64_t frontier_bytes; /* level-kernel bytes: frontier nodes/rows in and out, hits    */
    uint64_t level_launches; /* launches of the level kernels                               */
    double level_ms;         /* device time of the level kernels                            */
    double start_ms;         /* device time of the chain-start kernel (locate, domination, no-gap walk) */
    double general_ms;       /* device time of the one-lane chain walker                     */
    double wide_ms;          /* device time of the one-wave chain walkers                    */
    uint64_t chain_steps;    /* chain nodes computed by one lane                             */
    uint64_t wide_steps;     /* chain nodes computed by one wave                             */
    uint64_t promoted;       /* chains handed to the wave walkers                            */
    uint64_t dominated_gapped; /* states removed by the gapped domination test               */
    uint64_t chain_bytes;    /* row bytes read and written by the chain walkers              */
    double merge_ms;         /* device time of the sort + max-merge of hit records          */
    /* reuse of duplicate score calculations (Section 4): entries whose values were
     * copied from an identical fork instead of computed; the reusing ratio of
     * Equation 6 is reused / (reused + entries) */
    uint64_t reused;
    uint64_t replay_chains;  /* chains whose row was recognised as copies of one fork  */
    uint64_t partitioned;    /* lane-queue chains the work predictor sent to the first wave pass */
    uint64_t leftover;       /* wave-queue chains walked after the concurrent pass            */
    double order_ms;         /* device time of features, predictions and the partition        */
    double level_lane_ms;    /* device time of the two trie-expansion kernels of the levels   */
                             /* (node phase, then one lane per child row), wide rows apart   */
    uint64_t level_lane_launches; /* levels that ran them                                  */
    uint64_t tail_chains;    /* chain items made from the frontier's tail (one per occurrence of a node) */
    uint64_t tail_depth;     /* depth at which the frontier's tail went to the chain walkers (0: never) */
    /* the wave walkers (one wave, or the waves of one block, per chain) */
    uint64_t wide_entries;   /* DP entries they computed (part of entries)                    */
    uint64_t wide_max_steps; /* most rows walked for one chain item                            */
    double live_ms;          /* span of the wave pass that runs beside the lane walker, first start to last end */
    double wide_slowest_ms;  /* the chain item that took a wave-walker block longest: its time ... */
    uint64_t wide_slowest_rows; /* ... and the rows it walked (a chain's rows depend on each other)  */
    uint64_t dominated_qgram;   /* seed states dropped by the q-gram domination table (Definition 1, Lemma 1) */
    double wide_slowest_start_ms; /* when the slowest wave-walker item began, after its pass began */
    uint64_t device_levels;  /* levels run device-driven (alae_search_opts.level_graph), part of levels */
    uint64_t graph_captures; /* batches of level slots captured as a graph (the others were replayed) */
} alae_stats;

/*
 * Learned frontier ordering.  A chain item (a trie node with one text
 * occurrence, walked along the text by one lane or one wave) is described by
 * ALAE_MLP_FEATURES numbers: log2(1 + depth) / 8, log2(1 + live entries) / 10,
 * max M / H, log2(1 + sum of M) / 20, max G_a / H, log2(1 + column span) / 16,
 * (columns left after the best entry) / L_max, the walker (0: one lane,
 * 1: one wave), and the fraction of positive substitution scores between the
 * next 32 (then 128) text characters the chain will read and the query
 * characters after its best entry.  Its measured work is DP entries computed
 * plus rows stepped, including the work of its continuation when a lane walk
 * is handed to the wave walker.
 * A trace records (features, work) for every item of a search; an alae_mlp
 * trained on log2(1 + work) orders the walkers' queues by predicted work,
 * largest first.  Ordering never changes the hit set.
 */
#define ALAE_MLP_FEATURES 10
#define ALAE_MLP_HIDDEN 32
#define ALAE_MLP_PARAMS (ALAE_MLP_HIDDEN * ALAE_MLP_FEATURES + ALAE_MLP_HIDDEN + \
                         ALAE_MLP_HIDDEN * ALAE_MLP_HIDDEN + ALAE_MLP_HIDDEN + ALAE_MLP_HIDDEN + 1)

typedef struct alae_mlp alae_mlp;

typedef struct {
    float *features;   /* capacity * ALAE_MLP_FEATURES, caller-owned host memory */
    float *work;       /* capacity                                               */
    size_t capacity;
    size_t count;      /* out: items recorded (at most capacity)                 */
    size_t total;      /* out: items seen                                        */
} alae_trace;

/* Search options; pass NULL for the defaults. */
typedef struct {
    int32_t zero_floor_only;   /* 1: BWT-SW's rule alone (Section 2.4): every trie row is expanded
                                  while it holds a positive entry; no length filter (Theorem 1),
                                  score filter (Theorem 2), q-prefix seeding (Theorem 3, seeds at
                                  depth 1) or domination (Section 3.2).  Same hits, more work: the
                                  baseline of the filtering ratio (Equation 5).  Default 0.   */
    int32_t use_domination;    /* Section 3.2 domination: the q-gram table on the seeds    */
                               /* (Definition 1, Lemma 1) and the tests on states (default 1) */
    int32_t use_score_filter;  /* Theorem 2 (default 1)                                     */
    int32_t use_qprefix;       /* Theorem 3 q-prefix seeding (default 1)                    */
    int32_t use_reuse;         /* Section 4 reuse of duplicate forks (default 0)             */
    int32_t order_queues;      /* with order_model: 1 = lane-walker queue, 2 = wave-walker queue,
                                  3 = both; 0 = the default (2)                              */
    uint64_t entry_capacity;   /* frontier entries per level buffer, 0 = automatic          */
    uint64_t hit_capacity;     /* emitted hit records, 0 = automatic                        */
    alae_stats *stats;         /* filled when not NULL                                      */
    const alae_mlp *order_model; /* order the walkers' queues by predicted work (NULL: queue order) */
    alae_trace *trace;         /* record (features, work) of every chain item when not NULL */
    float partition_threshold; /* with order_model: predicted log2(1 + work) from which a lane-queue
                                  chain is walked by the wave walker from its start (<= 0: never) */
    /* launch shapes (alae_autotune picks them; none changes the hit set) */
    int32_t level_stage;        /* LDS stage entries per lane of the child phase: 2, 4 or 8 (0 = 4) */
    int32_t wide_blocks_per_cu; /* wave-walker blocks per compute unit, 1..8 (0 = 3)             */
    int32_t lane_waves_per_cu;  /* lane-walker waves per compute unit, 1..16 (0 = 8)             */
    /* 1: every level goes through the FM-index; 0 (default): once the frontier is small
       and has few occurrences, its nodes become chains, one per occurrence, walked along
       the text (the hit set is the same either way) */
    int32_t no_tail_split;
    /* batched searches: queries are taken in order in groups of at most this many columns
       (a longer query alone), one trie traversal per group; 0 = 2^19 */
    uint64_t batch_columns;
    /* device-driven levels: K in 1..64 runs the level loop in batches of K level slots with no
       host round trip between levels while the frontier holds at most 2^18 nodes, each batch
       a HIP graph captured once per buffer layout and start parity (kept in the workspace)
       and replayed; -K enqueues the same batches kernel by kernel (no graph).  Grids are
       sized for such a frontier and the kernels read the level's sizes and depth from device
       memory; a level that overflows a buffer, a larger frontier and the hand-over of the
       frontier's tail go back to the host.  0 (default): one host round trip a level.  The
       hit set is the same either way.  Not in the entry point that allocates nothing (there
       it is ignored). */
    int32_t level_graph;
} alae_search_opts;

/* Index options; pass NULL for the defaults. */
typedef struct {
    int32_t device;            /* HIP device ordinal used when the index goes to the GPU */
    int32_t builder;           /* 1: build on the host (SA-IS); 2: build on the GPU (prefix
                                  doubling) and keep the arrays resident there; 0 (default): the
                                  GPU for texts of 2^22 characters or more when the device exists,
                                  else the host.  Both give the same index. */
} alae_index_opts;

typedef struct alae_index alae_index;
typedef struct alae_workspace alae_workspace;
typedef struct alae_server alae_server;

/* Read-only description of an index. */
typedef struct {
    uint64_t n;                /* text length                                    */
    int32_t sigma;             /* 4 (DNA) or 20 (protein)                        */
    int32_t alphabet;          /* alae_alphabet                                  */
    uint64_t C[21];            /* C[c] = 1 + separators + #(text chars < c); C[sigma] = n + 1 */
    uint64_t dollar_row;       /* BWT row holding the terminator                 */
    uint64_t host_bytes;       /* bytes held on the host                         */
    uint64_t device_bytes;     /* bytes held on the device (0 until uploaded)    */
    uint64_t records;          /* records of the text (1 unless built from records) */
} alae_index_info;

/*
 * Build the FM-index of the reversed text with the terminator (Section 5:
 * the compressed suffix array of T^-1$, positions of T kept).  text holds n
 * characters of the given alphabet.  The suffix array stores, for every
 * BWT row, the 0-based text position where that occurrence ends (Section 5,
 * search (2): the start is the stored end minus |X| plus one); row 0 is the
 * terminator.  The index lives on the host until a search first needs it on
 * the device (the GPU builder leaves it there at once).  Errors: ALAE_E_ARG (null, n == 0), ALAE_E_ALPHABET,
 * ALAE_E_TOO_LONG (n >= 2^31 - 1), ALAE_E_NOMEM.
 */
alae_status alae_index_build(const char *text, size_t n, alae_alphabet alphabet, const alae_index_opts *opts,
                             alae_index **out);

/* Same, from already encoded characters (codes 0..sigma-1). */
alae_status alae_index_build_codes(const uint8_t *codes, size_t n, alae_alphabet alphabet,
                                   const alae_index_opts *opts, alae_index **out);

/*
 * A database of k records (Section 2.2 concatenates the sequences of a
 * database into one text): the records' codes lie end to end in `codes`
 * (lens[r] > 0 codes each) and the library joins them with a separator that
 * no alignment crosses, so every hit lies inside one record and is exactly
 * what a search of that record alone reports.  Text positions (hit text ends,
 * alae_index_range, the suffix array) count the separators: record r starts
 * at sum(lens[0..r-1]) + r.  The separator sorts after the terminator and
 * before every character; the occ blocks hold one byte per BWT character.
 * Errors as alae_index_build_codes, and ALAE_E_ARG for an empty record.
 */
alae_status alae_index_build_records(const uint8_t *codes, const size_t *lens, size_t k, alae_alphabet alphabet,
                                     const alae_index_opts *opts, alae_index **out);

/* The record holding text position text_pos and the offset inside it.
 * ALAE_E_ARG for a separator or a position past the text. */
alae_status alae_index_record_of(const alae_index *index, uint64_t text_pos, uint64_t *record, uint64_t *offset);

/*
 * Text-sharded index: the text is cut into shards of shard_len text ends,
 * each indexed from `overlap` characters before its first end (one FM-index
 * per shard, built as alae_index_build_codes builds one).  A search runs on
 * every shard and keeps each shard's hits whose text end it owns; by
 * Theorem 1 (Equation 1) this is exactly the whole text's hit set when the
 * query's L_max is at most overlap + 1, which alae_sharded_search checks
 * (ALAE_E_TOO_LONG otherwise).  Text ends are global (up to 2^36).  With
 * max_resident > 0 at most that many shards keep their device copy between
 * searches; the others stay in host memory and are uploaded for their turn
 * and released after it.  The union of the shards' hits is sorted on the GPU.
 * Errors as alae_index_build_codes and alae_search.
 */
typedef struct alae_sharded alae_sharded;
alae_status alae_sharded_build(const uint8_t *codes, uint64_t n, alae_alphabet alphabet, uint64_t shard_len,
                               uint64_t overlap, uint32_t max_resident, const alae_index_opts *opts,
                               alae_sharded **out);
void alae_sharded_free(alae_sharded *sharded);
alae_status alae_sharded_search(const alae_sharded *sharded, const char *query, size_t m,
                                const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                                alae_hits *out);

/* Write / read a versioned binary image of the index.  Errors: ALAE_E_IO, ALAE_E_NOMEM. */
alae_status alae_index_save(const alae_index *index, const char *path);
alae_status alae_index_load(const char *path, const alae_index_opts *opts, alae_index **out);

/* Release an index and its device copy.  NULL is ignored. */
void alae_index_free(alae_index *index);

alae_status alae_index_get_info(const alae_index *index, alae_index_info *out);

/* Copies of the host arrays, for inspection: sa_end has n+1 entries (row 0,
 * the terminator, holds UINT32_MAX); bwt has n+1 codes (255 for the
 * terminator). */
alae_status alae_index_copy_sa(const alae_index *index, uint32_t *sa_end);
alae_status alae_index_copy_bwt(const alae_index *index, uint8_t *bwt);

/*
 * Backward search on the host (Section 2.3 and Section 5, search (1)):
 * the BWT rows [lo, hi] whose occurrences end with `pattern` read forward
 * in T.  Empty when lo > hi.  Used by tests and by query preparation.
 */
alae_status alae_index_range(const alae_index *index, const uint8_t *pattern_codes, size_t len, uint64_t *lo,
                             uint64_t *hi);

/*
 * One search of one query (host buffers in and out).  query holds m
 * characters of the index's alphabet.  On success *out receives the sorted
 * hit set (library-allocated; free with alae_hits_free).  The index is
 * uploaded to the device on first use.  Errors: ALAE_E_ARG, ALAE_E_ALPHABET,
 * ALAE_E_SCORING, ALAE_E_TOO_LONG, ALAE_E_NOMEM, ALAE_E_DEVICE.
 */
alae_status alae_search(const alae_index *index, const char *query, size_t m, const alae_scoring *scoring,
                        int32_t H, const alae_search_opts *opts, alae_hits *out);

/*
 * k queries searched together (the batched form).  The queries are laid end
 * to end and share one traversal of the text's trie (Section 2.3): a node is
 * expanded once for all of them, its sparse row holding the live columns of
 * every query, while no alignment crosses from one query into the next (no
 * diagonal step, gap, seed q-gram or domination window spans a boundary;
 * U(j) of Theorem 2 runs to the end of j's own query; L_max of Theorem 1 is
 * that of the longest query, which only loosens the filter).  outs (k
 * elements, caller-owned array) receives k library-allocated result sets,
 * outs[i] exactly what alae_search returns for query i alone (an empty query
 * gets an empty set).  At most 65,536 non-empty queries.  On error no result
 * set is left allocated.  Errors as alae_search.
 */
alae_status alae_search_batch(const alae_index *index, const char *const *queries, const size_t *lens, size_t k,
                              const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                              alae_hits *outs);

void alae_hits_free(alae_hits *hits);

/*
 * Device-resident form.  A workspace owns the device buffers a search needs
 * (frontier levels, hit records, sort buffers) and keeps them between
 * searches.  alae_search_device takes the query as device memory holding
 * codes 0..sigma-1 and leaves the sorted result on the device, where
 * alae_workspace_result returns pointers into the workspace (valid until the
 * next search on it): keys[k] = (query_end << 32) | text_end, scores[k].
 * stream is a hipStream_t (NULL = the default stream); the call returns when
 * the result is complete on that stream.
 */
alae_status alae_workspace_create(const alae_index *index, alae_workspace **out);
void alae_workspace_free(alae_workspace *ws);
alae_status alae_search_device(alae_workspace *ws, const uint8_t *d_query_codes, size_t m,
                               const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                               void *stream, size_t *hit_count);
/*
 * Launch-shape autotuner.  Times searches of one device-resident query (as in
 * alae_search_device) with the launch shapes of alae_search_opts changed one
 * at a time (coordinate descent: wave-walker blocks per CU in {2,3,4,6},
 * lane-walker waves per CU in {4,8,12}, child-phase LDS stage in {2,4,8},
 * level_graph in {0,8}; a change is kept when it is at least 1% faster), each timing the mean device
 * time of `reps` searches after one warm-up search.  opts is in/out: its other
 * fields are used as given (trace is ignored) and the chosen shapes are
 * written back.  Every trial must return the same hit count, otherwise
 * ALAE_E_INTERNAL.  The workspace result afterwards is that of the last trial.
 */
typedef struct {
    int32_t level_stage, wide_blocks_per_cu, lane_waves_per_cu;
    double ms;  /* mean device time of a search with these shapes */
    int32_t level_graph;
} alae_tune_trial;
typedef struct {
    double default_ms;         /* with the shapes passed in (0 = defaults)  */
    double best_ms;            /* with the chosen shapes                     */
    int32_t trials;            /* entries of trial[] filled                  */
    alae_tune_trial trial[16];
} alae_tune_report;
alae_status alae_autotune(alae_workspace *ws, const uint8_t *d_query_codes, size_t m, const alae_scoring *scoring,
                          int32_t H, alae_search_opts *opts, int32_t reps, void *stream, alae_tune_report *report);

/*
 * Device-resident batch: d_query_codes holds the k queries end to end
 * (lens[i] > 0 codes each, host array lens).  The workspace result is then
 * grouped by query, in query order, each group sorted as a single search
 * would sort it, with keys holding query-local columns; after the call
 * alae_workspace_batch_offsets fills offsets[0..k] (host array of k+1) so
 * that query i owns records offsets[i] .. offsets[i+1]-1.
 */
alae_status alae_search_device_batch(alae_workspace *ws, const uint8_t *d_query_codes, const size_t *lens, size_t k,
                                     const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                                     void *stream, size_t *hit_count);
alae_status alae_workspace_batch_offsets(const alae_workspace *ws, size_t *offsets, size_t k);
alae_status alae_workspace_result(const alae_workspace *ws, const uint64_t **d_keys, const int32_t **d_scores,
                                  size_t *count);
/* Copy the workspace result into caller-owned buffers of at least `count`
 * elements: device memory, or pinned host memory (hipHostMalloc) to take the
 * hits off the GPU (asynchronous on `stream`, a hipStream_t or NULL). */
alae_status alae_workspace_copy_result(const alae_workspace *ws, uint64_t *d_keys, int32_t *d_scores, void *stream);

/* Put the index on its device now (otherwise the first search does).
 * Idempotent.  Errors: ALAE_E_ARG, ALAE_E_DEVICE. */
alae_status alae_index_upload(const alae_index *index);

/*
 * For callers that cannot allocate device memory (code that may not call
 * hipMalloc: tight serving loops, harnesses that forbid it).  The same search
 * as alae_search_device (same kernels, same result), with every buffer it
 * needs cut from one fixed array of ALAE_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends; the call
 * makes no device allocation and frees nothing.
 *   index:     already on the device (alae_index_upload or any search);
 *              otherwise ALAE_E_ARG.
 *   d_query_codes: m codes 0..sigma-1 in device memory.
 *   d_keys, d_scores: caller-owned device arrays of `capacity` records that
 *              receive the sorted result, keys as in alae_workspace_result
 *              ((query_end << 32) | text_end).  Complete when the call
 *              returns (it synchronises `stream`, a hipStream_t or NULL).
 *   *hit_count: the number of records written.
 *   opts:      as alae_search_device, except that order_model and trace are
 *              not accepted (ALAE_E_ARG).
 * Limits: a search whose buffers would not fit the fixed array fails with
 * ALAE_E_NOMEM (message says so; nothing is written); a result larger than
 * `capacity` fails with ALAE_E_NOMEM and sets *hit_count to the size needed,
 * writing nothing else.  The first call on a device looks up the array's
 * address there and creates that device's stream and timing events (no
 * device memory).  All calls on one GPU share its array, which keeps the last
 * call's contents; the library clears what must start at zero.  Calls that
 * overlap on one GPU would race on the array, so the library makes them take
 * turns (a second call waits for the first to return).
 */
#define ALAE_NOALLOC_SCRATCH_BYTES (256ull << 20)
alae_status alae_search_device_noalloc(const alae_index *index, const uint8_t *d_query_codes, size_t m,
                                       const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                                       void *stream, uint64_t *d_keys, int32_t *d_scores, size_t capacity,
                                       size_t *hit_count);

/*
 * Serving with continuous batching.  The server keeps the index resident and
 * runs max_inflight slots (a workspace, a HIP stream and a worker thread
 * each; default 4, or 2 for texts of 2^28 characters or more, where one
 * search already fills the GPU) at once, so the kernels of different
 * requests overlap on the device.
 * A request is admitted when a slot is free and the device-memory budget has
 * room for its estimated rows (two trie levels of m columns with
 * max(64, 2000 (n/1e9)^0.6) live 20-byte entries per column, n the text
 * length, doubled for buffer growth, plus the profile); requests are admitted in arrival order, and a
 * slot takes the head of the queue together with the requests right behind
 * it that share its scoring and threshold (up to max_batch requests, 2^20
 * query columns and a slot's share of the budget), running them as one
 * batched search.  After a search that held more than a slot's share (one
 * request larger than that) the slot frees the buffers it grew.  Every request's result is exactly what
 * alae_search returns for it alone.
 *   submit: copies the query; *req_id identifies it.  ALAE_E_ADMISSION if
 *           its estimate exceeds the whole budget (it could never run).
 *   poll:   ALAE_OK with the result (library-allocated, free with
 *           alae_hits_free) once done; with wait == 0 a pending request
 *           gives ALAE_OK and out->count == SIZE_MAX; ALAE_E_NOT_FOUND for
 *           an unknown or already collected id; a failed search returns
 *           its own status.
 *   get_stats: counts and latency percentiles (submit to completion) of the
 *           requests completed since creation or the last reset_stats.
 * destroy waits for the requests already admitted and drops the rest.
 */
typedef struct {
    uint64_t memory_budget;    /* device bytes for in-flight rows, 0 = half the free memory */
    int32_t max_inflight;      /* slots running at once (1..16), 0 = 4 (2 for n >= 2^28)   */
    int32_t max_batch;         /* requests per batched search, 0 = 16                       */
} alae_server_opts;

typedef struct {
    uint64_t submitted, completed, rejected, queued;
    uint64_t batches;          /* searches run (a batch counts once)                 */
    double mean_batch;         /* requests per search                                */
    double p50_ms, p99_ms, mean_ms, max_ms;  /* submit-to-completion latency        */
    double span_s;             /* first submit to last completion                    */
} alae_server_stats;

alae_status alae_server_create(const alae_index *index, const alae_server_opts *opts, alae_server **out);
alae_status alae_server_submit(alae_server *srv, const char *query, size_t m, const alae_scoring *scoring,
                               int32_t H, uint64_t *req_id);
alae_status alae_server_poll(alae_server *srv, uint64_t req_id, int wait, alae_hits *out);
alae_status alae_server_get_stats(alae_server *srv, alae_server_stats *out);
void alae_server_reset_stats(alae_server *srv);
void alae_server_destroy(alae_server *srv);

/*
 * The work predictor (feature layout above).  Parameters are fp32, laid out
 * as W1[32][F] (row = output unit), b1[32], W2[32][32], b2[32], W3[32], b3;
 * hidden units use ReLU.  All computation runs in the library's own HIP
 * kernels on `device`.  The loss is 0.5 * mean over samples of
 * (prediction - target)^2.
 *   create: He-uniform weights from seed, zero biases.
 *   predict: y[i] for the n feature rows x (host arrays).
 *   loss_grad: the loss and its gradient with respect to every parameter.
 *   train: epochs of Adam (beta 0.9 / 0.999) over shuffled minibatches;
 *          final_loss (nullable) gets the loss over all samples afterwards.
 * A model must not be used by two threads at once.
 */
alae_status alae_mlp_create(int device, uint64_t seed, alae_mlp **out);
void alae_mlp_free(alae_mlp *net);
alae_status alae_mlp_get_params(const alae_mlp *net, float *params);
alae_status alae_mlp_set_params(alae_mlp *net, const float *params);
alae_status alae_mlp_predict(alae_mlp *net, const float *x, size_t n, float *y);
alae_status alae_mlp_loss_grad(alae_mlp *net, const float *x, const float *t, size_t n, double *loss, float *grad);
alae_status alae_mlp_train(alae_mlp *net, const float *x, const float *t, size_t n, uint32_t epochs,
                           uint32_t batch, float lr, uint64_t seed, double *final_loss);

/*
 * Alignment starts and transcripts of reported cells (the paper's A(i,j).pos,
 * Section 2.1, Table 1; Algorithm 1 keeps the position with the maximum).
 * For each cell k (query_ends[k], text_ends[k], scores[k]) -- typically
 * records of a search result -- the optimal local alignment ending there is
 * located: among the alignments scoring A(i,j) the one with the largest text
 * start, then the largest query start (this makes .pos unique).  Its
 * transcript lists one op per alignment column from the start: 'M' a text
 * and a query character aligned, 'D' a text character against a gap, 'I' a
 * query character against a gap; its score (substitutions plus sg + r*ss per
 * maximal gap run) is A(i,j).  Runs on the index's GPU (one wave per cell).
 *   out->aln[k].status: ALAE_OK; ALAE_E_ARG when the cell's score is not
 *     A(i,j) (or the position is outside the text or query or a separator);
 *     ALAE_E_TOO_LONG when the search window (2^30 cells) or the transcript's
 *     matrices (2 GiB) would exceed the limits (the start is kept for the
 *     latter, with no ops).
 * Arrays are library-allocated; free with alae_alignments_free.  Errors of
 * the whole call: ALAE_E_ARG, ALAE_E_ALPHABET, ALAE_E_SCORING, ALAE_E_DEVICE.
 */
typedef struct {
    uint64_t text_start;   /* 0-based first text position of the alignment  */
    uint32_t query_start;  /* 0-based first query position                  */
    int32_t score;         /* A(i,j) as given                               */
    uint64_t ops_offset;   /* first op of the transcript in alae_alignments.ops */
    uint32_t ops_len;
    int32_t status;
} alae_alignment;
typedef struct {
    alae_alignment *aln;
    size_t count;
    char *ops;
    uint64_t ops_count;
} alae_alignments;
alae_status alae_traceback(const alae_index *index, const char *query, size_t m, const alae_scoring *scoring,
                           const uint32_t *query_ends, const uint64_t *text_ends, const int32_t *scores, size_t k,
                           alae_alignments *out);
void alae_alignments_free(alae_alignments *alignments);

/*
 * Threshold from an E-value (Section 7: H = ceil((ln(K m n) - ln E) / lambda),
 * with E = K m n exp(-lambda S)).  alae_karlin_altschul computes lambda, K and
 * the relative entropy H of ungapped local alignment scores (Karlin and
 * Altschul 1990) for a scoring scheme and a residue background (sigma
 * frequencies, normalised; NULL = uniform): lambda is the positive root of
 * sum p_a p_b exp(lambda s(a,b)) = 1 and K comes from the series of Karlin and
 * Altschul.  Gap scores are not used: for gapped scoring these are the
 * ungapped statistics (BLAST's gapped tables are not part of this library),
 * whose threshold is lower than a gapped one, so no hit a gapped threshold
 * reports is lost.  ALAE_E_SCORING unless the expected pair score is negative
 * and some pair score positive.  alae_evalue_threshold gives H (at least 1)
 * for query length m, text length n and E-value evalue > 0.
 */
typedef struct {
    double lambda;
    double K;
    double H;  /* relative entropy, nats per aligned pair */
} alae_karlin;
alae_status alae_karlin_altschul(const alae_scoring *scoring, alae_alphabet alphabet, const double *background,
                                 alae_karlin *out);
alae_status alae_evalue_threshold(const alae_karlin *stats, uint64_t m, uint64_t n, double evalue, int32_t *H);

/* Message for the last failing call on this thread. */
const char *alae_last_error(void);

/* Library version string. */
const char *alae_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ALAE_H */
