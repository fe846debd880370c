/*
 * swmi — exact Smith-Waterman protein database search on AMD MI355X (gfx950).
 *
 * C ABI of the shared library libswmi.so.  Every entry point returns 0 on
 * success or a negative SW_E* code; sw_last_error() then returns a message
 * (thread-local, valid until the next call on the same thread).  No C++
 * exception crosses this boundary.
 *
 * The method (section II.A, Eq. 1): for a query Q (length m) and a database
 * sequence S (length n) the score is max over i, j of H(i,j) with
 *   H(i,j) = max{0, H(i-1,j-1) + M[Q[j]][S[i]], E(i,j), F(i,j)}
 *   E(i,j) = max{E(i-1,j) - alpha, H(i-1,j) - beta}
 *   F(i,j) = max{F(i,j-1) - alpha, H(i,j-1) - beta}
 * and H, E, F zero on row 0 and column 0.  alpha is the gap extension
 * penalty, beta = gap open + extension.  The matrix row is the query residue
 * (as in the query profile of section III.B.2).  Scores are exact int32.
 *
 * Memory: every pointer argument is HOST memory unless its name ends in
 * _dev.  The library copies what it needs; callers keep ownership of their
 * buffers and may free them as soon as a call returns.  The only objects the
 * library allocates for the caller are the opaque sw_db / sw_server handles,
 * released by sw_db_close / sw_server_stop.
 *
 * Threads: calls on one sw_db are serialised by an internal lock.  The server
 * (sw_server_*) is the concurrent path; its submit/wait may be called from any
 * number of threads.
 */
#ifndef SWMI_H
#define SWMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_OK        0
#define SW_EINVAL   (-1)   /* bad argument: code >= alphabet, alphabet not in 1..32,
                              alpha < 0, beta < alpha, beta > 2^30, qlen < 1 or > 2^24,
                              subject longer than 2^24, k < 1 or k > SW_MAX_K, NULL pointer */
#define SW_ENOMEM   (-2)   /* host or device allocation failed */
#define SW_EDEVICE  (-3)   /* a HIP runtime call or kernel launch failed */
#define SW_EBUSY    (-4)   /* server: request queue full (back-pressure) */
#define SW_ENOTFOUND (-5)  /* server: unknown or already collected ticket */
#define SW_ESTOPPED (-6)   /* server: stopped before the request completed */

#define SW_MAX_ALPHABET 32
#define SW_MAX_LEN      (1 << 24)
#define SW_MAX_K        4096

typedef struct sw_db sw_db;
typedef struct sw_server sw_server;

/* Scoring scheme (section II.A).  matrix: alphabet*alphabet int8, row-major,
 * matrix[q*alphabet + s] scores query residue q against subject residue s.
 * 0 <= alpha <= beta <= 2^30.  alphabet must equal the database's. */
typedef struct sw_scoring {
    int32_t alphabet;
    const int8_t *matrix;
    int32_t alpha;
    int32_t beta;
} sw_scoring;

/* Options for sw_db_open; pass NULL for defaults (all fields 0). */
typedef struct sw_db_opts {
    int32_t device;          /* HIP device ordinal; <= 0 means device 0 */
    int32_t long_threshold;  /* subjects longer than this use the wave-per-pair kernel;
                                0 = chosen from the length distribution, -1 = none
                                (all subjects use the lane-per-subject kernel), 1 = all
                                subjects use the wave-per-pair kernel */
    int32_t reserved[6];
} sw_db_opts;

/* Lane tiers of the lane-per-subject kernel. */
#define SW_TIER_AUTO  0
#define SW_TIER_F16X2 1   /* two subjects per 32-bit lane, packed fp16 holding exact
                             integers, values offset by up to 35 x alpha; exact while the
                             best score < 1920 - 36 x alpha, else the pair is flagged and
                             recomputed in int32 (every pair when alpha > 53).  The planner
                             uses it when alpha <= 28 and SW_TIER_I16X2 otherwise. */
#define SW_TIER_I16X2 2   /* two subjects per lane, saturating int16; exact below 32767 */

/* Search tuning knobs (planner overrides; 0 = let the planner/autotuner choose). */
typedef struct sw_search_opts {
    int32_t tier;           /* SW_TIER_* */
    int32_t strip;          /* query columns per register strip: 16, 32 or 64 */
    int32_t waves;          /* waves per workgroup of the lane-per-subject kernel: 4, 6, 8 */
    int32_t sat_threshold;  /* test knob: if > 0, a narrow-tier lane whose best score reaches
                               min(this, tier ceiling) is flagged and recomputed in int32 */
    int32_t graph;          /* sw_db_search_batch: 0 = capture the device work of a batch shape in
                               a HIP graph and replay it on later calls of that shape, -1 = launch
                               eagerly every time */
    int32_t profile;        /* substitution scores of the lane-per-subject kernel: SW_PROFILE_PAIR
                               (0) or SW_PROFILE_SCORE; the planner never picks the latter itself */
    int32_t reserved[2];
} sw_search_opts;

/* Profiles of the lane-per-subject kernel (sw_search_opts.profile). */
#define SW_PROFILE_PAIR  0   /* query profile per strip, read at each lane's subject-residue pair
                                (section III.B.2; two subjects per 32-bit lane) */
#define SW_PROFILE_SCORE 1   /* score profile (section III.B.3): each lane's row of its subject
                                residues' scores against every query letter, read at the query
                                letter.  Taken only with the fp16 tier, strip 32, 4 waves and an
                                alphabet of at most 23 letters (searches through sw_db_search,
                                sw_db_search_dev, sw_db_topk and sw_db_search_batch); otherwise
                                the pair profile runs.  sw_stats.profile reports which ran. */

/* Statistics of the last search call on a database handle. */
typedef struct sw_stats {
    int64_t cells;            /* sum over queries of |Q| * sum |S| (real residues) */
    int64_t padded_cells;     /* cells actually evaluated, padding included */
    int64_t inter_cells;      /* real cells handled by the lane-per-subject kernel */
    int64_t recomputed_pairs; /* pairs flagged by a narrow tier and recomputed in int32 */
    int64_t intra_pairs;      /* pairs evaluated by the wave-per-pair kernel */
    double  kernel_ms;        /* device time of the alignment kernels (HIP events) */
    double  total_ms;         /* wall time of the whole call */
    double  inter_ms;         /* device time of the lane-per-subject kernel alone (-1 when the
                                 work ran as a graph, which is timed as a whole) */
    int32_t tier;             /* tier used */
    int32_t strip;            /* strip width used */
    int32_t waves;            /* waves per workgroup used */
    int32_t graphed;          /* 1 if the device work ran as a captured HIP graph */
    int32_t fused_long;       /* 1 if the long list (wave-per-pair, int32) ran inside the
                                 lane-per-subject kernel's work queue, 0 if as its own kernel */
    double  recompute_ms;     /* device time of the exact int32 recompute of flagged pairs
                                 (-1 when the work ran as a graph) */
    double  long_ms;          /* device time of the wave-per-pair kernel when it ran alone
                                 (no lane-per-subject work in the call, not fused); -1
                                 otherwise (a fused long list is timed in inter_ms) */
    int32_t profile;          /* SW_PROFILE_* of the lane-per-subject kernel */
    int32_t reserved0;
} sw_stats;

/* Open a database (section III, stage ii: sequences are sorted by length and
 * laid out for the device once).
 *   residues: concatenated codes, each < alphabet (offsets[n_seqs] bytes)
 *   offsets:  n_seqs + 1 non-decreasing int64, offsets[0] == 0
 *   n_seqs >= 0; zero-length sequences are allowed (score 0)
 * Copies everything to device memory; *out receives the handle. */
int sw_db_open(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs,
               int32_t alphabet, const sw_db_opts *opts, sw_db **out);

/* Release a database and its device memory.  NULL is ignored. */
void sw_db_close(sw_db *db);

/* Number of sequences in the database (-1 for NULL). */
int64_t sw_db_size(const sw_db *db);

/* Override planner choices for later searches on this handle (NULL resets). */
int sw_db_set_opts(sw_db *db, const sw_search_opts *opts);

/* Statistics of the last search on this handle. */
int sw_db_last_stats(sw_db *db, sw_stats *out);

/* Score one query against every database sequence (section II.A, Eq. 1).
 *   scores: n_seqs int32, in the caller's original database order
 *   hip_stream: a hipStream_t to order the work on, or NULL for the library's own
 * Returns after the scores are in host memory. */
int sw_db_search(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                 int32_t *scores, void *hip_stream);

/* Same, but scores_dev is DEVICE memory (n_seqs int32) on the database's device;
 * returns once the work is enqueued on hip_stream (NULL = library stream,
 * which is then synchronised before returning). */
int sw_db_search_dev(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                     int32_t *scores_dev, void *hip_stream);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the search of
 * sw_db_search_dev with no allocation of any kind.  Every intermediate buffer
 * (query profile, work lists, overflow list, counters, boundary columns, pass
 * buffers) lives in one fixed device array of SW_NOALLOC_SCRATCH_BYTES per GPU,
 * set up by sw_db_open and held until the process ends.
 *   query_dev:  qlen residue codes in DEVICE memory on the database's device.
 *               Codes are not checked (they are never read on the host): a code
 *               >= alphabet scores 0 against every residue.
 *   scores_dev: n_seqs int32 in DEVICE memory, caller's database order.
 *   hip_stream: the work is enqueued on it and the call returns at once; NULL =
 *               the library's stream, synchronised before returning.
 * Scores equal sw_db_search's.  Launch grids are sized to fit the scratch, so
 * long groups on a large database run at reduced occupancy; a query whose fixed
 * state (profile, work lists, 8 bytes per subject of overflow list) or whose
 * smallest launch does not fit fails with SW_EINVAL before any GPU work.
 * Every call on one GPU shares that GPU's array and leaves its contents there:
 * calls that overlap on one GPU (two databases, two streams, two threads) race
 * and must be ordered by the caller.  sw_db_last_stats reports the plan and cell
 * counts; times and the recompute count are -1 (nothing is read back). */
#define SW_NOALLOC_SCRATCH_BYTES (256LL << 20)
int sw_db_search_dev_noalloc(sw_db *db, const uint8_t *query_dev, int32_t qlen,
                             const sw_scoring *sc, int32_t *scores_dev, void *hip_stream);

/* The k best database sequences for one query (section III, stage iv: scores
 * sorted in descending order; equal scores by ascending database index).
 * top_scores[k], top_idx[k]; if k > n_seqs the tail is filled with -1. */
int sw_db_topk(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
               int32_t k, int32_t *top_scores, int64_t *top_idx, void *hip_stream);

/* Many queries in one fused launch over the database.  No passage of the
 * paper defines a batched call: SWAPHI searches one query at a time.  This is
 * the GPU form of its work distribution (section III.A: sequence profiles
 * handed to threads by a guided schedule), with the (query, subject group)
 * pairs of all queries in one persistent work queue.
 *   q_res / q_off: nq queries concatenated, q_off has nq + 1 entries
 *   top_scores / top_idx: nq * k (row per query), same order rules as sw_db_topk
 *   all_scores: NULL, or nq * n_seqs int32 (row per query, database order) */
int sw_db_search_batch(sw_db *db, int32_t nq, const uint8_t *q_res, const int64_t *q_off,
                       const sw_scoring *sc, int32_t k, int32_t *top_scores, int64_t *top_idx,
                       int32_t *all_scores, void *hip_stream);

/* ---- alignment with traceback ---- */

/* One optimal local alignment (see sw_db_align).  Positions are 0-based and
 * inclusive; all four are -1 when the score is 0 (empty alignment). */
typedef struct sw_alignment {
    int32_t score;
    int32_t q_begin, q_end;   /* query residues q_begin..q_end */
    int32_t n_ops;            /* runs of this alignment in `ops` */
    int64_t s_begin, s_end;   /* subject residues s_begin..s_end */
    int64_t ops_offset;       /* index of its first run in `ops` */
} sw_alignment;

#define SW_OP_PAIR   0   /* a query residue aligned with a subject residue */
#define SW_OP_QGAP   1   /* a query residue against a gap */
#define SW_OP_SGAP   2   /* a subject residue against a gap */

/* Optimal local alignments, with traceback, of one query against the listed
 * database sequences (alignment reconstruction is the future work the
 * conclusion names; scores are those of section II.A, Eq. 1, and equal
 * sw_db_search's).  Among equal-scoring alignments the result is fixed:
 *   - it ends at the first cell, subject position outer and query position
 *     inner, whose H equals the score;
 *   - walking back, H is taken from the diagonal before E (subject residue
 *     against a gap) before F (query residue against a gap), and E and F from
 *     the gap opening before the extension;
 *   - it starts at the first diagonal step whose predecessor H is 0.
 *   ids: n_ids database indices (repeats allowed); out: n_ids results, in order.
 *   ops: runs in forward order, each (length << 2) | SW_OP_*; every gap (one
 *        opening and its extensions) is its own run, aligned pairs in a row
 *        share one.  Alignment k's runs are ops[out[k].ops_offset ..
 *        + out[k].n_ops - 1], packed one after another.
 *   ops_cap: length of ops.  The library needs sum over ids of (len + qlen)
 *        (an upper bound); *ops_needed (if non-NULL) receives it, and a smaller
 *        ops_cap fails with SW_EINVAL.
 * Device memory: one byte per cell of the pairs aligned together (batches of
 * up to 1 GiB; a single subject needing more than 16 GiB fails with
 * SW_ENOMEM).  Synchronous on the database's own stream. */
int sw_db_align(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                const int64_t *ids, int32_t n_ids, sw_alignment *out, uint32_t *ops,
                int64_t ops_cap, int64_t *ops_needed);

/* Run the autotuner: for each query-length bucket of the given lengths, time
 * every candidate plan on a sample of this database's blocks, re-time the two
 * fastest on the whole database (best of two runs) and keep the faster.  With
 * more than one length, also time the distinct winners and the default plan on
 * a batch of up to 32 of the lengths (a sample of the blocks) and keep the
 * fastest as the plan of every launch of several queries (sw_db_search_batch;
 * bucket -1 in the cache).  If cache_path is non-NULL the table is read from /
 * written to that JSON file.
 * No passage of the paper defines it; it plays the part of the paper's
 * empirical choices of thread count and schedule (section III.A) and of the
 * score profile's depth (section III.B.3). */
int sw_db_autotune(sw_db *db, const sw_scoring *sc, const int32_t *qlens, int32_t n_qlens,
                   const char *cache_path);

/* ---- serving (continuous batching over a resident database) ----
 * No passage of the paper defines a server: SWAPHI is a batch program.  The
 * server keeps the database resident (the paper re-offloads it chunk by chunk
 * per run, section III, whose fixed costs it found to dominate small
 * workloads, section IV.C) and coalesces the requests in flight into shared
 * passes over database chunks. */

typedef struct sw_server_opts {
    int64_t memory_budget;   /* bytes of per-request device state the admitted requests may
                                hold together: each request is charged its query profile
                                ((alphabet + 1) x qlen rounded up to 32 bytes) and its top-k
                                (12 x k bytes).  A request that does not fit waits; smaller
                                later ones may pass it until it has waited 2 s.  The score
                                rows (max_active x n_seqs x 4 bytes) and the pass workspaces
                                are allocated once, at start, outside this budget.
                                0 = 1 GiB */
    int32_t max_active;      /* requests admitted at once (each pass serves the ones with the
                                least work left first; the oldest always advances).  Requests
                                whose alpha exceeds 28 run in an int16 sub-pass of each pass,
                                the others in the fp16 tier.  0 = 64 */
    int32_t queue_capacity;  /* waiting requests before submit returns SW_EBUSY; 0 = 65536 */
    int32_t chunk_groups;    /* database chunk (one scan position), in groups of 128 subjects;
                                0 = chosen by the server (1/16 of the lane-per-subject groups) */
    int32_t reserved[5];
} sw_server_opts;

typedef struct sw_req_stats {
    double queue_ms;   /* submit -> admitted into the database scan */
    double total_ms;   /* submit -> result ready */
    int64_t cells;     /* |Q| * sum |S| */
    int32_t passes;    /* server passes (launches) this request took part in */
    int32_t shared_passes;   /* of those, passes that also served another request */
} sw_req_stats;

/* Start a server over an open database.  The database must outlive the server
 * and must not be searched directly while the server runs. */
int sw_server_start(sw_db *db, const sw_server_opts *opts, sw_server **out);

/* Queue one query (copied).  *ticket identifies it for sw_server_wait. */
int sw_server_submit(sw_server *srv, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                     int32_t k, uint64_t *ticket);

/* Block until the request completes; writes k scores / indices as sw_db_topk.
 * stats may be NULL.  A ticket can be collected once. */
int sw_server_wait(sw_server *srv, uint64_t ticket, int32_t *top_scores, int64_t *top_idx,
                   sw_req_stats *stats);

/* Stop the server: requests not yet complete fail with SW_ESTOPPED; threads
 * blocked in sw_server_wait return before this call does.  No sw_server_* call
 * may use the handle afterwards.  NULL is ignored. */
void sw_server_stop(sw_server *srv);

/* ---- databases larger than device memory ----
 * Section III's workflow: the database is sorted and indexed offline, and the
 * search loads it chunk by chunk.  The index file holds the subjects sorted by
 * length and dealt round-robin over chunks of at most chunk_residues residues
 * (so that every chunk holds the whole length distribution), or, when the
 * longest subject exceeds a quarter of a chunk, cut into consecutive runs of
 * the length order; each chunk is stored in the packed device layout of
 * sw_db_open (its subjects in ascending database order).  A search keeps the whole index on the device when it fits the
 * memory budget; otherwise it streams the chunks through two device slots,
 * loading chunk c+1 (host thread, copies on the slot's own stream) while
 * chunk c is searched.  Results equal sw_db_search_batch on the same database
 * opened whole: the per-chunk top-k lists merge by (score desc, database index
 * asc). */
typedef struct sw_index sw_index;

typedef struct sw_index_opts {
    int32_t device;          /* HIP device ordinal; <= 0 means device 0 */
    int32_t reserved0;
    int64_t memory_budget;   /* device bytes the database copies may take (search workspaces
                                come on top); 0 = half of the device's free memory.  The index
                                stays resident when all chunks fit, else it is streamed, which
                                needs two of its largest chunk to fit (else SW_ENOMEM). */
    int32_t reserved[4];
} sw_index_opts;

typedef struct sw_index_stats {
    int64_t chunks;          /* chunks in the index */
    int32_t resident;        /* 1 if every chunk stays on the device */
    int32_t reserved0;
    int64_t bytes_loaded;    /* chunk bytes copied to the device by the last search */
    int64_t cells;           /* sum |Q| * sum |S| */
    double  load_ms;         /* host-thread time loading chunks (overlaps the searches) */
    double  search_ms;       /* wall time of the per-chunk searches */
    double  kernel_ms;       /* device time of their kernels */
    double  total_ms;        /* wall time of the whole call */
} sw_index_stats;

/* Write an index of the database (residues/offsets as in sw_db_open) to path.
 * chunk_residues >= 1: residues per chunk (a chunk holds at least one subject).
 * Needs no GPU: chunks are packed for 256 compute units (MI355X). */
int sw_index_write(const char *path, const uint8_t *residues, const int64_t *offsets,
                   int64_t n_seqs, int32_t alphabet, int64_t chunk_residues);

/* Map an index file and prepare its device slots (opts may be NULL). */
int sw_index_open(const char *path, const sw_index_opts *opts, sw_index **out);

/* Release an index (NULL is ignored). */
void sw_index_close(sw_index *ix);

/* Number of sequences in the index (-1 for NULL). */
int64_t sw_index_size(const sw_index *ix);

/* Statistics of the last search on this index. */
int sw_index_last_stats(sw_index *ix, sw_index_stats *out);

/* Many queries against the whole index; arguments and results as
 * sw_db_search_batch (host memory, database order), synchronous. */
int sw_index_search_batch(sw_index *ix, int32_t nq, const uint8_t *q_res, const int64_t *q_off,
                          const sw_scoring *sc, int32_t k, int32_t *top_scores, int64_t *top_idx,
                          int32_t *all_scores);

/* Message for the last failed call on this thread ("" if none). */
const char *sw_last_error(void);

/* Library version string. */
const char *sw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_H */
