/*
 * peanut.h — C ABI of the MI355X (gfx950) read-mapping hot path after
 * PEANUT (Koester & Rahmann, "Massively parallel read mapping on GPUs with
 * PEANUT", arXiv 1403.1706).
 *
 * The library maps a batch of DNA reads against a reference and both of its
 * strands.  It builds a q-group index over the reads on the device
 * (Section 2.2, Algorithm 1), streams every reference q-gram through it to
 * produce (read, diagonal) candidates (Section 3.2, Algorithm 2) and
 * verifies each candidate with a banded bit-parallel semiglobal edit
 * distance (Section 3.3).  It reports every hit with at most k errors, or
 * only the best stratum (Section 3.4), as (read_id, strand, end_pos, errors).
 *
 * The result is defined without reference to the filter.  For read x of
 * length n and text T (strand 0: the reference R; strand 1: its reverse
 * complement, T[i] = complement(R[L-1-i])), let E be the semiglobal edit
 * matrix with unit costs: E[0][j] = 0, E[i][0] = i,
 * E[i][j] = min(E[i-1][j-1] + [x[i-1] != T[j-1]], E[i-1][j] + 1, E[i][j-1] + 1)
 * (Section 3.3: E_ij is the smallest edit distance between the read prefix of
 * length i and any substring of the reference ending at j).  A hit is
 * (r, s, e = j-1, E[n][j]) with E[n][j] <= k_r.  In best-stratum mode only
 * hits whose error count equals the read's minimum over both strands are
 * kept.  The filter loses nothing when every read satisfies
 * (k_r + 1) * q <= n_r (q-gram lemma, Section 2.2); calls check this.
 *
 * Conventions
 *  - Every call returns a status (PN_OK = 0 or a negative PN_E* code).  On
 *    error, out-parameters are left untouched and nothing leaks.  The
 *    library never aborts and never prints.
 *  - Input host pointers are borrowed for the duration of the call.  Handles
 *    are owned by the caller and released with the matching _free/_destroy;
 *    passing NULL to those is a no-op.  Host hit arrays returned by the
 *    library are released with pn_hits_free.
 *  - Device ("_dev") variants take device pointers and a hipStream_t passed
 *    as void*; all device work of such a call is ordered on that stream.
 *    The caller keeps device inputs alive until the call returns.
 *  - A handle is not thread-safe; distinct contexts are.
 *  - Sequences are ASCII A, C, G, T in either case; anything else is
 *    PN_EALPHABET.  Base codes are A=0, C=1, G=2, T=3 (Section 2.2).
 *  - Limits: reference length L < 2^32 - 2^16; reads per index < 2^21;
 *    read length <= 256; 1 <= q <= 16 (q = 16 with a reference of at most
 *    2^31 - 1 letters: a position-set key holds the position beside the
 *    32-bit q-gram); w in {32, 64}; 0 <= k_r <= 31 (a band of 2 k_r + 1 <= 63
 *    diagonals around a candidate's diagonal, Section 3.3; bands of up to
 *    31 diagonals run in 32-bit words, wider ones in a 64-bit pass).
 */
#ifndef PEANUT_H
#define PEANUT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PN_OK 0
#define PN_EINVAL (-1)     /* bad argument or limit exceeded */
#define PN_EALPHABET (-2)  /* a letter other than A/C/G/T */
#define PN_ENOMEM (-3)     /* device or host allocation failed */
#define PN_EDEVICE (-4)    /* HIP runtime error or no device */
#define PN_ELEMMA (-5)     /* some read has (k_r + 1) * q > n_r */
#define PN_ETRUNC (-6)     /* output capacity too small; required count returned */
#define PN_EBUDGET (-7)    /* request does not fit the memory budget */

typedef struct pn_ctx pn_ctx;
typedef struct pn_ref pn_ref;
typedef struct pn_index pn_index;

typedef enum { PN_ALL_HITS = 0, PN_BEST_STRATUM = 1 } pn_mode;

/* One reported hit, 12 bytes.  read_id: 0-based position of the read in the
 * batch.  strand: 0 = reference, 1 = reverse complement.  end_pos: 0-based
 * last aligned text position in that strand's own coordinates (a strand-1
 * end e corresponds to forward position L-1-e, where the reverse-complemented
 * read starts).  errors: the exact edit distance E[n][end_pos+1]. */
typedef struct {
    uint32_t read_id;
    uint32_t end_pos;
    uint8_t strand;
    uint8_t errors;
    uint16_t reserved;
} pn_hit;

/* A filtration hit (Algorithm 2): read, strand and hit diagonal
 * d = p - o, the text position where the read would start if the q-gram at
 * read offset o matched text position p without indels. */
typedef struct {
    uint32_t read_id;
    uint8_t strand;
    uint8_t reserved[3];
    int64_t diagonal;
} pn_candidate;

/* Sizes of a built q-group index (Section 2.2): |I| = n_groups words of w
 * bits, S has n_groups + 1 entries, S' has n_distinct + 1 entries (D = the
 * number of distinct q-grams present), O has n_qgrams = |T| entries.
 * after_sorted: 1 when each slice of O is ordered by the letters after its
 * q-gram first (see pn_index_export). */
typedef struct {
    uint64_t n_reads;
    uint64_t n_bases;
    uint64_t n_qgrams;
    uint64_t n_distinct;
    uint64_t n_groups;
    int32_t q;
    int32_t w;
    int32_t max_len;
    int32_t after_sorted;
    int32_t s_sample; /* 1: S holds every group start; 2: every second (pn_index_sample_s) */
} pn_index_info;

/* Human-readable name of a status code; never NULL. */
const char *pn_strerror(int status);

/* ---- context ---------------------------------------------------------- */

/* Bind HIP device `device`, create the context's stream (default priority)
 * and its workspace pool.  PN_EDEVICE if the device does not exist. */
int pn_ctx_create(int device, pn_ctx **out);
void pn_ctx_destroy(pn_ctx *ctx);
/* The context's own hipStream_t (as void*), used by the host-pointer calls. */
int pn_ctx_stream(pn_ctx *ctx, void **stream);

/* Stage timing and work counters of a context.  While timing is enabled,
 * every stage of the path is bracketed by hipEvents on the stream it runs on
 * and its device time is accumulated (ms) with its kernel-launch count.
 * Counters accumulate always: occurrence pairs seen by filtration (n_seeds),
 * candidates verified, band rows computed by verification, records emitted,
 * hits reported, and index entries filtration actually read (n_visited:
 * the seed rules skip the rest); verify_rows_long is the second pass's share
 * of verify_rows.  pn_ctx_get_stats copies them out and optionally
 * resets them. */
enum {
    PN_STAGE_INGEST = 0,       /* ASCII -> 2-bit codes, read metadata, read planes */
    PN_STAGE_INDEX = 1,        /* Algorithm 1 */
    PN_STAGE_FILTER_HEAVY = 2, /* Algorithm 2: occurrence lists set aside as too long
                                  for one lane, a wave per slice of them */
    PN_STAGE_FILTER_EMIT = 3,  /* Algorithm 2: the scan of the reference (one kernel) */
    PN_STAGE_VERIFY = 4,       /* banded bit-parallel validation, first pass (one kernel) */
    PN_STAGE_SORT = 5,         /* radix sort of hit records */
    PN_STAGE_FINISH = 6,       /* duplicate removal, strata, output */
    PN_STAGE_RULES = 7,        /* per-read seed rules, low-complexity side lists */
    PN_STAGE_VERIFY_LONG = 8,  /* validation, second pass: the candidates still open
                                  after the first pass's rows (one kernel) */
    PN_STAGE_COUNT = 9,        /* indexes of reads from repeat families: the count filter
                                  (q-gram lemma on disjoint 4-letter pieces of the read)
                                  in place of the first pass (one kernel) */
    PN_STAGE_ALIGN = 10,       /* pn_align: start positions and alignments of hits */
    PN_N_STAGES = 11
};
typedef struct {
    double ms[PN_N_STAGES];
    uint64_t launches[PN_N_STAGES];
    uint64_t n_seeds;
    uint64_t n_candidates;
    uint64_t verify_rows;
    uint64_t n_records;
    uint64_t n_hits;
    uint64_t n_visited;
    uint64_t verify_rows_long;   /* the part of verify_rows computed by the second pass */
    uint64_t n_visited_heavy;    /* the part of n_visited read by FILTER_HEAVY */
    uint64_t n_heavy_items;      /* work items (32 bytes each) handed to FILTER_HEAVY */
    uint64_t n_candidates_heavy; /* the part of n_candidates written by FILTER_HEAVY */
    uint64_t count_letters;      /* read letters the count filter looked at */
} pn_stats;
int pn_ctx_set_timing(pn_ctx *ctx, int enable);
int pn_ctx_get_stats(pn_ctx *ctx, pn_stats *out, int reset);

/* ---- reference (resident in HBM) -------------------------------------- */

/* Pack an ASCII reference of `len` letters to two bits per base on the
 * device and derive both strands' verification bit planes (Section 3.2: the
 * reference and its reverse complement are scanned; strand 1's q-grams are
 * computed from strand 0's packed words, only its bit planes are stored).
 * `seq` is host memory (pn_ref_load) or device memory (pn_ref_load_dev). */
int pn_ref_load(pn_ctx *ctx, const char *seq, uint64_t len, pn_ref **out);
int pn_ref_load_dev(pn_ctx *ctx, const char *d_seq, uint64_t len, void *stream, pn_ref **out);
void pn_ref_free(pn_ref *ref);
uint64_t pn_ref_length(const pn_ref *ref);

/* Precompute the reference's position set for q-gram length q: every
 * position of both strands, sorted by its q-gram (Section 3.2, where the
 * paper takes P sorted from its precomputed reference index so that
 * neighbouring threads probe neighbouring parts of the q-group index),
 * with the letters around each q-gram.  Mapping with an index of this q
 * builds it on first use anyway; calling this moves that one-time cost out
 * of the first mapping.  It stays resident until pn_ref_free: 10 bytes per
 * position and strand (2 GB for 100 Mbp) for each q used.  Safe to call
 * from several threads. */
int pn_ref_prepare(pn_ref *ref, int q);

/* Repeat masking (Section 3.2: exceedingly frequent q-grams are left out of
 * the position set; the paper does not fix "frequent"): after this call,
 * filtration with q-gram length q skips every position whose q-gram occurs
 * more than max_occ times on the two strands together (so a q-gram and its
 * reverse complement are masked together); max_occ = 0 turns masking off
 * again.  Mapping a masked reference is no longer lossless: the hits are
 * those of the remaining candidates' bands (the per-read seed rules that
 * rely on every position being present are switched off), a subset of the
 * unmasked hits whose error counts may be larger.  The mask (4^q bits) is
 * owned by the reference.  Not to be called while a mapping with this
 * reference and q runs.  PN_EINVAL for q outside 1..16. */
int pn_ref_mask(pn_ref *ref, int q, uint32_t max_occ);

/* ---- q-group index over a read batch (Algorithm 1) --------------------- */

/* Build the q-group index (I, S, S', O) of all q-grams of the reads
 * (Section 2.2 and Algorithm 1: presence bitmap I, S = exclusive prefix sum
 * of popcount(I[i]), S' = exclusive prefix sum of per-q-gram counts, O =
 * occurrence positions in q-gram order).  Read r is
 * reads[offsets[r] .. offsets[r+1]); a read shorter than q contributes no
 * q-gram.  The index keeps its own copy of everything it needs.
 * The _dev variant takes device `d_reads`/`d_offsets` (offsets u64[n+1],
 * n_bases = offsets[n]) and orders its work on `stream`; it synchronises
 * once to validate the batch. */
int pn_index_build(pn_ctx *ctx, const char *reads, const uint64_t *offsets, uint32_t n_reads,
                   int q, int w, pn_index **out);
int pn_index_build_dev(pn_ctx *ctx, const char *d_reads, const uint64_t *d_offsets,
                       uint32_t n_reads, uint64_t n_bases, int q, int w, void *stream,
                       pn_index **out);
void pn_index_free(pn_index *idx);
int pn_index_get_info(const pn_index *idx, pn_index_info *out);

/* Sampling S (Section 2.2): keep only the even entries S[0], S[2], ..., S[2 t]
 * (t = n_groups / 2) and free the full array, halving S's memory; a lookup
 * in an odd group adds the population count of the group before it.  The
 * hits of every later mapping are unchanged.  Idempotent.  pn_index_export
 * then writes n_groups / 2 + 1 words of S. */
int pn_index_sample_s(pn_index *idx);

/* Copy the index arrays to host buffers sized from pn_index_get_info:
 * I: n_groups words of w bits (uint32 for w = 32, uint64 for w = 64);
 * S: n_groups + 1 uint32 (sampled: n_groups / 2 + 1); S': n_distinct + 1
 * uint32; O: n_qgrams uint64.
 * An O entry holds one occurrence (read r, offset o) of its q-gram: the high
 * 32 bits are (cls << 29) | (r << 8) | o, where cls is the code of the
 * letter before the q-gram in its read (4 when o == 0); the low 32 bits are
 * (next4 << 24) | (nav << 21): the nav = min(4, n_r - o - q) letters after
 * the q-gram, first letter in the top bits (unused letters 0).  Inside each
 * q-gram's slice of O, entries are in the order (r, o).  For q <= 12, when
 * at least 1/128 of all occurrences fall into slices of more than 32 (reads
 * from repeat families), the slices are first ordered by the letters after
 * the q-gram (the code next4 when nav = 4, else 256 + the three letters,
 * 320 + two, 336 + one, 340 for none; pn_index_info.after_sorted = 1), so
 * that filtration can find the entries whose next letters agree with the
 * text by binary search; bit 20 marks a piece start (offset a multiple of
 * q + 4 with four letters after the q-gram).  Each mapping call writes its
 * per-read seed-rule byte into bits 0-7 and the read's length - 1 into bits
 * 8-15 (both 0 in a freshly built index).  Any pointer may be NULL to skip
 * that array. */
int pn_index_export(const pn_index *idx, void *I, uint32_t *S, uint32_t *S_prime, uint64_t *O);

/* ---- mapping ----------------------------------------------------------- */

/* Map the indexed reads against both strands of `ref`.  k >= 0 applies to
 * every read; k < 0 takes k_per_read[r] (host array for pn_map, device
 * array for pn_map_dev).  Hits are sorted by (read_id, strand, end_pos).
 * PN_ELEMMA if some read has (k_r + 1) * q > n_r; PN_EINVAL if k_r > 31.
 * pn_map returns a library-allocated host array (free with pn_hits_free).
 * pn_map_dev writes at most `capacity` hits to device `d_hits`, stores the
 * total in *n_hits (host) and returns PN_ETRUNC if it exceeded capacity. */
int pn_map(pn_ctx *ctx, const pn_ref *ref, const pn_index *idx, int k,
           const uint8_t *k_per_read, pn_mode mode, pn_hit **hits, uint64_t *n_hits);
int pn_map_dev(pn_ctx *ctx, const pn_ref *ref, const pn_index *idx, int k,
               const uint8_t *d_k_per_read, pn_mode mode, pn_hit *d_hits, uint64_t capacity,
               uint64_t *n_hits, void *stream);
void pn_hits_free(pn_hit *hits);

/* ---- the two steps on their own (for inspection) ----------------------- */

/* Filtration only (Algorithm 2, both strands), with the error budget the
 * mapping would use (k >= 0 for all reads, or k < 0 and host k_per_read).
 * Returns the candidates pn_map verifies, each (read, strand, diagonal
 * d = p - o) for an occurrence pair (reference position p, read offset o)
 * of a q-gram, sorted by (read, strand, diagonal), duplicates kept.  Pairs
 * are left out only when the mapping provably does not need them, so the
 * hit list is unchanged (Section 2.2, q-gram lemma): a pair whose left
 * neighbours agree (the pair one step up-left is on the same diagonal), the
 * low-complexity q-grams (period <= 2) of a read with more than k_r q other
 * q-grams, and a pair whose exact run along its diagonal is shorter than the
 * run every alignment with <= k_r errors must contain.  *n_seeds (if not
 * NULL) receives the number of all occurrence pairs (sum over positions of
 * k_end - k_start).  PN_ELEMMA / PN_EINVAL as for pn_map.  Free with
 * pn_hits_free. */
int pn_filter(pn_ctx *ctx, const pn_ref *ref, const pn_index *idx, int k,
              const uint8_t *k_per_read, pn_candidate **cands, uint64_t *n_cands,
              uint64_t *n_seeds);

/* Validation only (Section 3.3): banded bit-parallel edit distance over
 * diagonals [d - k_r, d + k_r] for each given candidate; returns every
 * (read, strand, end, value) with value <= k_r, one record per candidate
 * and end (duplicates across candidates kept), sorted.  Free with
 * pn_hits_free. */
int pn_validate(pn_ctx *ctx, const pn_ref *ref, const pn_index *idx, const pn_candidate *cands,
                uint64_t n_cands, int k, const uint8_t *k_per_read, pn_hit **records,
                uint64_t *n_records);

/* Start position and alignment of hits (Section 3.3 runs the verification
 * backwards from a hit's end to find its start; Section 3.4 makes the
 * alignment in postprocessing).  hits: n_hits records as pn_map returns
 * them, against `ref` and the reads of `idx` (read_id < n_reads, strand 0
 * or 1, end_pos < L, errors <= 31: the hit's exact error count).  For
 * each hit h, in host arrays of n_hits entries:
 *   starts[h]  first aligned text position, in the strand's own
 *              coordinates (the hit covers [start, end_pos]); of all
 *              starts whose alignment has the hit's error count, the
 *              latest one (the shortest text span);
 *   errors[h]  the alignment's edit distance, equal to the hit's; 255 when
 *              no alignment with the given error count ends at end_pos
 *              (start 0, no ops);
 *   ops        (may be NULL) row h of ops_stride bytes: the operations from
 *              the read's first letter on, 0 '=' match, 1 'X' substitution,
 *              2 'I' read letter not in the text, 3 'D' text letter not in
 *              the read; among equally good alignments the one that, walking
 *              back from the read's first letter, takes a diagonal step
 *              first, then 'I', then 'D'.  At most n + errors operations;
 *              a longer row is cut at ops_stride;
 *   n_ops[h]   (may be NULL: then ops is not written) the number of
 *              operations.
 * The caller owns every array.  PN_EINVAL for a record outside those
 * bounds or a NULL starts / errors with n_hits > 0; PN_ENOMEM when the
 * device work space cannot be had. */
int pn_align(pn_ctx *ctx, const pn_ref *ref, const pn_index *idx, const pn_hit *hits,
             uint64_t n_hits, uint32_t *starts, uint8_t *errors, uint8_t *ops,
             uint32_t ops_stride, uint16_t *n_ops);

/* pn_validate for callers that cannot allocate device memory: tight serving
 * loops and harnesses that forbid hipMalloc.  (It reads counts back and
 * synchronises, so it cannot itself be recorded into a HIP graph.)
 * Same candidates, k and records as pn_validate, but device arrays in and
 * out, ordered on `stream` (NULL: the context's stream): d_cands holds
 * n_cands pn_candidate entries, d_k_per_read (k < 0) one byte per read of
 * idx, and the records, sorted, go to d_records (room for `capacity`);
 * *n_records (host) receives their count.  The call synchronises the stream
 * and allocates nothing: its working memory is one fixed 37 MiB device array
 * per device, set up by pn_ctx_create and held until the process ends.
 * Limits: n_cands <= 65536 and at most 2^20 records (and 32768 in each of
 * the 64 output regions that blocks of 256 candidates append to in turn);
 * beyond them PN_EINVAL.  PN_ETRUNC with *n_records = the required count
 * when capacity is too small.  PN_EINVAL for a candidate with read_id >=
 * n_reads, strand > 1 or a diagonal outside [-256, L]; PN_EINVAL /
 * PN_ELEMMA for k as pn_map.  Every call on one device shares its array and
 * leaves its contents behind: calls that overlap on one device (on two
 * streams or threads) race and must be serialised by the caller. */
int pn_validate_noalloc(pn_ctx *ctx, const pn_ref *ref, const pn_index *idx,
                        const pn_candidate *d_cands, uint64_t n_cands, int k,
                        const uint8_t *d_k_per_read, pn_hit *d_records, uint64_t capacity,
                        uint64_t *n_records, void *stream);

/* ---- batching: parameter choice ----------------------------------------- */

/* Pick q in {10, 11, 12} and group width w in {32, 64} for a read batch
 * (device arrays as for pn_index_build_dev; k >= 0 for all reads, or
 * k < 0 and device k_per_read).  q must satisfy the q-gram lemma
 * (k_r + 1) q <= n_r for every read of the batch (Section 2.2); each such
 * (q, w) is timed (index build + pn_map_dev, best of two runs after a
 * warm-up) on the batch's first sample_reads reads and on half as many; the
 * line through the two times is evaluated at the whole batch (a fixed part,
 * the reference scan, plus a part per read) and the fastest prediction is
 * returned in *best_q, *best_w.  results[] (room for 6) receives every
 * candidate with its predicted time (ms) or status (PN_ELEMMA when the
 * lemma excludes it); *n_results their count.  The hits do not depend on the choice: the
 * filter is lossless for every admitted q.  PN_ELEMMA if no q is
 * admitted. */
typedef struct {
    int q, w;
    double ms;
    int status;
} pn_tune_result;
int pn_autotune(pn_ctx *ctx, const pn_ref *ref, const char *d_reads, const uint64_t *d_offsets,
                uint32_t n_reads, uint64_t n_bases, int k, const uint8_t *d_k_per_read,
                pn_mode mode, uint32_t sample_reads, pn_tune_result *results, int *n_results,
                int *best_q, int *best_w);

/* Map a read set of any size (host memory, reads of mixed lengths with
 * per-read k_per_read[r]) against both strands of `ref`.  The reads are
 * taken in input order in sub-batches that each fit one q-group index
 * (at most 2^21 reads, and about 48 bytes per base of the device memory
 * free at the call, halved): the paper buffers reads and indexes each
 * buffer on the device (Section 3.1).  Each sub-batch is copied to the
 * device, indexed (Algorithm 1) and mapped as pn_map does; its hits come
 * back and are appended with read ids relative to the whole set, so the
 * result is sorted by (read_id, strand, end_pos) and equals pn_map's on one
 * index of all the reads (per read, the hits do not depend on the batch).
 * q and w: with tune_cache == NULL, w = 64 and the largest q <= 12 that the
 * q-gram lemma admits for every read ((k_r + 1) q <= n_r, Section 2.2).
 * Otherwise tune_cache names a text file of lines "<key> <q> <w>", the key
 * describing the reference length, read count (power of two), length and
 * k ranges and mode: a line for this key is used; without one, pn_autotune
 * picks (q, w) on a sample of the first sub-batch and a line is appended
 * (a cache that cannot be written is not an error).  PN_EINVAL for a read
 * shorter than 1 or longer than 256, k_r > 31 or decreasing offsets;
 * PN_ELEMMA if no q >= 1 satisfies the lemma; the hit array is freed with
 * pn_hits_free. */
int pn_map_batched(pn_ctx *ctx, const pn_ref *ref, const char *reads, const uint64_t *offsets,
                   uint32_t n_reads, const uint8_t *k_per_read, pn_mode mode,
                   const char *tune_cache, pn_hit **hits, uint64_t *n_hits);

/* ---- serving: continuous batching over a resident reference ------------ */

/* A request loop around the mapping path (the paper's layered pipeline of
 * Fig. 2 with queues between the stages, and its buffering of reads into
 * batches for one index, Section 3.1).  Submitted requests wait in a FIFO
 * queue; each of `slots` workers, with its own context and HIP stream on
 * the reference's device, takes as many queued requests as fit one batch
 * (at most max_batch_reads reads, and the batch's estimated working set
 * within what is left of hbm_budget), builds one q-group index over their
 * concatenated reads, maps them against both strands of the resident
 * reference, and hands each request its own hits.  Requests that arrive
 * while batches run are admitted when a slot and budget free up; the slots'
 * work overlaps on the device.  A request's hits do not depend on what it
 * was batched with: per read they are exactly pn_map's (read ids relative
 * to the request, sorted by (read_id, strand, end_pos)).
 *
 * Working-set estimate of a batch (bytes): 12 per base + 4096 per read +
 * 16 MiB.  A request whose own estimate exceeds hbm_budget, or with more
 * than 2^21 reads (one index), is refused with PN_EBUDGET at submit.  A
 * batch always takes at least one request, however many reads it has, so
 * serial one-request-at-a-time mapping is slots = 1, max_batch_reads = 1. */
typedef struct pn_server pn_server;
typedef struct {
    int q;                    /* q-gram length of every batch index, 1..16 */
    int w;                    /* group width, 32 or 64 */
    uint64_t hbm_budget;      /* bytes of estimated working sets in flight */
    uint32_t max_batch_reads; /* reads merged into one batch, 1..2^21 */
    int slots;                /* batches in flight, 1..8 */
} pn_server_config;
typedef struct {
    uint64_t requests;        /* completed */
    uint64_t batches;         /* run */
    uint64_t reads;           /* mapped */
    uint64_t hits;            /* delivered */
    uint64_t max_batch_reads; /* largest batch run */
} pn_server_stats;
/* The server runs on the device of `ctx` (which must be the reference's);
 * each slot makes its own context there.  `ctx` and `ref` stay owned by
 * the caller and must outlive the server. */
int pn_server_create(pn_ctx *ctx, const pn_ref *ref, const pn_server_config *cfg,
                     pn_server **out);
/* Queue a request: reads[offsets[i] .. offsets[i+1]) for i < n_reads
 * (host memory, copied before return), error budget k >= 0 for all reads
 * or k < 0 and k_per_read[i] (host).  Checked here: letters ACGT (either
 * case), 1 <= n_r <= 256, k_r <= 31, (k_r + 1) q <= n_r; PN_EALPHABET /
 * PN_EINVAL / PN_ELEMMA / PN_EBUDGET.  *ticket identifies the request. */
int pn_server_submit(pn_server *srv, const char *reads, const uint64_t *offsets, uint32_t n_reads,
                     int k, const uint8_t *k_per_read, pn_mode mode, uint64_t *ticket);
/* Block until the request is done; returns its status.  On PN_OK, *hits
 * (free with pn_hits_free) and *n_hits receive its hits; *latency_ms (if
 * not NULL) the time from submit to completion.  A ticket is redeemed
 * once. */
int pn_server_wait(pn_server *srv, uint64_t ticket, pn_hit **hits, uint64_t *n_hits,
                   double *latency_ms);
/* Non-blocking pn_server_wait: PN_PENDING (1) while the request is queued
 * or running (nothing is written); otherwise exactly what pn_server_wait
 * returns, and the ticket is redeemed. */
#define PN_PENDING 1
int pn_poll(pn_server *srv, uint64_t ticket, pn_hit **hits, uint64_t *n_hits,
            double *latency_ms);
int pn_server_get_stats(pn_server *srv, pn_server_stats *out);
/* Finishes every queued request, then stops the workers. */
void pn_server_destroy(pn_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* PEANUT_H */
