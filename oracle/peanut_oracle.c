/*
 * Plain CPU oracle for PEANUT read mapping (Koester & Rahmann, "Massively
 * parallel read mapping on GPUs with PEANUT", arXiv 1403.1706).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation, and the HIP
 * implementation never calls it.
 *
 * Input convention: sequences arrive as base codes 0..3 (A=0, C=1, G=2, T=3,
 * Section 2.2, "The q-group index", the two-bit encoding of letters); the
 * Python wrapper converts ASCII to codes.  The reverse-complement strand is
 * T1[i] = 3 - R[L-1-i] (complement of the code is 3 - code for this encoding).
 *
 * What is computed (all integer arithmetic):
 *
 *  - orc_qgram_index: the conventional q-gram index of the concatenated
 *    reads: address table A (4^q + 1 entries) and position table P, so that
 *    P[A[g]] .. P[A[g+1]-1] are the occurrences of q-gram g (Section 2.2,
 *    "The q-group index", first paragraphs).  A position is the pair
 *    (read r, offset o) with 0 <= o <= n_r - q; buckets list positions in
 *    ascending (r, o).  The q-gram code puts the first base in the most
 *    significant two bits: g = sum_t c(x_t) * 4^(q-1-t).
 *
 *  - orc_candidates: filtration (Section 3.2, Algorithm 2) done with the
 *    conventional index: for both strands s and every reference position p
 *    in [0, L-q], look up the bucket of the q-gram at p and emit, for every
 *    occurrence (r, o), the hit diagonal d = p - o (the putative read start).
 *    With repeat masking (max_occ > 0; Section 3.2 leaves exceedingly
 *    frequent q-grams out of P, without fixing "frequent"), positions whose
 *    q-gram occurs more than max_occ times on the two strands together
 *    emit nothing.
 *
 *  - orc_banded: validation of one candidate (Section 3.3): the semiglobal
 *    edit-distance matrix E (unit costs) restricted to the diagonal band
 *    [d-k, d+k], computed cell by cell.  E[0][j] = 0 inside the band (free
 *    start), E[i][0] = i, cells outside the band or outside columns [0, L]
 *    do not exist.  Reports (e = j-1, E[n][j]) for every end column j of the
 *    last row with E[n][j] <= k.
 *
 *  - orc_map_filtered: the method's steps in order: index over the reads,
 *    filtration of both strands, removal of duplicate candidates (the same
 *    read, strand and diagonal found through several q-grams, Section 3.4),
 *    validation, removal of duplicate hits (same read, strand and end; the
 *    smallest error count is kept), and for best-stratum mode the hits whose
 *    error count equals the read's minimum (Section 3.4, strata).
 *
 *  - orc_map_sellers: the plain definition of the result, with no filter:
 *    the full semiglobal matrix E of every read against every column of both
 *    strands (Section 3.3 defines E_ij as the smallest edit distance between
 *    the read prefix of length i and any reference substring ending at j),
 *    reporting every (r, s, e = j-1, E[n][j]) with E[n][j] <= k_r.
 *
 *  - orc_align: the start and the alignment of one hit (Section 3.3 runs
 *    the verification backwards from a hit's end to find where it starts;
 *    the actual alignment is made in postprocessing, Section 3.4).  For a
 *    read x of length n ending at text position e, the read reversed is
 *    aligned to the text read backwards from e with the same unit costs:
 *    F[i][j] = edit distance of the last i read letters and the j text
 *    letters ending at e (F[0][j] = j, F[i][0] = i, no free start).  The
 *    hit's error count is the least F[n][j]; the start is e + 1 - j for the
 *    smallest such j (the latest start, the shortest text span).  The
 *    alignment is read off from (n, j) back to (0, 0), which walks the read
 *    from its first letter on; of the predecessors whose value explains the
 *    cell, the diagonal one (a match '=' or a substitution 'X') is taken
 *    first, then the one above (a read letter not in the text, 'I'), then
 *    the one to the left (a text letter not in the read, 'D').  That rule
 *    makes the alignment unique.
 *
 * Hit records are 12-byte structs (read_id u32, end_pos u32, strand u8,
 * errors u8, 2 padding bytes), sorted by (read_id, strand, end_pos).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_INF 0x3fffffff
#define ORC_DBIAS 65536LL

typedef struct {
    uint32_t read_id;
    uint32_t end_pos;
    uint8_t strand;
    uint8_t errors;
    uint16_t pad;
} orc_hit;

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */

static int orc_threads(int want) {
    if (want > 0) return want;
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

typedef struct {
    uint64_t *v;
    size_t n, cap;
} u64vec;

static int vec_push(u64vec *a, uint64_t x) {
    if (a->n == a->cap) {
        size_t nc = a->cap ? a->cap * 2 : 1024;
        uint64_t *nv = (uint64_t *)realloc(a->v, nc * sizeof(uint64_t));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* code of the q-gram starting at s[0], first base most significant,
 * computed directly from its q letters */
static uint64_t qgram_code(const uint8_t *s, int q) {
    uint64_t g = 0;
    for (int t = 0; t < q; t++) g = g * 4 + s[t];
    return g;
}

static uint8_t *reverse_complement(const uint8_t *ref, uint64_t L) {
    uint8_t *rc = (uint8_t *)malloc(L ? L : 1);
    if (!rc) return NULL;
    for (uint64_t i = 0; i < L; i++) rc[i] = (uint8_t)(3 - ref[L - 1 - i]);
    return rc;
}

/* generic parallel-for over [0, n) in contiguous slices */
typedef void (*range_fn)(void *arg, int tid, uint64_t lo, uint64_t hi);
typedef struct {
    range_fn fn;
    void *arg;
    int tid;
    uint64_t lo, hi;
} range_job;

static void *range_thread(void *p) {
    range_job *j = (range_job *)p;
    j->fn(j->arg, j->tid, j->lo, j->hi);
    return NULL;
}

static void parallel_for(int nthreads, uint64_t n, range_fn fn, void *arg) {
    if (nthreads <= 1 || n < 2) {
        fn(arg, 0, 0, n);
        return;
    }
    if ((uint64_t)nthreads > n) nthreads = (int)n;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    range_job *jobs = (range_job *)malloc(sizeof(range_job) * nthreads);
    for (int t = 0; t < nthreads; t++) {
        jobs[t].fn = fn;
        jobs[t].arg = arg;
        jobs[t].tid = t;
        jobs[t].lo = n * (uint64_t)t / (uint64_t)nthreads;
        jobs[t].hi = n * (uint64_t)(t + 1) / (uint64_t)nthreads;
        pthread_create(&th[t], NULL, range_thread, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
}

/* ------------------------------------------------------------------------ */
/* conventional q-gram index over the reads                                  */

/* Number of indexed positions |T| = sum_r max(0, n_r - q + 1). */
uint64_t orc_qgram_count(const uint64_t *offsets, uint32_t n_reads, int q) {
    uint64_t t = 0;
    for (uint32_t r = 0; r < n_reads; r++) {
        uint64_t n = offsets[r + 1] - offsets[r];
        if (n >= (uint64_t)q) t += n - (uint64_t)q + 1;
    }
    return t;
}

/* A has 4^q + 1 entries; P_read / P_off have orc_qgram_count() entries. */
int orc_qgram_index(const uint8_t *codes, const uint64_t *offsets, uint32_t n_reads, int q,
                    uint64_t *A, uint32_t *P_read, uint32_t *P_off) {
    if (q < 1 || q > 15) return -1;
    const uint64_t G = 1ULL << (2 * q);
    memset(A, 0, sizeof(uint64_t) * (G + 1));
    /* counts of each q-gram, stored one slot to the right */
    for (uint32_t r = 0; r < n_reads; r++) {
        uint64_t n = offsets[r + 1] - offsets[r];
        const uint8_t *x = codes + offsets[r];
        for (uint64_t o = 0; o + (uint64_t)q <= n; o++) A[qgram_code(x + o, q) + 1]++;
    }
    /* running sum: A[g] = number of positions of q-grams smaller than g */
    for (uint64_t g = 0; g < G; g++) A[g + 1] += A[g];
    uint64_t *next = (uint64_t *)malloc(sizeof(uint64_t) * G);
    if (!next) return -2;
    memcpy(next, A, sizeof(uint64_t) * G);
    for (uint32_t r = 0; r < n_reads; r++) {
        uint64_t n = offsets[r + 1] - offsets[r];
        const uint8_t *x = codes + offsets[r];
        for (uint64_t o = 0; o + (uint64_t)q <= n; o++) {
            uint64_t k = next[qgram_code(x + o, q)]++;
            P_read[k] = r;
            P_off[k] = (uint32_t)o;
        }
    }
    free(next);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* filtration with the conventional index                                    */

typedef struct {
    const uint8_t *text[2];
    uint64_t L;
    int q;
    const uint64_t *A;
    const uint32_t *P_read, *P_off;
    const uint64_t *masked; /* ascending q-gram codes left out of P */
    uint64_t n_masked;
    u64vec *out; /* one per thread */
    int failed;
} cand_job;

static int is_masked(const cand_job *j, uint64_t g) {
    uint64_t lo = 0, hi = j->n_masked;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (j->masked[mid] < g)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < j->n_masked && j->masked[lo] == g;
}

/* Repeat masking (Section 3.2 leaves exceedingly frequent q-grams out of
 * P): the q-grams occurring more than max_occ times among the positions of
 * both strands, ascending.  The counts come from sorting the codes of all
 * 2 (L - q + 1) positions and measuring each run of equal codes. */
static int masked_qgrams(const uint8_t *ref, const uint8_t *rc, uint64_t L, int q,
                         uint32_t max_occ, uint64_t **out, uint64_t *n_out) {
    *out = NULL;
    *n_out = 0;
    if (L < (uint64_t)q) return 0;
    const uint64_t npos = L - (uint64_t)q + 1;
    uint64_t *codes = (uint64_t *)malloc(sizeof(uint64_t) * 2 * npos);
    if (!codes) return -2;
    for (uint64_t p = 0; p < npos; p++) {
        codes[p] = qgram_code(ref + p, q);
        codes[npos + p] = qgram_code(rc + p, q);
    }
    qsort(codes, 2 * npos, sizeof(uint64_t), cmp_u64);
    uint64_t m = 0;
    for (uint64_t a = 0; a < 2 * npos;) {
        uint64_t b = a;
        while (b < 2 * npos && codes[b] == codes[a]) b++;
        if (b - a > (uint64_t)max_occ) codes[m++] = codes[a];
        a = b;
    }
    *out = codes;
    *n_out = m;
    return 0;
}

/* candidate key: read (31 bits) | strand (1 bit) | diagonal + bias (32 bits) */
static uint64_t cand_key(uint32_t r, int s, int64_t d) {
    return ((uint64_t)r << 33) | ((uint64_t)s << 32) | (uint64_t)(uint32_t)(d + ORC_DBIAS);
}

static void cand_range(void *arg, int tid, uint64_t lo, uint64_t hi) {
    cand_job *j = (cand_job *)arg;
    u64vec *out = &j->out[tid];
    /* the range covers 2 * (L - q + 1) (strand, position) pairs */
    const uint64_t npos = j->L - (uint64_t)j->q + 1;
    for (uint64_t x = lo; x < hi; x++) {
        int s = (int)(x / npos);
        uint64_t p = x % npos;
        uint64_t g = qgram_code(j->text[s] + p, j->q);
        if (j->n_masked && is_masked(j, g)) continue;
        for (uint64_t k = j->A[g]; k < j->A[g + 1]; k++) {
            int64_t d = (int64_t)p - (int64_t)j->P_off[k];
            if (vec_push(out, cand_key(j->P_read[k], s, d))) {
                j->failed = 1;
                return;
            }
        }
    }
}

/* max_occ > 0: positions whose q-gram occurs more than max_occ times on
 * the two strands together emit nothing (repeat masking) */
static int collect_candidates(const uint8_t *ref, const uint8_t *rc, uint64_t L, int q,
                              const uint64_t *A, const uint32_t *P_read, const uint32_t *P_off,
                              uint32_t max_occ, int nthreads, uint64_t **keys, uint64_t *n_keys) {
    *keys = NULL;
    *n_keys = 0;
    if (L < (uint64_t)q) return 0;
    nthreads = orc_threads(nthreads);
    cand_job j;
    j.masked = NULL;
    j.n_masked = 0;
    if (max_occ > 0) {
        uint64_t *mk = NULL;
        if (masked_qgrams(ref, rc, L, q, max_occ, &mk, &j.n_masked)) return -2;
        j.masked = mk;
    }
    j.text[0] = ref;
    j.text[1] = rc;
    j.L = L;
    j.q = q;
    j.A = A;
    j.P_read = P_read;
    j.P_off = P_off;
    j.failed = 0;
    j.out = (u64vec *)calloc((size_t)nthreads, sizeof(u64vec));
    if (!j.out) {
        free((void *)j.masked);
        return -2;
    }
    parallel_for(nthreads, 2 * (L - (uint64_t)q + 1), cand_range, &j);
    free((void *)j.masked);
    size_t total = 0;
    for (int t = 0; t < nthreads; t++) total += j.out[t].n;
    uint64_t *all = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
    int rc_ = (all && !j.failed) ? 0 : -2;
    size_t at = 0;
    for (int t = 0; t < nthreads; t++) {
        if (all && j.out[t].n) memcpy(all + at, j.out[t].v, sizeof(uint64_t) * j.out[t].n);
        at += j.out[t].n;
        free(j.out[t].v);
    }
    free(j.out);
    if (rc_) {
        free(all);
        return rc_;
    }
    *keys = all;
    *n_keys = total;
    return 0;
}

/* Every (read, strand, diagonal) pair emitted by filtration, one entry per
 * q-gram occurrence pair (so duplicates are kept).  Output arrays are
 * malloc'ed; free with orc_free. */
int orc_candidates(const uint8_t *ref, uint64_t L, const uint8_t *codes, const uint64_t *offsets,
                   uint32_t n_reads, int q, uint32_t mask_max_occ, int nthreads,
                   uint32_t **out_read, uint8_t **out_strand, int64_t **out_diag,
                   uint64_t *n_out) {
    const uint64_t G = 1ULL << (2 * q);
    uint64_t T = orc_qgram_count(offsets, n_reads, q);
    uint64_t *A = (uint64_t *)malloc(sizeof(uint64_t) * (G + 1));
    uint32_t *Pr = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
    uint32_t *Po = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
    uint8_t *rc = reverse_complement(ref, L);
    int st = (A && Pr && Po && rc) ? orc_qgram_index(codes, offsets, n_reads, q, A, Pr, Po) : -2;
    uint64_t *keys = NULL, n = 0;
    if (!st) st = collect_candidates(ref, rc, L, q, A, Pr, Po, mask_max_occ, nthreads, &keys, &n);
    free(A);
    free(Pr);
    free(Po);
    free(rc);
    if (st) return st;
    qsort(keys, n, sizeof(uint64_t), cmp_u64);
    *out_read = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    *out_strand = (uint8_t *)malloc(n ? n : 1);
    *out_diag = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    for (uint64_t i = 0; i < n; i++) {
        (*out_read)[i] = (uint32_t)(keys[i] >> 33);
        (*out_strand)[i] = (uint8_t)((keys[i] >> 32) & 1);
        (*out_diag)[i] = (int64_t)(uint32_t)keys[i] - ORC_DBIAS;
    }
    free(keys);
    *n_out = n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* validation: banded semiglobal DP, cell by cell                            */

/* Writes up to 2k+1 (end, errors) pairs; returns how many.  k <= 31. */
int orc_banded(const uint8_t *text, uint64_t L, const uint8_t *x, uint32_t n, int64_t d, int k,
               int32_t *out_end, int32_t *out_err) {
    if (k < 0 || k > 31) return -1;
    const int W = 2 * k + 1;
    const int64_t lo = d - k; /* leftmost diagonal of the band */
    int prev[64], cur[64];
    /* row 0: free start on every existing column of the band */
    for (int b = 0; b < W; b++) {
        int64_t c = lo + b;
        prev[b] = (c >= 0 && c <= (int64_t)L) ? 0 : ORC_INF;
    }
    for (uint32_t i = 1; i <= n; i++) {
        int rowmin = ORC_INF;
        for (int b = 0; b < W; b++) {
            int64_t c = (int64_t)i + lo + b; /* column of band cell b in row i */
            int v = ORC_INF;
            if (c < 0 || c > (int64_t)L) {
                v = ORC_INF;
            } else if (c == 0) {
                v = (int)i; /* E[i][0] = i */
            } else {
                /* diagonal predecessor (i-1, c-1) is band cell b of row i-1 */
                if (prev[b] < ORC_INF) v = prev[b] + (x[i - 1] != text[c - 1]);
                /* predecessor above (i-1, c) is band cell b+1 of row i-1 */
                if (b + 1 < W && prev[b + 1] < ORC_INF && prev[b + 1] + 1 < v) v = prev[b + 1] + 1;
                /* predecessor on the left (i, c-1) is band cell b-1 of row i */
                if (b > 0 && cur[b - 1] < ORC_INF && cur[b - 1] + 1 < v) v = cur[b - 1] + 1;
            }
            cur[b] = v;
            if (v < rowmin) rowmin = v;
        }
        /* costs never decrease along a path, and a path into the last row
         * either crosses row i or starts at a boundary cell E[i'][0] = i'
         * with i' > i.  Once i >= k those boundary cells already exceed k,
         * so a whole row above k ends the band (Ukkonen's cut-off); before
         * that, a band lying left of column 0 may still meet column 0. */
        if (rowmin > k && (int)i >= k) return 0;
        memcpy(prev, cur, sizeof(int) * W);
    }
    int m = 0;
    for (int b = 0; b < W; b++) {
        int64_t c = (int64_t)n + lo + b;
        if (c >= 1 && c <= (int64_t)L && prev[b] <= k) {
            out_end[m] = (int32_t)(c - 1);
            out_err[m] = prev[b];
            m++;
        }
    }
    return m;
}

/* record key for sorting hits: read (26 bits) | strand | end (32 bits) | errors (5 bits) */
static uint64_t hit_key(uint32_t r, int s, uint32_t e, int v) {
    return ((uint64_t)r << 38) | ((uint64_t)s << 37) | ((uint64_t)e << 5) | (uint64_t)v;
}

/* sort records, keep the smallest error count per (read, strand, end), and
 * in best-stratum mode keep only each read's minimum error count */
static int finish_hits(uint64_t *keys, uint64_t n, uint32_t n_reads, int best, orc_hit **out,
                       uint64_t *n_out) {
    qsort(keys, n, sizeof(uint64_t), cmp_u64);
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (m > 0 && (keys[m - 1] >> 5) == (keys[i] >> 5)) continue; /* same (r, s, e): first has min v */
        keys[m++] = keys[i];
    }
    uint8_t *minv = NULL;
    if (best) {
        minv = (uint8_t *)malloc(n_reads ? n_reads : 1);
        if (!minv) return -2;
        memset(minv, 0xff, n_reads ? n_reads : 1);
        for (uint64_t i = 0; i < m; i++) {
            uint32_t r = (uint32_t)(keys[i] >> 38);
            uint8_t v = (uint8_t)(keys[i] & 31);
            if (v < minv[r]) minv[r] = v;
        }
    }
    orc_hit *h = (orc_hit *)malloc(sizeof(orc_hit) * (m ? m : 1));
    if (!h) {
        free(minv);
        return -2;
    }
    uint64_t o = 0;
    for (uint64_t i = 0; i < m; i++) {
        uint32_t r = (uint32_t)(keys[i] >> 38);
        uint8_t v = (uint8_t)(keys[i] & 31);
        if (best && v != minv[r]) continue;
        h[o].read_id = r;
        h[o].strand = (uint8_t)((keys[i] >> 37) & 1);
        h[o].end_pos = (uint32_t)((keys[i] >> 5) & 0xffffffffULL);
        h[o].errors = v;
        h[o].pad = 0;
        o++;
    }
    free(minv);
    *out = h;
    *n_out = o;
    return 0;
}

typedef struct {
    const uint8_t *text[2];
    uint64_t L;
    const uint8_t *codes;
    const uint64_t *offsets;
    const uint8_t *k_per_read;
    const uint64_t *cands; /* unique candidate keys */
    u64vec *out;
    int failed;
} verify_job;

static void verify_range(void *arg, int tid, uint64_t lo, uint64_t hi) {
    verify_job *j = (verify_job *)arg;
    int32_t ee[64], vv[64];
    for (uint64_t c = lo; c < hi; c++) {
        uint32_t r = (uint32_t)(j->cands[c] >> 33);
        int s = (int)((j->cands[c] >> 32) & 1);
        int64_t d = (int64_t)(uint32_t)j->cands[c] - ORC_DBIAS;
        uint32_t n = (uint32_t)(j->offsets[r + 1] - j->offsets[r]);
        int k = j->k_per_read[r];
        int m = orc_banded(j->text[s], j->L, j->codes + j->offsets[r], n, d, k, ee, vv);
        for (int t = 0; t < m; t++)
            if (vec_push(&j->out[tid], hit_key(r, s, (uint32_t)ee[t], vv[t]))) {
                j->failed = 1;
                return;
            }
    }
}

/* Filtration + validation with the conventional index.  Requires
 * (k_r + 1) * q <= n_r for every read (q-gram lemma, Section 2.2). */
int orc_map_filtered(const uint8_t *ref, uint64_t L, const uint8_t *codes, const uint64_t *offsets,
                     uint32_t n_reads, int q, const uint8_t *k_per_read, int best,
                     uint32_t mask_max_occ, int nthreads, orc_hit **out, uint64_t *n_out) {
    *out = NULL;
    *n_out = 0;
    for (uint32_t r = 0; r < n_reads; r++) {
        uint64_t n = offsets[r + 1] - offsets[r];
        if ((uint64_t)(k_per_read[r] + 1) * (uint64_t)q > n || k_per_read[r] > 31) return -3;
    }
    nthreads = orc_threads(nthreads);
    const uint64_t G = 1ULL << (2 * q);
    uint64_t T = orc_qgram_count(offsets, n_reads, q);
    uint64_t *A = (uint64_t *)malloc(sizeof(uint64_t) * (G + 1));
    uint32_t *Pr = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
    uint32_t *Po = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
    uint8_t *rc = reverse_complement(ref, L);
    int st = (A && Pr && Po && rc) ? orc_qgram_index(codes, offsets, n_reads, q, A, Pr, Po) : -2;
    uint64_t *cands = NULL, nc = 0;
    if (!st)
        st = collect_candidates(ref, rc, L, q, A, Pr, Po, mask_max_occ, nthreads, &cands, &nc);
    free(A);
    free(Pr);
    free(Po);
    if (st) {
        free(rc);
        return st;
    }
    /* the same (read, strand, diagonal) reached through several q-grams is
     * validated once */
    qsort(cands, nc, sizeof(uint64_t), cmp_u64);
    uint64_t nu = 0;
    for (uint64_t i = 0; i < nc; i++)
        if (nu == 0 || cands[nu - 1] != cands[i]) cands[nu++] = cands[i];

    verify_job j;
    j.text[0] = ref;
    j.text[1] = rc;
    j.L = L;
    j.codes = codes;
    j.offsets = offsets;
    j.k_per_read = k_per_read;
    j.cands = cands;
    j.failed = 0;
    j.out = (u64vec *)calloc((size_t)nthreads, sizeof(u64vec));
    if (!j.out) st = -2;
    if (!st) parallel_for(nthreads, nu, verify_range, &j);
    free(cands);
    free(rc);
    if (st) return st;
    size_t total = 0;
    for (int t = 0; t < nthreads; t++) total += j.out[t].n;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
    size_t at = 0;
    for (int t = 0; t < nthreads; t++) {
        if (keys && j.out[t].n) memcpy(keys + at, j.out[t].v, sizeof(uint64_t) * j.out[t].n);
        at += j.out[t].n;
        free(j.out[t].v);
    }
    free(j.out);
    if (!keys || j.failed) {
        free(keys);
        return -2;
    }
    st = finish_hits(keys, total, n_reads, best, out, n_out);
    free(keys);
    return st;
}

/* ------------------------------------------------------------------------ */
/* the plain definition: full semiglobal DP against both strands             */

typedef struct {
    const uint8_t *text[2];
    uint64_t L;
    const uint8_t *codes;
    const uint64_t *offsets;
    const uint8_t *k_per_read;
    u64vec *out;
    int failed;
} sellers_job;

static void sellers_range(void *arg, int tid, uint64_t lo, uint64_t hi) {
    sellers_job *j = (sellers_job *)arg;
    for (uint64_t x = lo; x < hi; x++) {
        uint32_t r = (uint32_t)(x / 2);
        int s = (int)(x % 2);
        const uint8_t *read = j->codes + j->offsets[r];
        const uint32_t n = (uint32_t)(j->offsets[r + 1] - j->offsets[r]);
        const int k = j->k_per_read[r];
        const uint8_t *t = j->text[s];
        int *col = (int *)malloc(sizeof(int) * (n + 1));
        if (!col) {
            j->failed = 1;
            return;
        }
        for (uint32_t i = 0; i <= n; i++) col[i] = (int)i; /* column 0: E[i][0] = i */
        for (uint64_t jc = 1; jc <= j->L; jc++) {
            int diag = col[0]; /* E[0][j-1] */
            col[0] = 0;        /* E[0][j] = 0: an occurrence may start anywhere */
            const uint8_t tj = t[jc - 1];
            for (uint32_t i = 1; i <= n; i++) {
                int left = col[i]; /* E[i][j-1] */
                int v = diag + (read[i - 1] != tj);
                if (left + 1 < v) v = left + 1;
                if (col[i - 1] + 1 < v) v = col[i - 1] + 1; /* E[i-1][j] */
                diag = left;
                col[i] = v;
            }
            if (col[n] <= k && vec_push(&j->out[tid], hit_key(r, s, (uint32_t)(jc - 1), col[n]))) {
                j->failed = 1;
                free(col);
                return;
            }
        }
        free(col);
    }
}

int orc_map_sellers(const uint8_t *ref, uint64_t L, const uint8_t *codes, const uint64_t *offsets,
                    uint32_t n_reads, const uint8_t *k_per_read, int best, int nthreads,
                    orc_hit **out, uint64_t *n_out) {
    *out = NULL;
    *n_out = 0;
    nthreads = orc_threads(nthreads);
    uint8_t *rc = reverse_complement(ref, L);
    if (!rc) return -2;
    sellers_job j;
    j.text[0] = ref;
    j.text[1] = rc;
    j.L = L;
    j.codes = codes;
    j.offsets = offsets;
    j.k_per_read = k_per_read;
    j.failed = 0;
    j.out = (u64vec *)calloc((size_t)nthreads, sizeof(u64vec));
    if (!j.out) {
        free(rc);
        return -2;
    }
    parallel_for(nthreads, 2 * (uint64_t)n_reads, sellers_range, &j);
    free(rc);
    size_t total = 0;
    for (int t = 0; t < nthreads; t++) total += j.out[t].n;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
    size_t at = 0;
    for (int t = 0; t < nthreads; t++) {
        if (keys && j.out[t].n) memcpy(keys + at, j.out[t].v, sizeof(uint64_t) * j.out[t].n);
        at += j.out[t].n;
        free(j.out[t].v);
    }
    free(j.out);
    if (!keys || j.failed) {
        free(keys);
        return -2;
    }
    int st = finish_hits(keys, total, n_reads, best, out, n_out);
    free(keys);
    return st;
}

/* ------------------------------------------------------------------------ */
/* start and alignment of one hit, by the full matrix of the reversed read  */

/* ops: 0 '=' (match), 1 'X' (substitution), 2 'I' (read letter not in the
 * text), 3 'D' (text letter not in the read), first op first.  Returns the
 * number of ops (<= n + span), with *start and *errors; -1 if span_max < 0
 * or memory runs out.  Text columns considered: j = 0 .. min(e + 1,
 * span_max). */
int orc_align(const uint8_t *text, uint64_t L, const uint8_t *x, uint32_t n, uint64_t e,
              int span_max, int64_t *start, int32_t *errors, uint8_t *ops) {
    if (span_max < 0 || e >= L) return -1;
    const int J = (uint64_t)span_max < e + 1 ? span_max : (int)(e + 1);
    const int W = J + 1;
    int *F = (int *)malloc(sizeof(int) * (size_t)(n + 1) * (size_t)W);
    if (!F) return -1;
#define ORC_F(i, j) F[(size_t)(i) * (size_t)W + (size_t)(j)]
    for (int j = 0; j <= J; j++) ORC_F(0, j) = j;
    for (uint32_t i = 1; i <= n; i++) {
        const uint8_t xi = x[n - i]; /* the i-th letter from the read's end */
        ORC_F(i, 0) = (int)i;
        for (int j = 1; j <= J; j++) {
            const uint8_t tj = text[e + 1 - (uint64_t)j]; /* the j-th letter back from e */
            int v = ORC_F(i - 1, j - 1) + (xi != tj);
            if (ORC_F(i - 1, j) + 1 < v) v = ORC_F(i - 1, j) + 1;
            if (ORC_F(i, j - 1) + 1 < v) v = ORC_F(i, j - 1) + 1;
            ORC_F(i, j) = v;
        }
    }
    int best = 0;
    for (int j = 1; j <= J; j++)
        if (ORC_F(n, j) < ORC_F(n, best)) best = j;
    *errors = ORC_F(n, best);
    *start = (int64_t)e + 1 - best;
    int m = 0;
    int i = (int)n, j = best;
    while (i > 0 || j > 0) {
        const int v = ORC_F(i, j);
        if (i > 0 && j > 0) {
            const int sub = x[n - (uint32_t)i] != text[e + 1 - (uint64_t)j];
            if (ORC_F(i - 1, j - 1) + sub == v) {
                ops[m++] = (uint8_t)sub;
                i--;
                j--;
                continue;
            }
        }
        if (i > 0 && ORC_F(i - 1, j) + 1 == v) {
            ops[m++] = 2;
            i--;
            continue;
        }
        ops[m++] = 3;
        j--;
    }
#undef ORC_F
    free(F);
    return m;
}

void orc_free(void *p) { free(p); }
