// Internal declarations shared by the HIP translation units of libpeanut.
// Device layouts:
//  * packed text: 2 bits per base, 16 bases per uint32, first base in the
//    most significant bits (base t lives in word t/16 at bits 30-2(t%16)),
//    so a q-gram code with its first base most significant is a funnel
//    shift of two words.
//  * bit planes (verification): per 32 positions one uint4 {H, L, V, 0}
//    with bit b of H / L = high / low bit of the base code at position
//    32*blk + b and V = 1 where the position lies inside [0, L).  Arrays are
//    padded by PN_PAD_BLOCKS blocks on each side so that band windows that
//    hang over either end of the reference read "no base here".
//  * read planes: per read, PN_READ_WORDS uint2 {H, L} words (LSB-first).
//  * O entry (64 bits): high word (cls << 29) | (read << 8) | offset, cls =
//    code of the letter before the q-gram in its read or 4 at offset 0; low
//    word (next4 << 24) | (nav << 21) | (piece << 20) | rule byte: the (up
//    to) four read letters after the q-gram, first letter in the top bits,
//    how many exist (0..4), whether the entry starts a piece (offset a
//    multiple of q + 4 and nav = 4: the read's disjoint windows of q + 4
//    letters), and in the low byte the read's seed-rule bits of the current
//    mapping call (written by launch_stamp_rules).
//  * low-complexity q-grams: period <= 2 (homopolymers and dinucleotide
//    repeats), see pn_low_complexity.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PN_MAX_READ_LEN 256
#define PN_READ_WORDS (PN_MAX_READ_LEN / 32)
#define PN_MAX_READS (1u << 21)
#define PN_MAX_K 31   // 2k + 1 <= 63 band diagonals
#define PN_BAND_K 15  // largest k whose band fits one 32-bit word (the fast passes)
#define PN_MAX_Q 16  // a q-gram code fills at most one 32-bit word
#define PN_PAD_BLOCKS 16
#define PN_PAD_POS (32 * PN_PAD_BLOCKS)
#define PN_DBIAS 65536u
#define PN_CLS_NONE 4u
#define PN_CAND_NONE 0xffffffffu  // padding slot in the candidate array
// Candidate word x: read id (bits 0-20) | (read length - 1) << 21 (bits
// 21-28) | PN_CAND_TAIL | strand << 31.  PN_CAND_TAIL asks verification's
// first pass to check the read's last rows instead of its first ones (set
// for reads whose low-complexity q-grams lie mostly in their first half,
// whose first rows would match along a repeat run); either check only
// drops a candidate without a hit.  The length travels in the candidate so
// that verification need not gather the read's offsets.
#define PN_CAND_TAIL 0x40000000u
#define PN_CAND_READ 0x001fffffu
#define PN_CAND_LEN_SHIFT 21
__host__ __device__ inline int pn_cand_len(uint32_t x) {
    return (int)((x >> PN_CAND_LEN_SHIFT) & 0xffu) + 1;
}

// Blocks for a kernel that walks n elements with a grid-stride loop.  A
// dispatch covers fewer than 2^32 work-items (the packet's grid size is a
// 32-bit count), so one thread per element cannot cover the position set
// of a reference past 2^31 bases (both strands); the grid is capped well
// below that and every thread takes several elements.
inline unsigned pn_stride_blocks(uint64_t n, unsigned threads) {
    const uint64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < (1ull << 20) ? (b ? b : 1) : (1ull << 20));
}

// ---------------------------------------------------------------------------
// descriptors passed by value to kernels

struct PnRefDev {
    const uint32_t *packed;  // 2-bit text, ceil(L/16) + 4 words
    const uint4 *planes[2];  // strand 0 and strand 1 bit planes (padded)
    uint64_t L;
    uint64_t n_plane_blocks;
};

struct PnIndexDev {
    const uint32_t *packed;   // 2-bit concatenated reads
    const uint64_t *offsets;  // n_reads + 1
    const uint2 *rplanes;     // n_reads * PN_READ_WORDS
    const uint2 *rplanes_rc;  // the same for each read's reverse complement
    const void *I;            // n_groups words of w bits
    const uint32_t *S;        // n_groups + 1 (s_half: every second one, S[0], S[2], ...)
    const uint32_t *Sp;       // n_distinct + 1
    const unsigned long long *O;  // n_qgrams 64-bit entries
    const uint32_t *lcinfo;   // per read: low-complexity offsets | (intervals << 16)
    const uint32_t *tab_id;   // ordered index: per slot, its slice table or ~0 (or null)
    const uint32_t *tabs;     // slice tables, pn::kTabWidth words each
    uint32_t n_reads;
    uint32_t max_len;
    int q;
    int log2w;
    uint64_t n_groups;
    int after_sorted;  // each slice of O ordered by the letters after the q-gram first
    int s_half;        // S sampled at even groups (pn_group_start)
};

// ---------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ uint32_t pn_base_at(const uint32_t *packed, uint64_t t) {
    return (packed[t >> 4] >> (30 - 2 * (uint32_t)(t & 15))) & 3u;
}

// 32 bits of packed text starting at base t: bases t..t+15, first base in
// the top two bits.
__device__ __forceinline__ uint32_t pn_window16(const uint32_t *packed, uint64_t t) {
    uint64_t wi = t >> 4;
    uint32_t sh = 2 * (uint32_t)(t & 15);
    uint32_t hi = packed[wi];
    uint32_t lo = packed[wi + 1];
    return sh ? (hi << sh) | (lo >> (32 - sh)) : hi;
}

// reverse complement of a q-gram code (first base most significant):
// complement every base (code xor 3) and reverse the order of the 2-bit
// groups.
__device__ __forceinline__ uint32_t pn_revcomp_code(uint32_t g, int q) {
    uint32_t x = ~g;
    x = __builtin_bitreverse32(x);                       // reverses bits
    x = ((x >> 1) & 0x55555555u) | ((x & 0x55555555u) << 1);  // restore bit order inside each base
    return x >> (32 - 2 * q);
}

// q-gram of q letters (2q bits) with period 1 or 2: letter t equals letter
// t+2 throughout.  Such q-grams (homopolymers, dinucleotide repeats) are the
// ones whose occurrence lists explode; reads that do not need them to be
// found skip them (see pn_filter.hip).
// (For q < 3 no q-gram is treated this way.)
__device__ __forceinline__ bool pn_low_complexity(uint32_t g, int q) {
    if (q < 3) return false;
    const uint32_t mask = (1u << (2 * (q - 2))) - 1u;
    return ((g ^ (g >> 4)) & mask) == 0u;
}

template <typename TW>
__device__ __forceinline__ int pn_popc(TW x);
template <>
__device__ __forceinline__ int pn_popc<uint32_t>(uint32_t x) { return __popc(x); }
template <>
__device__ __forceinline__ int pn_popc<uint64_t>(uint64_t x) { return __popcll(x); }

// S[i], the number of occurring q-grams in the groups before i.  A sampled
// S (Section 2.2, "Sampling S") keeps the even entries only; an odd one is
// the even one before it plus the population count of that group's word.
template <typename TW>
__device__ __forceinline__ uint32_t pn_group_start(const PnIndexDev &ix, const TW *I, uint32_t i) {
    if (!ix.s_half) return ix.S[i];
    const uint32_t v = ix.S[i >> 1];
    return (i & 1u) ? v + (uint32_t)pn_popc<TW>(I[i - 1]) : v;
}
template <>
__device__ __forceinline__ int pn_popc<unsigned long long>(unsigned long long x) {
    return __popcll(x);
}

// exclusive scan of one uint32 per thread over a 256-thread block (four
// waves of 64); returns the thread's exclusive prefix, *total = block sum.
// Every thread of the block must call it (it synchronises).
__device__ __forceinline__ uint32_t pn_block_excl_scan(uint32_t x, uint32_t *total) {
    __shared__ uint32_t ws[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
        before += w < wave ? ws[w] : 0u;
        all += ws[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

// ---------------------------------------------------------------------------
// host launchers (all asynchronous on `st`)

namespace pn {

// pn_pack.hip
void launch_pack2(const char *ascii, uint64_t n, uint32_t *packed, uint32_t *status,
                  hipStream_t st);
void launch_ref_planes(const uint32_t *packed, uint64_t L, uint4 *planes0, uint4 *planes1,
                       uint64_t n_blocks, hipStream_t st);
void launch_read_meta(const uint64_t *offsets, uint32_t n_reads, int q, uint64_t n_bases,
                      uint64_t *stats, hipStream_t st);
void launch_read_planes(const uint32_t *packed, const uint64_t *offsets, uint32_t n_reads,
                        uint2 *rplanes, hipStream_t st);  // rplanes: 2 * n_reads * PN_READ_WORDS (forward, then reverse complements)
void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);

// pn_scan.hip: exclusive prefix sums; out has n + 1 entries (out[n] = total)
void launch_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *partials,
                     hipStream_t st);
void launch_scan_popc(const void *I, int log2w, uint32_t *out, uint64_t n, uint32_t *partials,
                      hipStream_t st);
uint64_t scan_partials_size(uint64_t n);

// pn_index.hip (Algorithm 1)
void launch_read_nq(const PnIndexDev &ix, uint32_t *nq, hipStream_t st);
// index keys hold the four letters after each q-gram and their count when
// there is room: 2q bits of q-gram, 2 of the letter before, 9 of the
// letters after (with their count), 29 of read and offset <= 64
// (otherwise: 2q + 3 bits, the letter before or "none", then read and offset)
inline bool index_key_carries(int q) { return 2 * q + 2 + 9 + 29 <= 64; }
// bits [index_gram_lo(q), index_gram_lo(q) + 2q) of an index key hold the
// q-gram; when the key carries the letters after it, they are the 9 bits
// below (an index sorted by all 2q + 9 low bits has each slice of O ordered
// by those letters, which lets filtration find the entries whose next
// letters agree with the text by binary search)
inline int index_gram_lo(int q) { return index_key_carries(q) ? 9 : 0; }
// keys of all T occurrences (qoff: exclusive prefix of the reads' q-gram
// counts, qoff[n_reads] = T), with hist0 (tile-major, 256 words per tile of
// `tile` keys) the counts of their lowest 8 bits; first_read: one word per
// tile (scratch)
void launch_qgram_keys(const PnIndexDev &ix, const uint32_t *qoff, uint64_t T, uint64_t tile,
                       uint32_t *first_read, unsigned long long *keys, uint32_t *hist0,
                       hipStream_t st);
// O, group-start flags and I (zeroed by the caller) from keys sorted by
// their low 2q bits
void launch_index_from_sorted(const PnIndexDev &ix, const unsigned long long *keys, uint64_t T,
                              unsigned long long *O, uint8_t *flags, void *I, hipStream_t st);
// S' from the group-start flags of the sorted occurrences: Sp[x] = position
// of the x-th start, Sp[D] = T (partials: scan_partials_size(T) words)
void launch_starts_to_sp(const uint8_t *flags, uint64_t T, uint32_t *partials, uint32_t *Sp,
                         hipStream_t st);
void launch_read_lc(const PnIndexDev &ix, uint32_t *lcinfo, hipStream_t st);
// slice tables of an ordered index (pn_index.hip): for a slot x whose slice
// is longer than kTabMin, tabs[tab_id[x] * kTabWidth + t] = (first entry of
// the slice whose order value 2 code + piece is t or more) - slice start
constexpr uint32_t kTabWidth = 513;  // t = 0 .. 512: every 2N + 1 and 2N + 2, N < 256
constexpr uint32_t kTabMin = 128;
// flags[x] = slice of slot x longer than min_len (D slots)
void launch_tab_flags(const uint32_t *Sp, uint64_t D, uint32_t min_len, uint32_t *flags,
                      hipStream_t st);
// num: exclusive scan of those flags; writes tab_id (D words), list (n_tabs
// words: the slot of each table) and the n_tabs tables
void launch_tab_build(const unsigned long long *O, const uint32_t *Sp, uint64_t D,
                      uint32_t min_len, const uint32_t *num, uint32_t n_tabs, uint32_t *tab_id,
                      uint32_t *list, uint32_t *tabs, hipStream_t st);
// read lengths into candidate words made without them (pn_validate's
// host candidates); a read of length 0 or over PN_MAX_READ_LEN makes the
// candidate a padding slot
void launch_cands_len(uint2 *cands, uint64_t n, const uint64_t *offsets, hipStream_t st);
// the number of occurrences in slices of O longer than min_len, added to
// *out (D: device word holding the number of slices)
void launch_long_entries(const uint32_t *D, const uint32_t *Sp, uint32_t min_len,
                         unsigned long long *out, hipStream_t st);
// a sampled S from the full one: out[t] = S[2 t] for t = 0 .. n_groups / 2
void launch_sample_s(const uint32_t *S, uint64_t n_groups, uint32_t *out, hipStream_t st);

// Append-only output split into kShards regions of `region_cap` entries,
// each with its own counter: a thread block appends to region
// blockIdx.x % kShards.  One counter taken by every wave of the chip
// serialises at a single memory channel; 64 of them spread over channels.
constexpr uint32_t kShards = 64;
struct Shards {
    unsigned long long *counts;  // kShards counters (may exceed region_cap)
    uint64_t region_cap;
};

// pn_filter.hip (Algorithm 2)
constexpr int kFilterThreads = 256;
constexpr int kFilterPPT = 8;  // forward positions per thread
constexpr int kFilterBlockPos = kFilterThreads * kFilterPPT;
constexpr int kLcPatterns = 16;  // period <= 2 q-grams: first two letters
struct FilterOut {
    uint2 *cands;                 // (read | strand << 31, diagonal + PN_DBIAS), kShards regions
    Shards sh;                    // per-region append counters
    // entries whose occurrence ranges are longer than heavy_min, set aside
    // for k_filter_heavy: 2 uint4 per item, kShards regions
    uint4 *heavy;
    Shards hsh;
    uint32_t heavy_min;
    // per region g (work counters of k_filter): stats[4g] = occurrence pairs
    // seen (sum of k_end - k_start), stats[4g+1] = index entries read (by
    // either kernel), stats[4g+2] = the part of those set aside for
    // k_filter_heavy, stats[4g+3] = candidate slots k_filter wrote
    unsigned long long *stats;
};
// per read: bit 7 = keeps its low-complexity seeds, bit 6 = its
// low-complexity offsets lie mostly in its first half (candidates get
// PN_CAND_TAIL), bit 3 = piece mode (its candidates come from exact pieces
// only; then bits 4-6 = t, windows at offsets below 16 t lie in its first
// half and their candidates get PN_CAND_TAIL), bits 0-2 = extra letters of
// exact run required beyond q (0..4).
// Status: bit 2 some k_r too large, bit 4 the lemma fails for some read.
// plain: every read gets rule byte 0x80 (keeps its low-complexity seeds, no
// exact run required, no piece mode), for filtration of a masked position
// set, where a pair may be the only one left of its alignment
// rstamp (may be null): per read the rule byte | (length - 1) << 8, the
// word k_stamp_rules writes into the low 16 bits of the read's O entries
void launch_read_rules(const PnIndexDev &ix, int kglob, const uint8_t *kpr, uint8_t *rinfo,
                       uint16_t *rstamp, uint32_t *status, bool plain, hipStream_t st);
// sizes of the 16 low-complexity q-grams' O slices (for sizing side lists)
void launch_lc_sizes(const PnIndexDev &ix, uint32_t *sizes, hipStream_t st);
// low-complexity occurrence lists restricted to reads that keep them
// (grouped by preceding letter; side_cls: 6 bounds per q-gram)
// (scratch: 10 x kLcPatterns words)
void launch_lc_side(const PnIndexDev &ix, const uint8_t *rinfo, unsigned long long *side,
                    const uint32_t *region, uint32_t *side_cls, uint32_t *scratch,
                    hipStream_t st);
// write each read's rule byte into the low byte of its O entries
void launch_stamp_rules(unsigned long long *O, uint64_t n, const uint16_t *rstamp, hipStream_t st);
// the position set P of a reference for one q, sorted by q-gram.  Two
// layouts: keys ((p << 1 | strand) << 2q) | q-gram with a 16-bit context
// each (ctx), or, when (p << 1 | strand) fits in 54 - 2q bits, one packed
// word per entry and ctx == nullptr: (p << 1 | strand) << (2q + 10) | the
// letters after (8 bits) << (2q + 2) | the letter before << 2q | q-gram.
// In the packed form whether there is a letter before (p >= 1) and how many
// letters follow (min(L - q - p, 4)) come from p, on both strands.
struct RefQDev {
    const unsigned long long *keys;
    const uint16_t *ctx;
    uint64_t n;  // 2 (L - q + 1)
    // repeat masking: bit g set = q-gram g is left out of filtration (null:
    // no masking)
    const uint32_t *mask;
};
// repeat masking: bit g of `bits` (4^q bits, zeroed by the caller) set for
// every q-gram with more than max_occ entries in P
void launch_mask_runs(const RefQDev &P, int q, uint32_t max_occ, uint32_t *bits, hipStream_t st);
inline bool refq_packs(uint64_t L, int q) {
    int bits = 0;
    for (uint64_t v = 2 * L; v > 1; v >>= 1) bits++;  // (p << 1 | strand) < 2L
    return bits + 1 <= 54 - 2 * q;
}
// letters after the q-gram that P's sort keys carry (up to 4, as many as
// fit beside (p << 1 | strand) and the q-gram in 64 bits): P is ordered by
// q-gram and then by them
inline int refq_sort_letters(uint64_t L, int q) {
    int bits = 0;
    for (uint64_t v = 2 * L; v > 1; v >>= 1) bits++;
    const int a = (64 - 2 * q - (bits + 1)) / 2;
    return a < 0 ? 0 : (a > 4 ? 4 : a);
}
void launch_refq_keys(const PnRefDev &ref, int q, unsigned long long *keys, hipStream_t st);
// the contexts of the sorted keys: into ctx, or (ctx == nullptr) into the
// keys themselves in the packed layout
void launch_refq_ctx(const PnRefDev &ref, int q, unsigned long long *keys, uint64_t n,
                     uint16_t *ctx, hipStream_t st);
// Lists of O entries made per mapping call, read by filtration:
//  * side lists: the occurrences of the 16 low-complexity q-grams from reads
//    that keep them (rule 2), grouped by the letter before, with their
//    class bounds side_cls (6 per q-gram);
//  * lax lists (when sub_on: the index orders each slice by the letters
//    after the q-gram, piece starts last among equal letters): for each
//    slice longer than sub_min, its entries whose read is not in piece
//    mode, at laxO[lax[x].x .. lax[x].x + lax[x].y) for slot x.  Filtration
//    then visits, in such a slice, only the binary-searched piece starts
//    whose four letters equal the text's, plus the slice's lax list.
struct Lists {
    const unsigned long long *side;
    const uint32_t *side_cls;
    const unsigned long long *laxO;
    const uint2 *lax;
    uint32_t sub_min;
    int sub_on;
};
// an index orders its slices when a notable share of its occurrences lie in
// slices longer than kLongSlice (reads from repeat families); filtration
// then searches every slice of it longer than kSearchMin (and the lax lists
// cover those slices); shorter slices are walked whole (16: two binary
// searches cost more than walking a slice that short)
// (64: reads from repeat families put some 8 % of their occurrences into
// slices that long, a mixed-length batch of 2 M reads drawn uniformly from a
// reference with a few segmental copies 0.4 %, and ordering it only costs)
constexpr uint32_t kLongSlice = 64;
constexpr uint32_t kSearchMin = 16;
// the occurrence lists k_filter set aside (FilterOut::heavy)
void launch_filter_heavy(const PnIndexDev &ix, const Lists &ls, FilterOut out, hipStream_t st);
// the lax lists of the slots [0, n_slots) (count: one zeroed word, receives
// the number of entries written to laxO, which needs room for all of O)
void launch_lax_lists(const PnIndexDev &ix, uint64_t n_slots, uint32_t min_len, uint2 *lax,
                      unsigned long long *laxO, unsigned long long *count, hipStream_t st);
// the longest occurrence list k_filter walks itself: 32 when the lists are
// short on average (fewer than 16 entries per q-gram of the index: the long
// ones are rare and are better walked by a whole wave), else 64 (where most
// lists are long, a smaller bound would make nearly every list an item)
inline uint32_t filter_heavy_min(uint64_t n_qgrams, int q) {
    return n_qgrams < (16ull << (2 * q)) ? 32u : 64u;
}
void launch_filter(const PnRefDev &ref, const RefQDev &P, const PnIndexDev &ix, const Lists &ls,
                   FilterOut out, hipStream_t st);

// pn_verify.hip (Section 3.3)
struct VerifyIn {
    const uint2 *cands;
    const unsigned long long *counts;  // candidates per region (may exceed region_cap)
    uint32_t regions;                  // 1 or kShards
    uint64_t region_cap;
};
struct VerifyOut {
    unsigned long long *records;  // packed hit keys, kShards regions
    Shards sh;
    unsigned long long *rows;     // band rows computed (work counter)
    int ebits;                    // bits for end positions in a key
};
// Two passes: every candidate for at most 16 rows, then the candidates still
// alive from row 0 to the end.  `longc` (in.regions regions of
// in.region_cap entries) and its counters `n_long` (in.regions words, zeroed
// by the caller) hold the second pass's candidates.  `first` picks the pass;
// the second pass reads `longc` and ignores in.cands.  Candidates of reads
// with k > PN_BAND_K skip both passes: the first (and the count filter) puts
// them into `longc` as they are, for launch_verify_wide.
void launch_verify(const PnRefDev &ref, const PnIndexDev &ix, VerifyIn in, int kglob,
                   const uint8_t *kpr, VerifyOut out, uint2 *longc, unsigned long long *n_long,
                   bool first, hipStream_t st);
// The 64-bit band pass over `in` (the survivor list: longc and n_long) for
// the candidates of reads with PN_BAND_K < k <= PN_MAX_K; records into out.
void launch_verify_wide(const PnRefDev &ref, const PnIndexDev &ix, VerifyIn in, int kglob,
                        const uint8_t *kpr, VerifyOut out, hipStream_t st);

// The count filter (pn_verify.hip): each candidate of `in` whose band holds
// at least floor(n/4) - k exact pieces of 4 read letters (the q-gram lemma
// on disjoint pieces; Section 2.2) goes to surv (in's shape, counters n_surv
// zeroed by the caller) for the band pass; *letters += read letters looked at.
void launch_count(const PnRefDev &ref, const PnIndexDev &ix, VerifyIn in, int kglob,
                  const uint8_t *kpr, uint2 *surv, unsigned long long *n_surv,
                  unsigned long long *letters, hipStream_t st);
// candidates in the C ABI's 16-byte layout (device) to verification words;
// out-of-range ones become padding and set bit 3 of *status
// (the read lengths from `offsets` go into the candidate words)
void launch_cands_in(const void *in, uint64_t n, uint32_t n_reads, uint64_t L,
                     const uint64_t *offsets, uint2 *out,
                     uint32_t *status, hipStream_t st);

// pn_scan.hip: concatenate the regions of a sharded list (8-byte entries)
// into dst; counts past region_cap are clipped
void launch_gather_shards(const unsigned long long *src, const unsigned long long *counts,
                          uint32_t regions, uint64_t region_cap, unsigned long long *dst,
                          hipStream_t st);

// pn_canon.hip: sort + duplicate removal + strata + output
uint64_t radix_temp_size(uint64_t n);  // bytes
// stable sort by bits [lo, bits) of the keys; the result is in the
// returned buffer (keys or tmp)
// (hist0: if given, the first pass's per-tile counts of the lowest 8 bits,
// hist0[tile][digit] over tiles of radix_tile_keys(n) keys)
unsigned long long *radix_sort_u64_any(unsigned long long *keys, unsigned long long *tmp,
                                       uint64_t n, int bits, void *temp, hipStream_t st,
                                       int lo = 0, const uint32_t *hist0 = nullptr);
uint64_t radix_tile_keys(uint64_t n);
// index keys that carry the letters after the q-gram (q <= 12), sorted by
// (q-gram, letters-after code, piece start); result in keys or tmp
unsigned long long *radix_sort_index_slices(unsigned long long *keys, unsigned long long *tmp,
                                            uint64_t n, int q, void *temp, hipStream_t st);
void radix_sort_u64(unsigned long long *keys, unsigned long long *tmp, uint64_t n, int bits,
                    void *temp, hipStream_t st, int lo = 0);
void launch_finish_hits(const unsigned long long *sorted, uint64_t n, int ebits, int best,
                        uint32_t n_reads, uint32_t *minv, uint32_t *flags, uint32_t *pos,
                        uint32_t *partials, void *out_hits, uint64_t capacity,
                        unsigned long long *n_out, hipStream_t st);
// start and alignment of the hits of error count v (pn_align.hip): hw the
// chunk's hit records, perm the chunk-local indices of the cnt hits, bp
// cnt * (longest read) words of work space
void launch_align(const PnRefDev &ref, const PnIndexDev &ix, int v, const uint32_t *hw,
                  const uint32_t *perm, uint32_t cnt, unsigned long long *bp, uint32_t *starts,
                  uint8_t *errs, uint8_t *ops, uint32_t stride, uint16_t *n_ops, hipStream_t st);
void launch_records_to_hits(const unsigned long long *sorted, uint64_t n, int ebits, void *out,
                            hipStream_t st);
void launch_cand_keys(const uint2 *c, uint64_t n, unsigned long long *keys, hipStream_t st);
void launch_keys_to_cands(const unsigned long long *keys, uint64_t n, void *out, hipStream_t st);

}  // namespace pn
