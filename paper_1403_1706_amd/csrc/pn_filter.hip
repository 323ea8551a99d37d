// Algorithm 2: filtration of reference positions through the q-group index
// (Section 3.2).  The position set P holds every (position, strand) of both
// strands (the q-gram of strand 1 at p = L-q-u is the reverse complement of
// the forward q-gram at u) and is sorted by q-gram, as the paper prepares
// it with its reference index: neighbouring lanes then probe the same
// parts of I, S, S' and O.  P is built once per reference and q
// (k_refq_keys, a radix sort, k_refq_ctx), with each entry's context: the
// letter before the q-gram and up to four letters after it (packed into the
// entry's word when there is room, else a 16-bit word beside it).  For every
// entry the occurrences of its q-gram are O[k_start .. k_end) (INDEXPAIR);
// each occurrence (read r, offset o) that passes the rules below becomes a
// candidate (r, strand, diagonal d = p - o).
//
// Every rule below drops a candidate only if another one is guaranteed to
// hold every alignment of the read with at most k_r errors, so the hits do
// not change.  They rest on the counting argument of the q-gram lemma
// (Section 2.2): an alignment with at most k edits leaves every read q-gram
// that no edit touches matched exactly on its diagonal, and one edit
// touches at most q of the read's q-grams.
//
//  1. Left extension.  If the letters before the q-gram agree in read and
//     text, the pair (p-1, o-1) is on the same diagonal and is itself a
//     candidate unless rule 2 drops it; (p, o) is dropped only when
//     (p-1, o-1) stays.
//  2. Low-complexity q-grams (period <= 2: homopolymers, dinucleotide
//     repeats) have huge occurrence lists.  A read with Q_r offsets whose
//     q-gram is not low-complexity keeps, under at most k_r edits, at least
//     Q_r - k_r q of them untouched; if that is >= 1 the read needs none of
//     its low-complexity seeds.  Only reads with Q_r <= k_r q keep them
//     (the per-read flag "keep"), and their occurrences of the 16 such
//     q-grams are collected in side lists so that the long original lists
//     are never walked.
//  3. Exact run length.  The untouched offsets fall into at most
//     k_r + 1 + h_r blocks (h_r = maximal runs of low-complexity offsets),
//     so some block of consecutive untouched offsets has at least
//     ceil((Q_r - k_r q) / (k_r + 1 + h_r)) members: an exact match of length
//     L_r >= q - 1 + that many letters.  (A read that keeps its
//     low-complexity seeds uses ceil((n_r - k_r) / (k_r + 1)), the plain
//     pigeonhole bound.)  The candidate that rule 1 keeps for that run
//     starts at or before the block, so every needed candidate has a forward
//     exact run of at least L_r letters; up to four letters past the q-gram
//     are compared (stored in the O entry and read from the reference
//     window).
//
// Candidates are staged per wave in LDS and appended to the block's output
// region (one of kShards, each with its own counter) with one atomic add
// per wave.  A lane that finds the wave's buffer full reserves output slots
// 64 at a time; slots it does not use are filled with PN_CAND_NONE, which
// verification skips.  Slots are counted even past a region's capacity so
// that the host can grow the buffer and run again.
#include <algorithm>

#include "pn_internal.h"

namespace {

constexpr int kT = pn::kFilterThreads;
constexpr int kPPT = pn::kFilterPPT;
constexpr int kWaves = kT / 64;
constexpr int kWBuf = 256;        // staged candidates per wave (k_filter)
// staged candidates per wave in k_filter_heavy, which flushes once 64 or
// fewer slots are free: fewer, longer flushes (each one's stores and its
// output-slot atomic hold up the wave).  An ordered index (reads from
// repeat families: billions of candidates) takes 896, the largest stage
// with which four blocks fit a CU's 160 KB of LDS (measured against 512,
// 640, 768 and 1024, which leaves room for three); otherwise 512, which
// keeps more waves for the long lists of a plain index.
constexpr int kWBufHeavy = 512;
constexpr int kWBufHeavyOrdered = 896;

// 64 bits of packed reference starting at signed base position B (base B+t
// in bits 63-2t .. 62-2t); packed[-1] and 3 words past the end are readable
__device__ __forceinline__ uint64_t window32(const uint32_t *packed, int64_t B) {
    int64_t wi = B >> 4;
    uint32_t sh = (uint32_t)(B & 15);
    uint64_t hi = ((uint64_t)packed[wi] << 32) | packed[wi + 1];
    if (sh == 0) return hi;
    return (hi << (2 * sh)) | (packed[wi + 2] >> (32 - 2 * sh));
}

__device__ __forceinline__ uint32_t base_rel(uint64_t X, int t) {
    return (uint32_t)(X >> (62 - 2 * t)) & 3u;
}

constexpr uint32_t kLaneChunk = 64;  // slots a lane reserves at a time

// Pointers with their address space spelled out: a plain pointer kept in a
// struct or chosen between two arrays is generic, and the compiler then
// uses flat loads and stores, which wait on both the vector-memory and the
// LDS counters.
typedef __attribute__((address_space(1))) const unsigned long long gu64;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;

__device__ __forceinline__ unsigned long long pack_cand(uint2 c) {
    return ((unsigned long long)c.y << 32) | c.x;
}

struct Stage {
    lds_u64 *buf;    // this wave's LDS buffer (candidates packed as y:x)
    uint32_t *cnt;   // this wave's LDS counter
    uint2 *cands;    // all output regions
    unsigned long long *counts;  // their counters
    uint64_t region_cap;
    uint32_t shard;  // region the next flush goes to (the same in every lane)
    uint32_t lane_shard;           // region of this lane's reserved slots
    unsigned long long lane_base;  // this lane's reserved slots
    uint32_t lane_left;
    uint32_t written;  // output slots this lane accounts for (work counter)
    uint32_t cap;      // slots of the LDS buffer
};

// The lanes that reach this together append one candidate each: one of
// them reserves stage slots for all (per-lane atomics on the one LDS
// counter would serialise), the others take consecutive slots in lane order.
__device__ __forceinline__ void push(Stage &sg, uint2 c) {
    const unsigned long long mask = __ballot(1);  // the lanes appending now
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t first = 0;
    if (lane == leader) first = atomicAdd(sg.cnt, (uint32_t)__popcll(mask));
    first = __shfl(first, leader);
    const uint32_t i = first + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (i < sg.cap) {
        sg.buf[i] = pack_cand(c);
        return;
    }
    if (sg.lane_left == 0) {
        sg.lane_shard = sg.shard;
        sg.lane_base = atomicAdd(sg.counts + sg.shard, (unsigned long long)kLaneChunk);
        sg.lane_left = kLaneChunk;
        sg.written += kLaneChunk;
    }
    const unsigned long long at = sg.lane_base + (kLaneChunk - sg.lane_left);
    sg.lane_left--;
    if (at < sg.region_cap) sg.cands[(uint64_t)sg.lane_shard * sg.region_cap + at] = c;
}

// Copy the wave's staged candidates out with one atomic add (whole wave,
// converged) and empty the stage.  Successive flushes of a wave go to
// successive regions, so the regions fill evenly however unevenly the work
// falls on the blocks.
__device__ __forceinline__ void flush(Stage &sg, int lane) {
    __builtin_amdgcn_wave_barrier();
    const uint32_t n = min(*sg.cnt, sg.cap);
    if (n) {
        uint2 *region = sg.cands + (uint64_t)sg.shard * sg.region_cap;
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(sg.counts + sg.shard, (unsigned long long)n);
            sg.written += n;
        }
        base = __shfl(base, 0);
        for (uint32_t i = lane; i < n; i += 64) {
            const unsigned long long v = sg.buf[i];
            if (base + i < sg.region_cap)
                region[base + i] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
        }
        sg.shard = (sg.shard + 1) % pn::kShards;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) *sg.cnt = 0;
    __builtin_amdgcn_wave_barrier();
}

// pad the unused part of this lane's reserved slots
__device__ __forceinline__ void pad_lane(Stage &sg) {
    for (uint32_t i = 0; i < sg.lane_left; i++) {
        const unsigned long long at = sg.lane_base + (kLaneChunk - sg.lane_left) + i;
        if (at < sg.region_cap)
            sg.cands[(uint64_t)sg.lane_shard * sg.region_cap + at] =
                make_uint2(PN_CAND_NONE, PN_CAND_NONE);
    }
    sg.lane_left = 0;
}

// one (position, strand): INDEXPAIR and the rules of the header comment
// One occurrence.  The read's rule bits (keep flag, required extra run) were
// stamped into the entry's low byte for this mapping call (k_stamp_rules).
// With `strict`, entries of reads that need fewer than four letters past the
// q-gram are skipped: the sub-range they were found in holds only the
// entries whose four letters agree with the text, and such entries are
// visited through the slice's lax list instead (see probe).
// visit_rules decides and hands the candidate to take(c) at the point where
// it is formed (the callers below append it or keep it).
template <typename Take>
__device__ __forceinline__ void visit_rules(const unsigned long long v, int64_t p, uint32_t s,
                                            bool has_prev, uint32_t prev, bool lh, uint32_t N,
                                            uint32_t avail, bool strict, Take &&take) {
    const uint32_t hi = (uint32_t)(v >> 32);
    const uint32_t cls = hi >> 29;
    uint32_t r = (hi >> 8) & (PN_MAX_READS - 1);
    const uint32_t o = hi & 0xffu;
    const uint32_t info = (uint32_t)v & 0xffu;
    // the read's length - 1, stamped beside the rule byte, into the candidate
    r |= ((uint32_t)v & 0xff00u) << (PN_CAND_LEN_SHIFT - 8);
    if ((info >> 3) & 1u) {
        // piece mode: a piece start whose q-gram and four letters after it
        // equal the text's
        if (!((v >> 20) & 1u) || avail < 4u || ((uint32_t)(v >> 24) & 0xffu) != N) return;
        // a window in the read's first half: verification's first pass
        // checks the read's last rows, away from the exact window
        const bool tail = o < 16u * ((info >> 4) & 7u);
        take(make_uint2(r | (tail ? PN_CAND_TAIL : 0u) | (s << 31),
                        (uint32_t)((int64_t)PN_DBIAS + p - (int64_t)o)));
        return;
    }
    // (a searched range of an ordered slice serves reads in piece mode only;
    // the slice's entries of the other reads are in its lax list)
    if (strict) return;
    const bool keep = (info >> 7) & 1u;
    const uint32_t need = info & 7u;                         // rule 3
    if (has_prev && cls == prev && (keep || !lh)) return;  // rule 1
    if (need) {
        const uint32_t nav = (uint32_t)(v >> 21) & 7u;
        const uint32_t next4 = (uint32_t)(v >> 24) & 0xffu;
        if (nav < need || avail < need || ((next4 ^ N) >> (8 - 2 * need)) != 0u) return;
    }
    const uint32_t tail = (info >> 6) & 1u;  // the read's first rows are mostly a repeat run
    take(make_uint2(r | (tail ? PN_CAND_TAIL : 0u) | (s << 31),
                    (uint32_t)((int64_t)PN_DBIAS + p - (int64_t)o)));
}

// the candidate appended to the stage where it is formed
__device__ __forceinline__ void visit(const unsigned long long v, int64_t p, uint32_t s,
                                      bool has_prev, uint32_t prev, bool lh, uint32_t N,
                                      uint32_t avail, bool strict, Stage &sg) {
    visit_rules(v, p, s, has_prev, prev, lh, N, avail, strict, [&](uint2 c) { push(sg, c); });
}

// the candidate kept in c (false: none)
__device__ __forceinline__ bool visit_cand(const unsigned long long v, int64_t p, uint32_t s,
                                           bool has_prev, uint32_t prev, bool lh, uint32_t N,
                                           uint32_t avail, bool strict, uint2 &c) {
    bool got = false;
    visit_rules(v, p, s, has_prev, prev, lh, N, avail, strict, [&](uint2 x) {
        c = x;
        got = true;
    });
    return got;
}

// Converged wave (every lane calls it): appends the lanes' candidates (has)
// to the wave's stage at its count n, a wave-uniform register (no LDS
// counter, no atomics); the caller keeps n + 64 <= the stage's size.
__device__ __forceinline__ void stage_put(const Stage &sg, uint32_t &n, bool has, uint2 c,
                                          int lane) {
    const unsigned long long m = __ballot(has);
    if (has) sg.buf[n + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = pack_cand(c);
    n += (uint32_t)__popcll(m);
}

// flush for a stage whose count is the register n (whole wave, converged)
__device__ __forceinline__ void flush_n(Stage &sg, int lane, uint32_t &n) {
    __builtin_amdgcn_wave_barrier();
    if (n) {
        uint2 *region = sg.cands + (uint64_t)sg.shard * sg.region_cap;
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(sg.counts + sg.shard, (unsigned long long)n);
            sg.written += n;
        }
        base = __shfl(base, 0);
        for (uint32_t i = lane; i < n; i += 64) {
            const unsigned long long v = sg.buf[i];
            if (base + i < sg.region_cap)
                region[base + i] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
        }
        sg.shard = (sg.shard + 1) % pn::kShards;
    }
    __builtin_amdgcn_wave_barrier();
    n = 0;
}

// Occurrence ranges longer than FilterOut::heavy_min are set aside for
// k_filter_heavy, in items of at most kItem occurrences; shorter ones are
// walked by their lane.
constexpr uint32_t kItem = 1024;
constexpr uint32_t kStrictHeavy = 4;
constexpr uint32_t kLongItem = 128;  // k_filter_heavy walks items this long one at a time
constexpr uint32_t kWalk = 4;  // entries a lane loads at a time

// INDEXPAIR(g) and the occurrence ranges to visit for one (position,
// strand): [a0, a1) of srcA and [b0, b1) of srcB (the rules' class cut
// applies to the low-complexity side lists).  Returns k_end - k_start.
// List ids (for the hand-off items): 0 = O, 1 = side lists, 2 = lax lists.
struct Ranges {
    gu64 *srcA, *srcB;
    uint32_t a0, a1, b0, b1;
    uint32_t idA, idB;
    bool strictA;
};

// the order of an O entry inside a slice of an ordered index (see
// pn_index.hip): twice the 9-bit code of its letters after the q-gram, plus
// one for a piece start
__device__ __forceinline__ uint32_t entry_after_code(unsigned long long v) {
    const uint32_t lo = (uint32_t)v;
    const uint32_t next4 = lo >> 24, nav = (lo >> 21) & 7u, piece = (lo >> 20) & 1u;
    uint32_t c;
    switch (nav) {
        case 4: c = next4; break;
        case 3: c = 256u + (next4 >> 2); break;
        case 2: c = 320u + (next4 >> 4); break;
        case 1: c = 336u + (next4 >> 6); break;
        default: c = 340u;
    }
    return 2u * c + piece;
}

// first position in O[lo, hi) whose order value is >= target (they ascend)
__device__ __forceinline__ uint32_t code_lower_bound(gu64 *O, uint32_t lo, uint32_t hi,
                                                     uint32_t target) {
    uint32_t n = hi - lo;
    while (n > 0) {
        const uint32_t half = n >> 1;
        if (entry_after_code(O[lo + half]) < target) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

template <typename TW, bool kSub>
__device__ __forceinline__ uint32_t probe(const PnIndexDev &ix, const pn::Lists &ls, uint32_t g,
                                          bool has_prev, uint32_t prev, uint32_t N,
                                          uint32_t avail, Ranges &rg) {
    rg.srcA = rg.srcB = (gu64 *)ix.O;
    rg.idA = rg.idB = 0;
    rg.strictA = false;
    rg.a0 = rg.a1 = rg.b0 = rg.b1 = 0;
    const TW *I = (const TW *)ix.I;
    const uint32_t wmask = (1u << ix.log2w) - 1;
    const uint32_t i = g >> ix.log2w, j = g & wmask;
    const TW word = I[i];
    if (!((word >> j) & 1)) return 0;
    const uint32_t jp = (uint32_t)pn_popc<TW>(word & (((TW)1 << j) - 1));  // GROUPRANK
    const uint32_t x = pn_group_start<TW>(ix, I, i) + jp;
    const uint32_t ks = ix.Sp[x], ke = ix.Sp[x + 1];
    if (pn_low_complexity(g, ix.q)) {
        // rule 2: only reads that keep these seeds, listed by preceding
        // letter; for those reads rule 1 drops the class equal to `prev`
        const uint32_t *cb = ls.side_cls + (g >> (2 * ix.q - 4)) * 6;
        rg.srcA = rg.srcB = (gu64 *)ls.side;
        rg.idA = rg.idB = 1;
        rg.a0 = cb[0];
        rg.b1 = cb[5];
        rg.a1 = has_prev ? cb[prev] : rg.b1;
        rg.b0 = has_prev ? cb[prev + 1] : rg.b1;
    } else if (kSub && ke - ks > ls.sub_min) {
        // A long slice, ordered by the letters after the q-gram: a read that
        // needs four of them (rule 3) can only pair here with the entries
        // whose four letters are the text's, found by binary search; the
        // entries of the other reads of this slice are in its lax list.
        // (the piece starts among them: the entries of reads in piece mode
        // that can pair here; the other reads' entries are in the lax list)
        if (avail == 4u) {
            const uint32_t tid = ix.tab_id[x];
            if (tid != 0xffffffffu) {
                // a long slice: its table
                const uint32_t *T = ix.tabs + (uint64_t)tid * pn::kTabWidth;
                rg.a0 = ks + T[2u * N + 1u];
                rg.a1 = ks + T[2u * N + 2u];
            } else {
                rg.a0 = code_lower_bound((gu64 *)ix.O, ks, ke, 2u * N + 1u);
                rg.a1 = code_lower_bound((gu64 *)ix.O, rg.a0, ke, 2u * N + 2u);
            }
        } else {
            rg.a0 = rg.a1 = ks;
        }
        rg.strictA = true;
        const uint2 lx = ls.lax[x];
        rg.srcB = (gu64 *)ls.laxO;
        rg.idB = 2;
        rg.b0 = lx.x;
        rg.b1 = lx.x + lx.y;
    } else {
        rg.a0 = ks;
        rg.a1 = ke;
        rg.b0 = rg.b1 = ke;
    }
    return ke - ks;
}

// visit one (position, strand): short ranges by this lane, long ones set
// aside for k_filter_heavy (every lane of the wave calls this together)
template <bool kSub>
__device__ __forceinline__ uint32_t visit_all(const Ranges &rg, int64_t p, uint32_t s,
                                              bool has_prev, uint32_t prev, bool lh, uint32_t N,
                                              uint32_t avail, bool valid, Stage &sg,
                                              const pn::FilterOut &out,
                                              unsigned long long &set_aside) {
    const uint32_t len = (rg.a1 - rg.a0) + (rg.b1 - rg.b0);
    // the longest ranges wait for k_filter_heavy (a wave per item); a
    // searched range of an ordered slice is nearly all candidates, so a lane
    // keeps fewer of them (its wave waits for its longest lane)
    const bool heavy = valid && len > (kSub && rg.strictA ? kStrictHeavy : out.heavy_min);
    // a set-aside entry becomes one item per kItem occurrences (a wave walks
    // an item), so that no single item is long
    const uint32_t nitems = heavy ? (len + kItem - 1) / kItem : 0u;
    const int hl = threadIdx.x & 63;
    // (most positions hand nothing on: the prefix is skipped then)
    if (__ballot(heavy)) {
        uint32_t incl = nitems;  // inclusive prefix over the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d);
            if (hl >= d) incl += y;
        }
        const uint32_t wtotal = __shfl(incl, 63);
        const uint32_t region = (blockIdx.x * kWaves + (threadIdx.x >> 6)) % pn::kShards;
        unsigned long long first = 0;
        if (hl == 0) first = atomicAdd(out.hsh.counts + region, (unsigned long long)wtotal);
        first = __shfl(first, 0);
        if (heavy) {
            set_aside += len;
            // position (32 bits in the item, the rest here), strand, letters
            // and which lists
            // (without sub-ranges both ranges lie in one list, O or the side lists)
            const uint32_t idA = kSub ? rg.idA : rg.idA, idB = kSub ? rg.idB : rg.idA;
            const uint32_t fl = (has_prev ? 1u : 0u) | (lh ? 2u : 0u) | (prev << 2) |
                                (avail << 4) | (N << 8) | (s << 16) | (idA << 17) |
                                (idB << 19) | (kSub && rg.strictA ? 1u << 21 : 0u) |
                                ((uint32_t)((uint64_t)p >> 32) << 22);
            const uint32_t la = rg.a1 - rg.a0;
            unsigned long long at = first + (incl - nitems);
            for (uint32_t c = 0; c < nitems; c++, at++) {
                if (at >= out.hsh.region_cap) break;
                // the part [c * kItem, (c + 1) * kItem) of the two ranges laid end to end
                const uint32_t k0 = c * kItem, k1 = min(len, k0 + kItem);
                const uint32_t a0 = rg.a0 + min(k0, la), a1 = rg.a0 + min(k1, la);
                const uint32_t b0 = rg.b0 + (k0 > la ? k0 - la : 0u);
                const uint32_t b1 = rg.b0 + (k1 > la ? k1 - la : 0u);
                uint4 *h = out.heavy + 2 * ((uint64_t)region * out.hsh.region_cap + at);
                h[0] = make_uint4((uint32_t)p, fl, a0, a1);
                h[1] = make_uint4(b0, b1, 0u, 0u);
            }
        }
    }

    if (valid && !heavy) {
        // kWalk entries loaded at a time: the walk waits on memory once per
        // kWalk entries, not once per entry
        for (uint32_t t = rg.a0; t < rg.a1; t += kWalk) {
            unsigned long long w[kWalk];
#pragma unroll
            for (uint32_t u = 0; u < kWalk; u++) w[u] = t + u < rg.a1 ? rg.srcA[t + u] : 0ull;
#pragma unroll
            for (uint32_t u = 0; u < kWalk; u++)
                if (t + u < rg.a1)
                    visit(w[u], p, s, has_prev, prev, lh, N, avail, kSub && rg.strictA, sg);
        }
        gu64 *srcB = kSub ? rg.srcB : rg.srcA;
        for (uint32_t t = rg.b0; t < rg.b1; t++)
            visit(srcB[t], p, s, has_prev, prev, lh, N, avail, false, sg);
    }
    return valid ? len : 0u;  // entries read for this lane's (position, strand)
}

// The context of the q-gram at forward position u on strand s, from the
// 64-bit window X of the packed reference that starts at base u - 5 - t0
// (the q-gram's first base is base t0 + 5 of X): the letter before the
// q-gram on that strand (0 when there is none), whether there is one, how
// many letters follow it (up to 4) and those letters, first letter in the
// top bits, missing ones 0.  Strand 1 reads the forward text backwards and
// complemented: T1[p-1] = comp(R[u+q]), T1[p+q+i] = comp(R[u-1-i]).
__device__ __forceinline__ void refq_context(uint64_t X, int t0, uint64_t L, int q, uint64_t u,
                                             uint32_t s, uint32_t &has, uint32_t &prev,
                                             uint32_t &N, uint32_t &avail) {
    const uint64_t after = L - u - q;  // forward letters after the q-gram
    if (!s) {
        has = u >= 1;
        prev = base_rel(X, t0 + 4);
        N = (uint32_t)((X << (2 * (t0 + 5 + q))) >> 56);
        avail = after < 4 ? (uint32_t)after : 4u;
    } else {
        has = after >= 1;
        prev = 3u - base_rel(X, t0 + 5 + q);
        const uint32_t F = (uint32_t)((X << (2 * t0)) >> 54) & 0xffu;  // R[u-4..u-1]
        N = (((F & 3u) << 6) | (((F >> 2) & 3u) << 4) | (((F >> 4) & 3u) << 2) | (F >> 6)) ^ 0xffu;
        avail = u < 4 ? (uint32_t)u : 4u;
    }
    if (!has) prev = 0;
    N &= (0xffu << (8 - 2 * avail)) & 0xffu;
}

// P's keys, one per forward position u: strand 0 at u, strand 1 at L-q-u;
// key = ((p << 1 | strand) << (2q + 2a)) | (q-gram << 2a) | the first a
// letters after the q-gram (a = refq_sort_letters), so that sorting the low
// 2q + 2a bits orders P by q-gram and then by the letters that follow
__global__ __launch_bounds__(256) void k_refq_keys(PnRefDev ref, int q, int a,
                                                   unsigned long long *__restrict__ keys) {
    const uint64_t L = ref.L;
    const uint64_t npos = L - q + 1;
    const uint64_t u0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kPPT;
    if (u0 >= npos) return;
    const uint64_t X = window32(ref.packed, (int64_t)u0 - 5);
    const int sh = 2 * q + 2 * a;
    for (int jj = 0; jj < kPPT && u0 + jj < npos; jj++) {
        const uint64_t u = u0 + jj;
        const uint32_t g0 = (uint32_t)((X << (2 * (jj + 5))) >> (64 - 2 * q));
        uint32_t has, prev, N0, N1, avail;
        refq_context(X, jj, L, q, u, 0u, has, prev, N0, avail);
        refq_context(X, jj, L, q, u, 1u, has, prev, N1, avail);
        keys[u] = ((unsigned long long)(u << 1) << sh) | ((unsigned long long)g0 << (2 * a)) |
                  (N0 >> (8 - 2 * a));
        keys[npos + u] = ((unsigned long long)(((L - q - u) << 1) | 1u) << sh) |
                         ((unsigned long long)pn_revcomp_code(g0, q) << (2 * a)) |
                         (N1 >> (8 - 2 * a));
    }
}

// context of a sorted entry: letter before the q-gram (bits 0-1), whether
// there is one (bit 2), letters after it that exist, up to 4 (bits 3-5),
// and those letters (bits 6-13, first letter highest)
__global__ __launch_bounds__(256) void k_refq_ctx(PnRefDev ref, int q, int a,
                                                  unsigned long long *__restrict__ keys,
                                                  uint64_t n, uint16_t *__restrict__ ctx) {
    const uint64_t L = ref.L;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const unsigned long long key = keys[i];
        const unsigned long long ps = key >> (2 * q + 2 * a);
        const uint32_t g = (uint32_t)((key >> (2 * a)) & ((1ull << (2 * q)) - 1ull));
        const uint64_t p = ps >> 1;
        const uint32_t s = (uint32_t)(ps & 1u);
        const uint64_t u = s ? L - q - p : p;  // forward position of the q-gram
        const uint64_t X = window32(ref.packed, (int64_t)u - 5);
        uint32_t has, prev, N, avail;
        refq_context(X, 0, L, q, u, s, has, prev, N, avail);
        if (ctx) {
            keys[i] = (ps << (2 * q)) | g;
            ctx[i] = (uint16_t)(prev | (has << 2) | (avail << 3) | (N << 6));
        } else {
            keys[i] = (ps << (2 * q + 10)) | ((unsigned long long)N << (2 * q + 2)) |
                      ((unsigned long long)prev << (2 * q)) | g;
        }
    }
}

// Repeat masking (Section 3.2 leaves exceedingly frequent q-grams out of
// P): bit g of `bits` is set when q-gram g has more than max_occ entries in
// P, i.e. occurrences on the two strands together.  P is ordered by q-gram,
// so these form one run; its first entry finds the run's end by binary
// search.
__global__ __launch_bounds__(256) void k_mask_runs(pn::RefQDev P, int q, uint32_t max_occ,
                                                   uint32_t *__restrict__ bits) {
    const uint64_t gmask = (1ull << (2 * q)) - 1ull;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += stride) {
        const uint64_t g = P.keys[i] & gmask;
        if (i > 0 && (P.keys[i - 1] & gmask) == g) continue;
        uint64_t lo = i + 1, hi = P.n;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if ((P.keys[mid] & gmask) <= g)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo - i > (uint64_t)max_occ) atomicOr(&bits[g >> 5], 1u << (uint32_t)(g & 31));
    }
}

// (compiled for 7 waves per SIMD: more waves hide more of the walk's load
// latency than the few registers this spills cost; 8 waves spill more than
// they gain, 6 need no spill but hide less)
template <typename TW, bool kPacked, bool kSub>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(7))) void k_filter(
    PnRefDev ref, pn::RefQDev P, PnIndexDev ix, pn::Lists ls, pn::FilterOut out) {
    __shared__ uint2 wbuf[kWaves][kWBuf];
    __shared__ uint32_t wcnt[kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x < kWaves) wcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t shard = blockIdx.x % pn::kShards;
    Stage sg{(lds_u64 *)wbuf[wave], &wcnt[wave], out.cands, out.sh.counts, out.sh.region_cap,
             (blockIdx.x * kWaves + wave) % pn::kShards, 0u, 0ull, 0u, 0u, (uint32_t)kWBuf};
    const int q = ix.q;
    const uint32_t gmask = (uint32_t)((1ull << (2 * q)) - 1ull);
    unsigned long long seeds = 0, visited = 0, set_aside = 0;
    // the block takes kT * kPPT consecutive entries of P, a wave 64
    // consecutive ones per round; every lane runs the same rounds so that
    // long slices can be shared by the wave
    const uint64_t i0 = (uint64_t)blockIdx.x * (kT * kPPT) + threadIdx.x;
    // the next entry of P is loaded while this one is probed and walked
    unsigned long long key_next = i0 < P.n ? P.keys[i0] : 0ull;
    uint32_t c_next = !kPacked && i0 < P.n ? P.ctx[i0] : 0u;
    for (int jj = 0; jj < kPPT; jj++) {
        const uint64_t i = i0 + (uint64_t)jj * kT;
        bool valid = i < P.n;
        const unsigned long long key = key_next;
        const uint32_t c = c_next;
        if (jj + 1 < kPPT) {
            const uint64_t in = i + kT;
            key_next = in < P.n ? P.keys[in] : 0ull;
            if (!kPacked) c_next = in < P.n ? P.ctx[in] : 0u;
        }
        const uint32_t g = (uint32_t)key & gmask;
        const unsigned long long ps = key >> (kPacked ? 2 * q + 10 : 2 * q);
        const int64_t p = (int64_t)(ps >> 1);
        const uint32_t s = (uint32_t)(ps & 1u);
        bool has;
        uint32_t prev, avail, N;
        if (kPacked) {
            has = p >= 1;
            prev = (uint32_t)(key >> (2 * q)) & 3u;
            N = (uint32_t)(key >> (2 * q + 2)) & 0xffu;
            const uint64_t after = ref.L - (uint64_t)q - (uint64_t)p;
            avail = after < 4 ? (uint32_t)after : 4u;
        } else {
            has = (c >> 2) & 1u;
            prev = c & 3u;
            avail = (c >> 3) & 7u;
            N = (c >> 6) & 0xffu;
        }
        if (P.mask) {
            // a masked q-gram emits nothing; rule 1 may drop a pair only
            // when the pair to its left is not masked
            if ((P.mask[g >> 5] >> (g & 31)) & 1u) valid = false;
            const uint32_t gl = (prev << (2 * (q - 1))) | (g >> 2);
            if ((P.mask[gl >> 5] >> (gl & 31)) & 1u) has = false;
        }
        const bool lh = has && pn_low_complexity((prev << (2 * (q - 1))) | (g >> 2), q);
        Ranges r;
        if (valid) {
            seeds += probe<TW, kSub>(ix, ls, g, has, prev, N, avail, r);
        } else {
            r.srcA = r.srcB = (gu64 *)ix.O;
            r.idA = r.idB = 0;
            r.strictA = false;
            r.a0 = r.a1 = r.b0 = r.b1 = 0;
        }
        visited += visit_all<kSub>(r, p, s, has, prev, lh, N, avail, valid, sg, out, set_aside);
        // the wave is converged here: empty the stage before it can overflow
        if (*sg.cnt >= kWBuf / 2) flush(sg, lane);
    }
    pad_lane(sg);
    flush(sg, lane);
    unsigned long long written = sg.written;
    for (int o = 32; o > 0; o >>= 1) {
        seeds += __shfl_xor(seeds, o);
        visited += __shfl_xor(visited, o);
        set_aside += __shfl_xor(set_aside, o);
        written += __shfl_xor(written, o);
    }
    unsigned long long *stats = out.stats + 4 * shard;
    if (lane == 0 && seeds) atomicAdd(stats, seeds);
    if (lane == 0 && visited) atomicAdd(stats + 1, visited);
    if (lane == 0 && set_aside) atomicAdd(stats + 2, set_aside);
    if (lane == 0 && written) atomicAdd(stats + 3, written);
}

// The ranges set aside by k_filter, each wave an even share of its region's
// items, 64 of them at a time: each lane
// loads one item, a wave-wide prefix sum lays their entries end to end, and
// the wave walks that sequence 64 entries per step, four steps' loads first
// (an item is mostly a few dozen entries: one item per wave left most lanes
// idle).  Lane e of a step finds its item from the count of items that start
// at or before the step's first entry (a ballot) plus the starts inside the
// step before it (a 64-bit mask built with one LDS atomic OR per start).
// The same rules, the same staging; a step adds at most 64 candidates, so
// flushing once 64 or fewer slots are free keeps the stage from
// overflowing.
__global__ __launch_bounds__(kT) void k_filter_heavy(PnIndexDev ix, pn::Lists ls,
                                                     pn::FilterOut out) {
    extern __shared__ uint2 wbuf_dyn[];  // kWaves stages of `cap` entries
    const uint32_t cap = ix.after_sorted ? kWBufHeavyOrdered : kWBufHeavy;
    __shared__ uint32_t wcnt[kWaves];
    __shared__ uint4 s_item[kWaves][64][2];
    __shared__ uint32_t s_pre[kWaves][64];
    __shared__ unsigned long long s_mask[kWaves][4];
    __shared__ uint8_t s_owner[kWaves][256];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x < kWaves) wcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t gw = blockIdx.x * kWaves + wave;  // this wave in the grid
    const uint32_t nw = gridDim.x * kWaves;
    Stage sg{(lds_u64 *)(wbuf_dyn + (uint64_t)wave * cap), &wcnt[wave], out.cands, out.sh.counts, out.sh.region_cap,
             gw % pn::kShards, 0u, 0ull, 0u, 0u, cap};
    // candidates in the wave's stage (wave-uniform: every lane takes part in
    // each stage_put, so the stage never needs the LDS counter)
    uint32_t staged = 0;
    const uint32_t region = gw % pn::kShards;
    const uint64_t n = min((uint64_t)out.hsh.counts[region], out.hsh.region_cap);
    const uint4 *items = out.heavy + 2 * (uint64_t)region * out.hsh.region_cap;
    // the region's items split evenly over its waves, 64 at a time
    const uint64_t wpr = nw / pn::kShards;
    const uint64_t chunk = (n + wpr - 1) / wpr;
    const uint64_t i_lo = (uint64_t)(gw / pn::kShards) * chunk;
    const uint64_t i_hi = min(n, i_lo + chunk);
    for (uint64_t ib = i_lo; ib < i_hi; ib += 64) {
        // this lane's item and the wave's exclusive prefix of their sizes
        const uint64_t my = ib + (uint64_t)lane;
        uint4 h0 = make_uint4(0u, 0u, 0u, 0u), h1 = h0;
        if (my < i_hi) {
            h0 = items[2 * my];
            h1 = items[2 * my + 1];
        }
        const uint32_t size = my < i_hi ? (h0.w - h0.z) + (h1.y - h1.x) : 0u;
        // long items: walked one at a time by the whole wave, as they fill
        // its lanes anyway
        unsigned long long longs = __ballot(size >= kLongItem);
        while (longs) {
            const int j = __ffsll((long long)longs) - 1;
            longs &= longs - 1;
            const uint4 a0 = make_uint4(__shfl(h0.x, j), __shfl(h0.y, j), __shfl(h0.z, j),
                                        __shfl(h0.w, j));
            const uint32_t b0 = __shfl(h1.x, j), b1 = __shfl(h1.y, j);
            const uint32_t fl = a0.y;
            const int64_t p = (int64_t)(((uint64_t)(fl >> 22) << 32) | a0.x);
            const uint32_t idA = (fl >> 17) & 3u, idB = (fl >> 19) & 3u;
            gu64 *srcA = idA == 1u ? (gu64 *)ls.side : (gu64 *)ix.O;
            gu64 *srcB = idB == 1u ? (gu64 *)ls.side : idB == 2u ? (gu64 *)ls.laxO : (gu64 *)ix.O;
            const bool strictA = (fl >> 21) & 1u;
            const bool has = fl & 1u, lh = (fl >> 1) & 1u;
            const uint32_t prev = (fl >> 2) & 3u, avail = (fl >> 4) & 7u, N = (fl >> 8) & 0xffu;
            const uint32_t s = (fl >> 16) & 1u;
            const uint32_t la = a0.w - a0.z, total = la + (b1 - b0);
            for (uint32_t base = 0; base < total; base += 256) {
                unsigned long long v[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t k = base + 64 * u + (uint32_t)lane;
                    v[u] = k < total ? (k < la ? srcA[a0.z + k] : srcB[b0 + (k - la)]) : 0ull;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t k = base + 64 * u + (uint32_t)lane;
                    uint2 c = make_uint2(0u, 0u);
                    const bool e = k < total &&
                                   visit_cand(v[u], p, s, has, prev, lh, N, avail,
                                              strictA && k < la, c);
                    stage_put(sg, staged, e, c, lane);
                    if (staged > cap - 64) flush_n(sg, lane, staged);
                }
            }
        }
        // the short ones laid end to end
        const uint32_t tot = size < kLongItem ? size : 0u;
        uint32_t incl = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        const uint32_t start = incl - tot;
        const uint32_t total = __shfl(incl, 63);
        if (total == 0) continue;
        s_item[wave][lane][0] = h0;
        s_item[wave][lane][1] = h1;
        s_pre[wave][lane] = start;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t base = 0; base < total; base += 256) {
            // for each of the four steps: which items start inside it
            if (lane < 4) s_mask[wave][lane] = 0ull;
            __builtin_amdgcn_wave_barrier();
            if (tot > 0 && start > base && start < base + 256) {
                const uint32_t rel = start - base;
                atomicOr(&s_mask[wave][rel >> 6], 1ull << (rel & 63));
                s_owner[wave][rel] = (uint8_t)lane;
            }
            __builtin_amdgcn_wave_barrier();
            unsigned long long v[4];
            uint32_t px[4], pf[4];
            bool st[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t t0 = base + 64u * (uint32_t)u;
                const uint32_t e = t0 + (uint32_t)lane;
                // the item of entry e: the last (non-empty) item starting at
                // or before it; the one holding t0 is the highest lane whose
                // item starts at or before t0, later starts inside the step
                // are marked in the mask with their lanes in s_owner
                const unsigned long long at0 = __ballot(tot > 0 && start <= t0);
                const uint32_t j0 = 63u - (uint32_t)__clzll(at0 | 1ull);
                const unsigned long long mm =
                    s_mask[wave][u] & ((2ull << lane) - 1ull) & ~1ull;
                const uint32_t j =
                    mm ? (uint32_t)s_owner[wave][64u * (uint32_t)u +
                                                 (63u - (uint32_t)__clzll(mm))]
                       : j0;
                v[u] = 0ull;
                px[u] = pf[u] = 0u;
                st[u] = false;
                if (e < total) {
                    const uint4 a0 = s_item[wave][j][0], a1 = s_item[wave][j][1];
                    const uint32_t k = e - s_pre[wave][j];
                    const uint32_t la = a0.w - a0.z;
                    const uint32_t fl = a0.y;
                    const uint32_t idA = (fl >> 17) & 3u, idB = (fl >> 19) & 3u;
                    gu64 *srcA = idA == 1u ? (gu64 *)ls.side : (gu64 *)ix.O;
                    gu64 *srcB = idB == 1u ? (gu64 *)ls.side
                                 : idB == 2u ? (gu64 *)ls.laxO
                                             : (gu64 *)ix.O;
                    v[u] = k < la ? srcA[a0.z + k] : srcB[a1.x + (k - la)];
                    px[u] = a0.x;
                    pf[u] = fl;
                    st[u] = ((fl >> 21) & 1u) && k < la;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t e = base + 64u * (uint32_t)u + (uint32_t)lane;
                uint2 c = make_uint2(0u, 0u);
                bool got = false;
                if (e < total) {
                    const uint32_t fl = pf[u];
                    const int64_t p = (int64_t)(((uint64_t)(fl >> 22) << 32) | px[u]);
                    const bool has = fl & 1u, lh = (fl >> 1) & 1u;
                    const uint32_t prev = (fl >> 2) & 3u, avail = (fl >> 4) & 7u,
                                   N = (fl >> 8) & 0xffu;
                    const uint32_t s = (fl >> 16) & 1u;
                    got = visit_cand(v[u], p, s, has, prev, lh, N, avail, st[u], c);
                }
                stage_put(sg, staged, got, c, lane);
                if (staged > cap - 64) flush_n(sg, lane, staged);
            }
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
    }
    flush_n(sg, lane, staged);
}

// ---------------------------------------------------------------------------
// map-time per-read rules

__device__ __forceinline__ uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// status bit 2: some k_r > PN_MAX_K; bit 4: some read violates (k_r+1) q <= n_r;
// bit 16 (no error): some k_r > PN_BAND_K (the 64-bit band pass is needed)
__global__ void k_read_rules(PnIndexDev ix, int kglob, const uint8_t *__restrict__ kpr,
                             uint8_t *__restrict__ rinfo, uint16_t *__restrict__ rstamp,
                             uint32_t *status, int plain) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < ix.n_reads) {
        const uint64_t off = ix.offsets[r];
        const uint32_t n = (uint32_t)(ix.offsets[r + 1] - off);
        const uint32_t k = kglob >= 0 ? (uint32_t)kglob : kpr[r];
        const uint32_t q = (uint32_t)ix.q;
        uint32_t bad = 0;
        if (k > PN_MAX_K) bad |= 2u;
        if ((k + 1) * q > n) bad |= 4u;
        // Piece mode (an index whose long slices are ordered with the piece
        // starts apart): the read's disjoint windows of q + 4 letters at
        // offsets 0, q + 4, 2 (q + 4), ...  An edit falls into one window at
        // most, so an alignment with at most k errors leaves a window
        // untouched when k + 1 of them can be looked up: an exact match of
        // the window's q-gram and the four letters after it, found by
        // filtration at its piece start.  Windows whose q-gram is
        // low-complexity are not looked up (rule 2) and do not count.
        uint32_t pieces = 0;
        if (!bad && !plain && ix.after_sorted) {
            const uint32_t ell = q + 4;
            for (uint32_t o = 0; o + ell <= n; o += ell)
                pieces += !pn_low_complexity(pn_window16(ix.packed, off + o) >> (32 - 2 * q), q);
        }
        if (!bad && k > PN_BAND_K) atomicOr(status, 16u);
        if (bad) {
            atomicOr(status, bad);
            rinfo[r] = 0;
        } else if (plain) {
            rinfo[r] = 0x80u;
        } else if (pieces >= k + 1) {
            // (its entries are in no lax list and no side list); bits 4-6:
            // windows starting below 16 times this lie in the read's first
            // half (their centre before the read's)
            const uint32_t half = (n - (q + 4)) / 2;
            rinfo[r] = (uint8_t)((1u << 3) | (min((half + 15) / 16, 7u) << 4) | 4u);
        } else {
            const uint32_t nq = n - q + 1;
            const uint32_t lc = ix.lcinfo[r] & 0xffffu, runs = (ix.lcinfo[r] >> 16) & 0x7fffu;
            const uint32_t front = ix.lcinfo[r] >> 31;
            const uint32_t Q = nq - lc;  // offsets whose q-gram is not low-complexity
            uint32_t keep, run;
            if (Q >= k * q + 1) {
                keep = 0;
                run = q - 1 + ceil_div(Q - k * q, k + 1 + runs);
            } else {
                keep = 1;
                run = ceil_div(n - k, k + 1);
            }
            const uint32_t need = run > q ? min(run - q, 4u) : 0u;
            rinfo[r] = (uint8_t)((keep << 7) | (front << 6) | need);
        }
        // the word stamped into the read's O entries: the rule byte and the
        // read's length - 1 (filtration hands it on in the candidate)
        if (rstamp) rstamp[r] = (uint16_t)(rinfo[r] | (((n - 1u) & 0xffu) << 8));
    }
}

// side lists: for each of the 16 low-complexity q-grams (first two letters
// x, y; then x y x y ...), the occurrences from reads that keep them, grouped
// by the letter before the q-gram (class 0..4).  Three kernels over all 16
// slices of O laid end to end: counts per (q-gram, class), the class bounds
// (side_cls[id*6 + c] = start of class c, side_cls[id*6 + 5] = end, inside
// the host-computed region of q-gram id), then the entries, each block
// reserving its slots once per (q-gram, class).  Order inside a class group
// is free.

// the 16 slices [ks, ks + len) and their prefix, in LDS
template <typename TW>
__device__ __forceinline__ void lc_slices(const PnIndexDev &ix, uint32_t *s_ks, uint32_t *s_pre) {
    __shared__ uint32_t s_len[pn::kLcPatterns];
    if (threadIdx.x < pn::kLcPatterns) {
        const uint32_t id = threadIdx.x;
        const uint32_t x = id >> 2, y = id & 3u;
        uint32_t g = 0;
        for (int t = 0; t < ix.q; t++) g = (g << 2) | ((t & 1) ? y : x);
        const TW *I = (const TW *)ix.I;
        const uint32_t wmask = (1u << ix.log2w) - 1;
        const uint32_t gi = g >> ix.log2w, gj = g & wmask;
        const TW word = I[gi];
        uint32_t ks = 0, ke = 0;
        if ((word >> gj) & 1) {
            const uint32_t slot =
                pn_group_start<TW>(ix, I, gi) + (uint32_t)pn_popc<TW>(word & (((TW)1 << gj) - 1));
            ks = ix.Sp[slot];
            ke = ix.Sp[slot + 1];
        }
        s_ks[id] = ks;
        s_len[id] = ke - ks;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int id = 0; id < pn::kLcPatterns; id++) {
            s_pre[id] = a;
            a += s_len[id];
        }
        s_pre[pn::kLcPatterns] = a;
    }
    __syncthreads();
}

// item t of the slices laid end to end: (q-gram id, O entry); cls = 8 when
// the entry's read does not keep its low-complexity seeds
__device__ __forceinline__ uint32_t lc_item(const PnIndexDev &ix, const uint8_t *rinfo,
                                            const uint32_t *s_ks, const uint32_t *s_pre,
                                            uint32_t t, unsigned long long &v, uint32_t &cls) {
    uint32_t id = 0;
    while (id + 1 < pn::kLcPatterns && s_pre[id + 1] <= t) id++;
    v = ix.O[s_ks[id] + (t - s_pre[id])];
    const uint32_t r = (uint32_t)(v >> 40) & (PN_MAX_READS - 1);
    cls = ((rinfo[r] >> 7) & 1u) ? (uint32_t)(v >> 61) : 8u;
    return id;
}

template <typename TW>
__global__ __launch_bounds__(256) void k_lc_count(PnIndexDev ix, const uint8_t *__restrict__ rinfo,
                                                  uint32_t *counts) {
    __shared__ uint32_t s_ks[pn::kLcPatterns], s_pre[pn::kLcPatterns + 1];
    __shared__ uint32_t h[5 * pn::kLcPatterns];
    lc_slices<TW>(ix, s_ks, s_pre);
    if (threadIdx.x < 5 * pn::kLcPatterns) h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t total = s_pre[pn::kLcPatterns];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        unsigned long long v;
        uint32_t cls;
        const uint32_t id = lc_item(ix, rinfo, s_ks, s_pre, t, v, cls);
        if (cls <= PN_CLS_NONE) atomicAdd(&h[id * 5 + cls], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 5 * pn::kLcPatterns && h[threadIdx.x])
        atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_lc_bounds(const uint32_t *region, const uint32_t *counts, uint32_t *side_cls,
                            uint32_t *cursors) {
    const uint32_t id = threadIdx.x;
    if (id >= pn::kLcPatterns) return;
    uint32_t at = region[id];
    for (uint32_t c = 0; c <= PN_CLS_NONE; c++) {
        side_cls[id * 6 + c] = at;
        cursors[id * 5 + c] = at;
        at += counts[id * 5 + c];
    }
    side_cls[id * 6 + 5] = at;
}

// each block takes one contiguous chunk of items: counts them, reserves
// its slots once per (q-gram, class), then places them
template <typename TW>
__global__ __launch_bounds__(256) void k_lc_scatter(PnIndexDev ix, const uint8_t *__restrict__ rinfo,
                                                    unsigned long long *side, uint32_t *cursors) {
    __shared__ uint32_t s_ks[pn::kLcPatterns], s_pre[pn::kLcPatterns + 1];
    __shared__ uint32_t h[5 * pn::kLcPatterns], base[5 * pn::kLcPatterns];
    lc_slices<TW>(ix, s_ks, s_pre);
    if (threadIdx.x < 5 * pn::kLcPatterns) h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t total = s_pre[pn::kLcPatterns];
    const uint32_t chunk = (total + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = min(total, blockIdx.x * chunk), t1 = min(total, t0 + chunk);
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        unsigned long long v;
        uint32_t cls;
        const uint32_t id = lc_item(ix, rinfo, s_ks, s_pre, t, v, cls);
        if (cls <= PN_CLS_NONE) atomicAdd(&h[id * 5 + cls], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 5 * pn::kLcPatterns) {
        const uint32_t n = h[threadIdx.x];
        base[threadIdx.x] = n ? atomicAdd(&cursors[threadIdx.x], n) : 0u;
        h[threadIdx.x] = 0;
    }
    __syncthreads();
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        unsigned long long v;
        uint32_t cls;
        const uint32_t id = lc_item(ix, rinfo, s_ks, s_pre, t, v, cls);
        if (cls <= PN_CLS_NONE) {
            const uint32_t k = id * 5 + cls;
            side[base[k] + atomicAdd(&h[k], 1u)] = v;
        }
    }
}

// copy each read's rule bits (keep flag << 7 | required extra run) into the
// low byte of its O entries, so that the filter reads them with the entry
__device__ __forceinline__ unsigned long long stamp(unsigned long long v,
                                                    const uint16_t *__restrict__ rstamp) {
    return (v & ~0xffffull) | rstamp[(uint32_t)(v >> 40) & (PN_MAX_READS - 1)];
}

// One pass per thread: kStampPer pairs of entries loaded (16 bytes each,
// coalesced across the wave), then their reads' rule bytes gathered, then
// the stores, so that no load waits behind a store of the same wave (O is
// 16-byte aligned)
constexpr int kStampPer = 8;

__global__ __launch_bounds__(256) void k_stamp_rules(unsigned long long *O, uint64_t n,
                                                     const uint16_t *__restrict__ rinfo) {
    ulonglong2 *O2 = (ulonglong2 *)O;
    const uint64_t n2 = n / 2;
    const uint64_t base = (uint64_t)blockIdx.x * (256 * kStampPer) + threadIdx.x;
    ulonglong2 v[kStampPer];
#pragma unroll
    for (int j = 0; j < kStampPer; j++) {
        const uint64_t i = base + (uint64_t)j * 256;
        v[j] = i < n2 ? O2[i] : make_ulonglong2(0ull, 0ull);
    }
#pragma unroll
    for (int j = 0; j < kStampPer; j++) {
        v[j].x = stamp(v[j].x, rinfo);
        v[j].y = stamp(v[j].y, rinfo);
    }
#pragma unroll
    for (int j = 0; j < kStampPer; j++) {
        const uint64_t i = base + (uint64_t)j * 256;
        if (i < n2) O2[i] = v[j];
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) O[n - 1] = stamp(O[n - 1], rinfo);
}

// occurrence counts of the 16 low-complexity q-grams (sizes of their O slices)
template <typename TW>
__global__ void k_lc_sizes(PnIndexDev ix, uint32_t *sizes) {
    const uint32_t id = threadIdx.x;
    if (id >= pn::kLcPatterns) return;
    const uint32_t x = id >> 2, y = id & 3u;
    uint32_t g = 0;
    for (int t = 0; t < ix.q; t++) g = (g << 2) | ((t & 1) ? y : x);
    const TW *I = (const TW *)ix.I;
    const uint32_t wmask = (1u << ix.log2w) - 1;
    const uint32_t gi = g >> ix.log2w, gj = g & wmask;
    const TW word = I[gi];
    uint32_t m = 0;
    if ((word >> gj) & 1) {
        const uint32_t slot =
            pn_group_start<TW>(ix, I, gi) + (uint32_t)pn_popc<TW>(word & (((TW)1 << gj) - 1));
        m = ix.Sp[slot + 1] - ix.Sp[slot];
    }
    sizes[id] = m;
}

// Lax lists (per mapping call, after the rule bytes are stamped): for every
// slice of O longer than min_len, its entries whose read is not in piece
// mode (the searched ranges hold piece starts only), in slice order,
// appended to laxO;
// lax[x] = {start, count} for such a slot x (other slots are not written).
// A lane looks at one slot; the wave then takes the long slots one by one,
// counts their lax entries with ballots, reserves room with one atomic add
// and writes them.
__global__ __launch_bounds__(kT) void k_lax_lists(PnIndexDev ix, uint64_t n_slots,
                                                  uint32_t min_len, uint2 *__restrict__ lax,
                                                  unsigned long long *__restrict__ laxO,
                                                  unsigned long long *count) {
    const uint32_t lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint64_t gw = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    gu64 *O = (gu64 *)ix.O;
    for (uint64_t base = gw * 64; base < n_slots; base += nw * 64) {
        const uint64_t x = base + lane;
        const uint32_t ks = x < n_slots ? ix.Sp[x] : 0u;
        const uint32_t ke = x < n_slots ? ix.Sp[x + 1] : 0u;
        unsigned long long todo = __ballot(ke - ks > min_len);
        while (todo) {
            const int l = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const uint32_t a = __shfl(ks, l), b = __shfl(ke, l);
            uint32_t n = 0;
            for (uint32_t t = a; t < b; t += 64) {
                const bool f = t + lane < b && !(((uint32_t)O[t + lane] >> 3) & 1u);
                n += (uint32_t)__popcll(__ballot(f));
            }
            unsigned long long at = 0;
            if (lane == 0 && n) at = atomicAdd(count, (unsigned long long)n);
            at = __shfl(at, 0);
            uint32_t w = 0;
            for (uint32_t t = a; t < b && w < n; t += 64) {
                const unsigned long long v = t + lane < b ? O[t + lane] : 0ull;
                const bool f = t + lane < b && !(((uint32_t)v >> 3) & 1u);
                const unsigned long long m = __ballot(f);
                if (f) laxO[at + w + (uint32_t)__popcll(m & lt)] = v;
                w += (uint32_t)__popcll(m);
            }
            if (lane == (uint32_t)l) lax[x] = make_uint2((uint32_t)at, n);
        }
    }
}

}  // namespace

namespace pn {

void launch_lc_sizes(const PnIndexDev &ix, uint32_t *sizes, hipStream_t st) {
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_lc_sizes<unsigned long long>, dim3(1), dim3(64), 0, st, ix, sizes);
    else
        hipLaunchKernelGGL(k_lc_sizes<uint32_t>, dim3(1), dim3(64), 0, st, ix, sizes);
}


void launch_read_rules(const PnIndexDev &ix, int kglob, const uint8_t *kpr, uint8_t *rinfo,
                       uint16_t *rstamp, uint32_t *status, bool plain, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_rules, dim3((ix.n_reads + 255) / 256), dim3(256), 0, st, ix, kglob,
                       kpr, rinfo, rstamp, status, plain ? 1 : 0);
}

void launch_mask_runs(const RefQDev &P, int q, uint32_t max_occ, uint32_t *bits, hipStream_t st) {
    if (!P.n) return;
    hipLaunchKernelGGL(k_mask_runs, dim3(pn_stride_blocks(P.n, 256)), dim3(256), 0, st, P, q,
                       max_occ, bits);
}

void launch_lc_side(const PnIndexDev &ix, const uint8_t *rinfo, unsigned long long *side,
                    const uint32_t *region, uint32_t *side_cls, uint32_t *scratch,
                    hipStream_t st) {
    uint32_t *counts = scratch, *cursors = scratch + 5 * kLcPatterns;
    launch_fill_u32(counts, 5 * kLcPatterns, 0u, st);
    const dim3 grid(1024), block(256);
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_lc_count<unsigned long long>, grid, block, 0, st, ix, rinfo, counts);
    else
        hipLaunchKernelGGL(k_lc_count<uint32_t>, grid, block, 0, st, ix, rinfo, counts);
    hipLaunchKernelGGL(k_lc_bounds, dim3(1), dim3(64), 0, st, region, (const uint32_t *)counts,
                       side_cls, cursors);
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_lc_scatter<unsigned long long>, grid, block, 0, st, ix, rinfo, side,
                           cursors);
    else
        hipLaunchKernelGGL(k_lc_scatter<uint32_t>, grid, block, 0, st, ix, rinfo, side, cursors);
}

void launch_stamp_rules(unsigned long long *O, uint64_t n, const uint16_t *rinfo, hipStream_t st) {
    if (!n) return;
    const uint64_t blocks = (n / 2 + 256 * kStampPer - 1) / (256 * kStampPer) + 1;
    hipLaunchKernelGGL(k_stamp_rules, dim3((unsigned)blocks), dim3(256), 0, st, O, n, rinfo);
}

void launch_refq_keys(const PnRefDev &ref, int q, unsigned long long *keys, hipStream_t st) {
    if (ref.L < (uint64_t)q) return;
    const uint64_t npos = ref.L - q + 1;
    const uint64_t threads = (npos + kPPT - 1) / kPPT;
    hipLaunchKernelGGL(k_refq_keys, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, ref,
                       q, refq_sort_letters(ref.L, q), keys);
}

void launch_refq_ctx(const PnRefDev &ref, int q, unsigned long long *keys, uint64_t n,
                     uint16_t *ctx, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_refq_ctx, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, ref, q,
                       refq_sort_letters(ref.L, q), keys, n, ctx);
}

template <typename TW, bool kPacked, bool kSub>
static void filter_variant(const PnRefDev &ref, const RefQDev &P, const PnIndexDev &ix,
                           const Lists &ls, FilterOut out, uint64_t nb, hipStream_t st) {
    hipLaunchKernelGGL((k_filter<TW, kPacked, kSub>), dim3((unsigned)nb), dim3(kT), 0, st, ref, P,
                       ix, ls, out);
}

template <typename TW>
static void filter_variant_tw(const PnRefDev &ref, const RefQDev &P, const PnIndexDev &ix,
                              const Lists &ls, FilterOut out, uint64_t nb, hipStream_t st) {
    const bool packed = P.ctx == nullptr;
    if (packed && ls.sub_on) filter_variant<TW, true, true>(ref, P, ix, ls, out, nb, st);
    else if (packed) filter_variant<TW, true, false>(ref, P, ix, ls, out, nb, st);
    else if (ls.sub_on) filter_variant<TW, false, true>(ref, P, ix, ls, out, nb, st);
    else filter_variant<TW, false, false>(ref, P, ix, ls, out, nb, st);
}

void launch_filter(const PnRefDev &ref, const RefQDev &P, const PnIndexDev &ix, const Lists &ls,
                   FilterOut out, hipStream_t st) {
    const uint64_t nb = (P.n + kFilterBlockPos - 1) / kFilterBlockPos;
    if (!nb || !ix.n_reads) return;
    if (ix.log2w == 6) filter_variant_tw<unsigned long long>(ref, P, ix, ls, out, nb, st);
    else filter_variant_tw<uint32_t>(ref, P, ix, ls, out, nb, st);
}

void launch_filter_heavy(const PnIndexDev &ix, const Lists &ls, FilterOut out, hipStream_t st) {
    if (!ix.n_reads) return;
    const size_t lds = (size_t)kWaves * (ix.after_sorted ? kWBufHeavyOrdered : kWBufHeavy) *
                       sizeof(uint2);
    hipLaunchKernelGGL(k_filter_heavy, dim3(128 * pn::kShards), dim3(kT), lds, st, ix, ls, out);
}

void launch_lax_lists(const PnIndexDev &ix, uint64_t n_slots, uint32_t min_len, uint2 *lax,
                      unsigned long long *laxO, unsigned long long *count, hipStream_t st) {
    if (!n_slots || !ix.n_reads) return;
    const uint64_t waves = (n_slots + 63) / 64;
    const unsigned blocks = (unsigned)std::min<uint64_t>((waves + kWaves - 1) / kWaves, 8192);
    hipLaunchKernelGGL(k_lax_lists, dim3(blocks), dim3(kT), 0, st, ix, n_slots, min_len, lax, laxO,
                       count);
}

}  // namespace pn
