// Algorithm 1: building the q-group index (I, S, S', O) of the read batch
// on the device (Section 2.2).  The paper fills O through per-q-gram
// counters and "next free entry" cursors; here the same arrays come from
// one sort, which needs no atomic per occurrence and leaves every slice of
// O ordered:
//   a. one 64-bit key per q-gram occurrence (read r, offset o): (r, o),
//      the class of the letter before the q-gram, the q-gram g and (q <= 12)
//      the letters after it with their count, all that an O entry holds
//      (k_qgram_keys)
//   b. stable LSD radix sort on g: occurrences grouped by g, inside a group
//      in the order (r, o); when (q <= 12) many occurrences fall into long
//      slices, sorted again on g and the letters after it, which orders
//      each slice by those letters first                         (pn_canon.hip)
//   c. O[i] from the i-th key; the first key of each g sets bit g of I
//      (Algorithm 1 step 1) and marks a group start               (k_index_from_sorted)
//   d. S = exclusive scan of popcount(I[i]) (steps 2-3); the rank of each
//      group start among the starts is its slot x = S[g/w] + GROUPRANK, so
//      S'[x] = its position in O (steps 4-6)                (pn_scan.hip, k_scan_down_sp)
// Each O entry also carries the letter before its q-gram and the (up to)
// four letters after it, which the filter compares with the reference
// without touching the reads.
#include <algorithm>

#include "pn_internal.h"

namespace {

// The (up to) four letters after a q-gram inside its read (first letter in
// the top bits, missing letters 0) and how many there are, nav = 0..4, in 9
// bits: nav = 4 takes the codes 0-255, nav = 3 the next 64, nav = 2 the next
// 16, nav = 1 the next 4 and nav = 0 the code 340.
__device__ __forceinline__ uint32_t after_code(uint32_t next4, uint32_t nav) {
    switch (nav) {
        case 4: return next4;
        case 3: return 256u + (next4 >> 2);
        case 2: return 320u + (next4 >> 4);
        case 1: return 336u + (next4 >> 6);
        default: return 340u;
    }
}
__device__ __forceinline__ void after_decode(uint32_t c, uint32_t &next4, uint32_t &nav) {
    if (c < 256u) {
        next4 = c;
        nav = 4;
    } else if (c < 320u) {
        next4 = (c - 256u) << 2;
        nav = 3;
    } else if (c < 336u) {
        next4 = (c - 320u) << 4;
        nav = 2;
    } else if (c < 340u) {
        next4 = (c - 336u) << 6;
        nav = 1;
    } else {
        next4 = 0;
        nav = 0;
    }
}

// q-gram starts per read (n_r - q + 1, or 0)
__global__ void k_read_nq(PnIndexDev ix, uint32_t *nq) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ix.n_reads) return;
    const uint64_t n = ix.offsets[r + 1] - ix.offsets[r];
    nq[r] = n >= (uint64_t)ix.q ? (uint32_t)(n - ix.q + 1) : 0u;
}

// Key of occurrence (r, o): ((r << 8 | o) << (2q + 3)) | (class << 2q) | g;
// with kCarry (q <= 12) the key holds all an O entry needs:
// ((r << 8 | o) << (2q + 11)) | (letter before << (2q + 9)) | (g << 9) |
// after_code(next4, nav), the letter before being "none" exactly at o = 0.
// Sorting looks at the q-gram's bits, so each slice keeps the order (read,
// offset); with kCarry an index may be sorted again by the low 2q + 9 bits
// (the q-gram, then the letters after it), ordering each slice by those
// letters first.
// The keys of a read's q-gram occurrences, at the read's offset in the key
// array (see the header).  A wave takes reads gw, gw + nw, ...; lane l
// holds word l of the read's packed text (a read touches at most 18 words),
// and every window a key needs is put together from two lanes' words, so a
// read costs one coalesced load, issued one read ahead of its use.
// for each tile of `tile` keys, the read its first key belongs to (a thread
// per read: the tiles whose first key lies in the read's key range)
__global__ void k_tile_first_read(const uint32_t *__restrict__ qoff, uint32_t n_reads,
                                  uint64_t tile, uint32_t *first_read) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_reads) return;
    const uint64_t a = qoff[r], e = qoff[r + 1];
    for (uint64_t t = (a + tile - 1) / tile; t * tile < e; t++) first_read[t] = r;
}

// The keys of the q-gram occurrences, a block per tile of `tile` keys
// (the radix sort's tiles): the block writes keys [b * tile, (b+1) * tile)
// and counts their lowest 8 bits, the first digit of the sort, so that the
// sort's first pass needs no histogram pass of its own (hist0[b][d]).  Wave
// w takes the block's reads first + w, first + w + 4, ...; lane l holds word
// l of a read's packed text (a read touches at most 18 words), and every
// window a key needs is put together from two lanes' words, so a read costs
// one coalesced load, issued one read ahead of its use.  A read that
// straddles two tiles is taken by both blocks, each writing its own part.
template <bool kCarry>
__global__ __launch_bounds__(256) void k_qgram_keys(PnIndexDev ix,
                                                    const uint32_t *__restrict__ qoff,
                                                    const uint32_t *__restrict__ first_read,
                                                    uint64_t T, uint64_t tile,
                                                    unsigned long long *__restrict__ keys,
                                                    uint32_t *__restrict__ hist0) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t K0 = (uint64_t)blockIdx.x * tile, K1 = min(T, K0 + tile);
    const uint32_t first = first_read[blockIdx.x];
    const int q = ix.q;
    const int sh = 2 * q + 3;
    struct Read {
        uint64_t off, n, base;
        uint32_t word;  // this lane's word of the read's packed text
    };
    // a read whose keys start before K1 (else n = 0 and base = K1)
    auto fetch = [&](uint32_t r) {
        Read d{0, 0, K1, 0u};
        if (r < ix.n_reads) {
            d.base = qoff[r];
            if (d.base < K1) {
                d.off = ix.offsets[r];
                d.n = ix.offsets[r + 1] - d.off;
                const uint32_t words = (uint32_t)(((d.off & 15) + d.n + 15) >> 4) + 1;
                if (lane < words) d.word = ix.packed[(d.off >> 4) + lane];
            }
        }
        return d;
    };
    Read cur = fetch(first + wave);
    for (uint32_t r = first + wave; cur.base < K1; r += 4) {
        const Read nxt = fetch(r + 4);
        if (cur.n >= (uint64_t)q) {
            const uint32_t nq = (uint32_t)(cur.n - q + 1);
            const uint64_t w0 = cur.off >> 4;
            // 16 letters starting at letter t of the text, first in the top bits
            auto window = [&](uint64_t t) {
                const int wi = (int)((t >> 4) - w0);
                const uint32_t hi = (uint32_t)__shfl((int)cur.word, wi);
                const uint32_t lo = (uint32_t)__shfl((int)cur.word, wi + 1);
                const uint32_t s2 = 2 * (uint32_t)(t & 15);
                return s2 ? (hi << s2) | (lo >> (32 - s2)) : hi;
            };
            for (uint32_t o0 = 0; o0 < nq; o0 += 64) {
                const uint32_t o = o0 + lane;
                // every lane takes part in the shuffles; lanes outside the
                // read or the tile store nothing
                const uint32_t wq = window(cur.off + (o ? o - 1 : 0));
                const uint32_t w4 = window(cur.off + o + q);
                uint32_t cls, g;
                if (q == 16) {
                    // the q-gram fills a whole 16-letter window
                    g = window(cur.off + o);
                    cls = o == 0 ? PN_CLS_NONE : wq >> 30;
                } else if (o == 0) {
                    cls = PN_CLS_NONE;
                    g = wq >> (32 - 2 * q);
                } else {
                    cls = wq >> 30;
                    g = (wq << 2) >> (32 - 2 * q);
                }
                unsigned long long key;
                if (kCarry) {
                    // the letter before as 2 bits (none exactly when o = 0)
                    // and the letters after with their count as 9
                    const uint32_t after = o < nq ? nq - 1 - o : 0u;  // n - q - o
                    const uint32_t nav = after < 4u ? after : 4u;
                    const uint32_t next4 = (w4 >> 24) & ((0xffu << (8 - 2 * nav)) & 0xffu);
                    key = ((unsigned long long)((r << 8) | o) << (2 * q + 11)) |
                          ((unsigned long long)(cls & 3u) << (2 * q + 9)) |
                          ((unsigned long long)g << 9) | after_code(next4, nav);
                } else {
                    key = ((unsigned long long)((r << 8) | o) << sh) |
                          ((unsigned long long)cls << (2 * q)) | g;
                }
                const uint64_t pos = cur.base + o;
                if (o < nq && pos >= K0 && pos < K1) {
                    // streamed out (read back only by the sort's first scatter)
                    __builtin_nontemporal_store(key, &keys[pos]);
                    // the first digit the sort looks at: the q-gram's low 8 bits
                    atomicAdd(&h[(uint32_t)(key >> (kCarry ? 9 : 0)) & 255u], 1u);
                }
            }
        }
        cur = nxt;
    }
    __syncthreads();
    hist0[(uint64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// O entries from the sorted keys, group starts, and the presence bitmap I.
// Each thread takes kPer entries, 256 apart, and issues the gathers of all
// of them (read bounds, then the letters after each q-gram) before using
// any, so that their latencies overlap.
constexpr int kPer = 4;

template <typename TW, bool kCarry>
__global__ __launch_bounds__(256) void k_index_from_sorted(PnIndexDev ix,
                                                           const unsigned long long *__restrict__ keys,
                                                           uint64_t T, unsigned long long *O,
                                                           uint8_t *flags, TW *I) {
    const int rsh = kCarry ? 2 * ix.q + 11 : 2 * ix.q + 3;  // where (r << 8 | o) starts
    const int gsh = kCarry ? 9 : 0;                            // where the q-gram starts
    const unsigned long long gmask = (1ull << (2 * ix.q)) - 1ull;
    const uint64_t i0 = (uint64_t)blockIdx.x * (256 * kPer) + threadIdx.x;
    unsigned long long k[kPer], kl[kPer];
    uint64_t off[kPer], end[kPer];
    uint32_t w[kPer], code[kPer];
    // every load before the first store (a wave's loads wait for its earlier
    // stores): the keys, and for lane 0 the key before its own
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const uint64_t i = i0 + (uint64_t)j * 256;
        k[j] = i < T ? keys[i] : 0ull;
        kl[j] = (threadIdx.x & 63) == 0 && i && i <= T ? keys[i - 1] : ~0ull;
    }
    if (kCarry) {
        // the letters after the q-gram and their count are in the key
#pragma unroll
        for (int j = 0; j < kPer; j++) code[j] = (uint32_t)k[j] & 511u;
    } else {
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const uint32_t r = (uint32_t)(k[j] >> rsh) >> 8;
            const bool ok = i0 + (uint64_t)j * 256 < T;
            off[j] = ok ? ix.offsets[r] : 0;
            end[j] = ok ? ix.offsets[r + 1] : 0;
        }
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const uint32_t o = (uint32_t)(k[j] >> rsh) & 0xffu;
            const bool ok = i0 + (uint64_t)j * 256 < T;
            w[j] = ok ? pn_window16(ix.packed, off[j] + o + ix.q) : 0u;
        }
    }
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const uint64_t i = i0 + (uint64_t)j * 256;
        if (i0 + (uint64_t)j * 256 - (threadIdx.x & 63) >= T) break;  // the whole wave is past T
        const bool live = i < T;
        const uint32_t g = (uint32_t)((k[j] >> gsh) & gmask);
        const uint32_t ro = (uint32_t)(k[j] >> rsh);
        const uint32_t r = ro >> 8, o = ro & 0xffu;
        const uint32_t cls = kCarry ? (o == 0 ? (uint32_t)PN_CLS_NONE
                                              : (uint32_t)(k[j] >> (2 * ix.q + 9)) & 3u)
                                    : (uint32_t)(k[j] >> (2 * ix.q)) & 7u;
        // the previous entry's key: the lane before, or memory for lane 0
        unsigned long long kp = __shfl_up(k[j], 1);
        if ((threadIdx.x & 63) == 0) kp = kl[j];
        const bool start = i == 0 || (uint32_t)((kp >> gsh) & gmask) != g;
        if (live) flags[i] = start;
        // I: lanes holding one word of I are contiguous (keys are sorted);
        // their bits are ORed across the run and the run's last lane alone
        // writes them (one atomic per word and wave, not one per q-gram)
        const uint32_t wmask = (1u << ix.log2w) - 1;
        const uint32_t word = g >> ix.log2w;
        TW bits = live && start ? (TW)1 << (g & wmask) : (TW)0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t ow = __shfl_up(word, d);
            const TW ob = (TW)__shfl_up((unsigned long long)bits, d);
            if ((int)(threadIdx.x & 63) >= d && ow == word) bits |= ob;
        }
        const uint32_t nw = __shfl_down(word, 1);
        const bool last = (threadIdx.x & 63) == 63 || nw != word ||
                          i + 1 >= T;  // lanes past T do not take part
        if (last && bits) atomicOr(&I[word], bits);
        if (!live) continue;
        // the letters after the q-gram inside the read (at most four)
        uint32_t next4, nav;
        if (kCarry) {
            after_decode(code[j], next4, nav);
        } else {
            const uint32_t n = (uint32_t)(end[j] - off[j]);
            const uint32_t after = n - o - (uint32_t)ix.q;
            nav = after < 4u ? after : 4u;
            next4 = (w[j] >> 24) & ((0xffu << (8 - 2 * nav)) & 0xffu);
        }
        // a piece start: the read offset is a multiple of q + 4 and the four
        // letters after the q-gram lie in the read (the q-gram and those
        // letters form one of the read's disjoint pieces of q + 4 letters)
        const uint32_t piece = nav == 4u && o % (uint32_t)(ix.q + 4) == 0u;
        const uint32_t hi = (cls << 29) | (r << 8) | o;
        const uint32_t lo = (next4 << 24) | (nav << 21) | (piece << 20);
        O[i] = ((unsigned long long)hi << 32) | lo;
    }
}

// S'[x] = position of the x-th group start; S'[D] = T

// 256-bit vectors (PN_READ_WORDS words, bit b of word m = position 32m+b)
struct Bits256 {
    uint32_t w[PN_READ_WORDS];
};
// v >> s (towards position 0), 0 < s < 32
__device__ __forceinline__ Bits256 bits_down(const Bits256 &v, int s) {
    Bits256 o;
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++)
        o.w[m] = (v.w[m] >> s) | (m + 1 < PN_READ_WORDS ? v.w[m + 1] << (32 - s) : 0u);
    return o;
}
__device__ __forceinline__ void bits_and(Bits256 &a, const Bits256 &b) {
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) a.w[m] &= b.w[m];
}
// bits [0, n) set
__device__ __forceinline__ Bits256 bits_prefix(int n) {
    Bits256 o;
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) {
        const int k = n - 32 * m;
        o.w[m] = k >= 32 ? 0xffffffffu : k > 0 ? (1u << k) - 1u : 0u;
    }
    return o;
}

// Per read: number of low-complexity q-gram offsets and of maximal runs of
// such offsets (both used by the map-time seed rules), and whether more of
// them lie in the first half of the offsets than in the second (bit 31: a
// hint for the direction of verification's first pass).  Bit-parallel over
// the read's planes: E[i] = (letter i == letter i+2); the q-gram at offset o
// is low-complexity (period <= 2) exactly when E[o .. o+q-3] are all set.
__global__ __launch_bounds__(256) void k_read_lc(PnIndexDev ix, uint32_t *lcinfo) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ix.n_reads) return;
    const int n = (int)min(ix.offsets[r + 1] - ix.offsets[r], (uint64_t)PN_MAX_READ_LEN);
    const int q = ix.q;
    const int nq = n >= q ? n - q + 1 : 0;
    if (q < 3 || nq == 0) {
        lcinfo[r] = 0;
        return;
    }
    Bits256 H, L;
    const uint2 *rp = ix.rplanes + (uint64_t)r * PN_READ_WORDS;
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) {
        const uint2 v = rp[m];
        H.w[m] = v.x;
        L.w[m] = v.y;
    }
    const Bits256 H2 = bits_down(H, 2), L2 = bits_down(L, 2);
    Bits256 E = bits_prefix(n - 2);  // positions i with letter i+2 inside the read
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) E.w[m] &= ~(H.w[m] ^ H2.w[m]) & ~(L.w[m] ^ L2.w[m]);
    // C[o] = AND of E[o .. o+len-1] for len = q-2, built by doubling
    Bits256 C = E, X = E;  // X: runs of `span` ones
    int span = 1, have = 1;
    while (2 * span <= q - 2) {
        Bits256 Y = bits_down(X, span);
        bits_and(X, Y);
        span *= 2;
    }
    C = X;
    have = span;
    while (have < q - 2) {
        const int add = min(span, q - 2 - have);
        // runs of `add` ones from E, shifted to start `have` positions later
        Bits256 Z = E;
        for (int t = 1; t < add; t++) {
            Bits256 Y = bits_down(E, t);
            bits_and(Z, Y);
        }
        Bits256 Zs = bits_down(Z, have);
        bits_and(C, Zs);
        have += add;
    }
    const Bits256 inside = bits_prefix(nq);
    bits_and(C, inside);
    const Bits256 front_mask = bits_prefix((nq + 1) / 2);
    uint32_t cnt = 0, front = 0, runs = 0, carry = 0;
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) {
        cnt += __popc(C.w[m]);
        front += __popc(C.w[m] & front_mask.w[m]);
        runs += __popc(C.w[m] & ~((C.w[m] << 1) | carry));  // starts of runs
        carry = C.w[m] >> 31;
    }
    lcinfo[r] = cnt | (runs << 16) | ((2 * front > cnt ? 1u : 0u) << 31);
}

// occurrences in slices longer than min_len (*Dp slots)
__global__ __launch_bounds__(256) void k_long_entries(const uint32_t *__restrict__ Dp,
                                                      const uint32_t *__restrict__ Sp,
                                                      uint32_t min_len, unsigned long long *out) {
    const uint64_t D = *Dp;
    unsigned long long acc = 0;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < D;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t len = Sp[x + 1] - Sp[x];
        if (len > min_len) acc += len;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

// Slice tables of an ordered index.  Inside a slice the entries are
// ordered by v = 2 x (9-bit code of the letters after the q-gram) + piece
// start, so for a text position whose four next letters are N the entries
// filtration takes lie at [lb(2N + 1), lb(2N + 2)), lb(t) = the first entry
// whose v is t or more.  For a slice longer than min_len the table holds
// lb(t) - (slice start) for t = 0 .. pn::kTabWidth - 1, two loads instead of
// a binary search over the slice.

__device__ __forceinline__ uint32_t order_value(unsigned long long v) {
    const uint32_t lo = (uint32_t)v;
    return 2u * after_code(lo >> 24, (lo >> 21) & 7u) + ((lo >> 20) & 1u);
}

// flags[x] = 1 for a slot whose slice is longer than min_len
__global__ void k_tab_flags(const uint32_t *__restrict__ Sp, uint64_t D, uint32_t min_len,
                            uint32_t *__restrict__ flags) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < D; x += stride)
        flags[x] = Sp[x + 1] - Sp[x] > min_len ? 1u : 0u;
}

// tab_id[x] = the table's number (num: exclusive scan of the flags) or ~0;
// list[number] = x
__global__ void k_tab_ids(const uint32_t *__restrict__ Sp, uint64_t D, uint32_t min_len,
                          const uint32_t *__restrict__ num, uint32_t *__restrict__ tab_id,
                          uint32_t *__restrict__ list) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < D; x += stride) {
        const bool lng = Sp[x + 1] - Sp[x] > min_len;
        tab_id[x] = lng ? num[x] : 0xffffffffu;
        if (lng) list[num[x]] = (uint32_t)x;
    }
}

// a block per table: counts of each v below kTabWidth, then their prefix
__global__ __launch_bounds__(256) void k_tab_fill(const unsigned long long *__restrict__ O,
                                                  const uint32_t *__restrict__ Sp,
                                                  const uint32_t *__restrict__ list,
                                                  uint32_t n_tabs, uint32_t *__restrict__ tabs) {
    constexpr uint32_t W = pn::kTabWidth;
    __shared__ uint32_t h[W + 1];
    for (uint32_t t = blockIdx.x; t < n_tabs; t += gridDim.x) {
        for (uint32_t b = threadIdx.x; b <= W; b += 256) h[b] = 0;
        __syncthreads();
        const uint32_t x = list[t];
        const uint32_t ks = Sp[x], ke = Sp[x + 1];
        for (uint32_t i = ks + threadIdx.x; i < ke; i += 256) {
            const uint32_t v = order_value(O[i]);
            if (v + 1 < W) atomicAdd(&h[v + 1], 1u);  // counted into lb(v + 1) onwards
        }
        __syncthreads();
        // inclusive prefix over h[0 .. W-1] by the first wave: h[t] = #(v < t)
        if (threadIdx.x < 64) {
            const uint32_t lane = threadIdx.x;
            constexpr uint32_t per = (W + 63) / 64;
            uint32_t sum = 0;
            for (uint32_t j = 0; j < per; j++) {
                const uint32_t b = lane * per + j;
                if (b < W) sum += h[b];
            }
            uint32_t incl = sum;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o);
                if ((int)lane >= o) incl += y;
            }
            uint32_t run = incl - sum;
            uint32_t *T = tabs + (uint64_t)t * W;
            for (uint32_t j = 0; j < per; j++) {
                const uint32_t b = lane * per + j;
                if (b < W) {
                    run += h[b];
                    T[b] = run;
                }
            }
        }
        __syncthreads();
    }
}

inline unsigned grid_for(uint64_t n, unsigned threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

namespace pn {

void launch_read_nq(const PnIndexDev &ix, uint32_t *nq, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_nq, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, nq);
}

void launch_qgram_keys(const PnIndexDev &ix, const uint32_t *qoff, uint64_t T, uint64_t tile,
                       uint32_t *first_read, unsigned long long *keys, uint32_t *hist0,
                       hipStream_t st) {
    if (!ix.n_reads || !T) return;
    const uint64_t tiles = (T + tile - 1) / tile;
    hipLaunchKernelGGL(k_tile_first_read, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, qoff,
                       ix.n_reads, tile, first_read);
    if (index_key_carries(ix.q))
        hipLaunchKernelGGL(k_qgram_keys<true>, dim3((unsigned)tiles), dim3(256), 0, st, ix, qoff,
                           (const uint32_t *)first_read, T, tile, keys, hist0);
    else
        hipLaunchKernelGGL(k_qgram_keys<false>, dim3((unsigned)tiles), dim3(256), 0, st, ix, qoff,
                           (const uint32_t *)first_read, T, tile, keys, hist0);
}

void launch_index_from_sorted(const PnIndexDev &ix, const unsigned long long *keys, uint64_t T,
                              unsigned long long *O, uint8_t *flags, void *I, hipStream_t st) {
    if (!T) return;
    const unsigned blocks = grid_for(T, 256 * kPer);
    const bool c = index_key_carries(ix.q);
    if (ix.log2w == 6 && c)
        hipLaunchKernelGGL((k_index_from_sorted<unsigned long long, true>), dim3(blocks), dim3(256),
                           0, st, ix, keys, T, O, flags, (unsigned long long *)I);
    else if (ix.log2w == 6)
        hipLaunchKernelGGL((k_index_from_sorted<unsigned long long, false>), dim3(blocks),
                           dim3(256), 0, st, ix, keys, T, O, flags, (unsigned long long *)I);
    else if (c)
        hipLaunchKernelGGL((k_index_from_sorted<uint32_t, true>), dim3(blocks), dim3(256), 0, st, ix,
                           keys, T, O, flags, (uint32_t *)I);
    else
        hipLaunchKernelGGL((k_index_from_sorted<uint32_t, false>), dim3(blocks), dim3(256), 0, st,
                           ix, keys, T, O, flags, (uint32_t *)I);
}


void launch_long_entries(const uint32_t *D, const uint32_t *Sp, uint32_t min_len,
                         unsigned long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_long_entries, dim3(1024), dim3(256), 0, st, D, Sp, min_len, out);
}

// the even entries of S (a sampled S): out[t] = S[2 t], t <= n_groups / 2
__global__ void k_sample_s(const uint32_t *__restrict__ S, uint64_t n_half,
                           uint32_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_half; t += stride)
        out[t] = S[2 * t];
}

void launch_sample_s(const uint32_t *S, uint64_t n_groups, uint32_t *out, hipStream_t st) {
    const uint64_t n_half = n_groups / 2 + 1;
    hipLaunchKernelGGL(k_sample_s, dim3(pn_stride_blocks(n_half, 256)), dim3(256), 0, st, S,
                       n_half, out);
}

void launch_tab_flags(const uint32_t *Sp, uint64_t D, uint32_t min_len, uint32_t *flags,
                      hipStream_t st) {
    if (!D) return;
    hipLaunchKernelGGL(k_tab_flags, dim3(pn_stride_blocks(D, 256)), dim3(256), 0, st, Sp, D,
                       min_len, flags);
}

void launch_tab_build(const unsigned long long *O, const uint32_t *Sp, uint64_t D,
                      uint32_t min_len, const uint32_t *num, uint32_t n_tabs, uint32_t *tab_id,
                      uint32_t *list, uint32_t *tabs, hipStream_t st) {
    if (!D) return;
    hipLaunchKernelGGL(k_tab_ids, dim3(pn_stride_blocks(D, 256)), dim3(256), 0, st, Sp, D,
                       min_len, num, tab_id, list);
    if (n_tabs)
        hipLaunchKernelGGL(k_tab_fill, dim3(std::min<uint32_t>(n_tabs, 65536u)), dim3(256), 0, st,
                           O, Sp, (const uint32_t *)list, n_tabs, tabs);
}

void launch_read_lc(const PnIndexDev &ix, uint32_t *lcinfo, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_lc, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, lcinfo);
}

}  // namespace pn
