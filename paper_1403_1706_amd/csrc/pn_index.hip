// Algorithm 1: building the q-group index (I, S, S', O) of the read batch
// on the device (Section 2.2).  The paper fills O through per-q-gram
// counters and "next free entry" cursors; here the same arrays come from
// one sort, which needs no atomic per occurrence and leaves every slice of
// O ordered:
//   a. one 64-bit key per q-gram occurrence (read r, offset o): (r, o),
//      the class of the letter before the q-gram and the q-gram g (k_qgram_keys)
//   b. stable LSD radix sort on the 2q bits of g: occurrences grouped by g,
//      inside a group in the order (r, o)                          (pn_canon.hip)
//   c. O[i] from the i-th key; the first key of each g sets bit g of I
//      (Algorithm 1 step 1) and marks a group start               (k_index_from_sorted)
//   d. S = exclusive scan of popcount(I[i]) (steps 2-3); the rank of each
//      group start among the starts is its slot x = S[g/w] + GROUPRANK, so
//      S'[x] = its position in O (steps 4-6)                (pn_scan.hip, k_scan_down_sp)
// Each O entry also carries the letter before its q-gram and the (up to)
// four letters after it, which the filter compares with the reference
// without touching the reads.
#include "pn_internal.h"

namespace {

// q-gram code at read offset o (first base most significant) and the class
// of the letter before it (its code, or PN_CLS_NONE at o == 0)
__device__ __forceinline__ uint32_t qgram_at(const PnIndexDev &ix, uint64_t off, uint32_t o,
                                             uint32_t &cls) {
    if (o == 0) {
        cls = PN_CLS_NONE;
        return pn_window16(ix.packed, off) >> (32 - 2 * ix.q);
    }
    uint32_t w = pn_window16(ix.packed, off + o - 1);  // letter o-1 then the q-gram
    cls = w >> 30;
    return (w << 2) >> (32 - 2 * ix.q);
}

// q-gram starts per read (n_r - q + 1, or 0) and read lengths (<= 256)
__global__ void k_read_nq(PnIndexDev ix, uint32_t *nq, uint16_t *len) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ix.n_reads) return;
    const uint64_t n = ix.offsets[r + 1] - ix.offsets[r];
    nq[r] = n >= (uint64_t)ix.q ? (uint32_t)(n - ix.q + 1) : 0u;
    len[r] = (uint16_t)n;
}

// key of occurrence (r, o): ((r << 8 | o) << (2q + 3)) | (class << 2q) | g;
// with kCarry (q <= 12, where 8 bits are left) the four letters after the
// q-gram sit between (r, o) and the class: ((r << 8 | o) << (2q + 11)) |
// (next4 << (2q + 3)) | (class << 2q) | g.  Sorting looks at the low 2q
// bits (the q-gram) only, so each slice keeps the order (read, offset).  One wave per read: lane l takes offsets l, l + 64, ..., so a
// wave reads one stretch of the packed reads and writes one stretch of keys.
template <bool kCarry>
__global__ __launch_bounds__(256) void k_qgram_keys(PnIndexDev ix,
                                                    const uint32_t *__restrict__ qoff,
                                                    unsigned long long *__restrict__ keys) {
    const uint32_t r = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (r >= ix.n_reads) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t off = ix.offsets[r];
    const uint64_t n = ix.offsets[r + 1] - off;
    if (n < (uint64_t)ix.q) return;
    const uint32_t nq = (uint32_t)(n - ix.q + 1);
    const int sh = 2 * ix.q + 3;
    const uint64_t base = qoff[r];
    for (uint32_t o = lane; o < nq; o += 64) {
        uint32_t cls;
        const uint32_t g = qgram_at(ix, off, o, cls);
        unsigned long long key = ((unsigned long long)cls << (2 * ix.q)) | g;
        if (kCarry) {
            const uint32_t next4 = pn_window16(ix.packed, off + o + ix.q) >> 24;
            key |= ((unsigned long long)((r << 8) | o) << (sh + 8)) |
                   ((unsigned long long)next4 << sh);
        } else {
            key |= (unsigned long long)((r << 8) | o) << sh;
        }
        keys[base + o] = key;
    }
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
                                                           uint8_t *flags, TW *I,
                                                           const uint16_t *__restrict__ len) {
    const int sh = 2 * ix.q + 3;
    const int rsh = kCarry ? sh + 8 : sh;  // where (r << 8 | o) starts
    const unsigned long long gmask = (1ull << (2 * ix.q)) - 1ull;
    const uint64_t i0 = (uint64_t)blockIdx.x * (256 * kPer) + threadIdx.x;
    unsigned long long k[kPer], kl[kPer];
    uint64_t off[kPer], end[kPer];
    uint32_t w[kPer];
    // every load before the first store (a wave's loads wait for its earlier
    // stores): the keys, and for lane 0 the key before its own
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const uint64_t i = i0 + (uint64_t)j * 256;
        k[j] = i < T ? keys[i] : 0ull;
        kl[j] = (threadIdx.x & 63) == 0 && i && i <= T ? keys[i - 1] : ~0ull;
    }
    if (kCarry) {
        // the letters are in the key; only the read's length is looked up
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const uint32_t r = (uint32_t)(k[j] >> rsh) >> 8;
            const bool ok = i0 + (uint64_t)j * 256 < T;
            off[j] = 0;
            end[j] = ok ? len[r] : 0;
            w[j] = (uint32_t)((k[j] >> sh) & 0xffu) << 24;
        }
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
        const uint32_t g = (uint32_t)(k[j] & gmask);
        const uint32_t cls = (uint32_t)(k[j] >> (2 * ix.q)) & 7u;
        const uint32_t ro = (uint32_t)(k[j] >> rsh);
        const uint32_t r = ro >> 8, o = ro & 0xffu;
        // the previous entry's key: the lane before, or memory for lane 0
        unsigned long long kp = __shfl_up(k[j], 1);
        if ((threadIdx.x & 63) == 0) kp = kl[j];
        const bool start = i == 0 || (uint32_t)(kp & gmask) != g;
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
        const uint32_t n = (uint32_t)(end[j] - off[j]);
        const uint32_t after = n - o - (uint32_t)ix.q;
        const uint32_t nav = after < 4u ? after : 4u;
        uint32_t next4 = w[j] >> 24;
        next4 &= (0xffu << (8 - 2 * nav)) & 0xffu;
        const uint32_t hi = (cls << 29) | (r << 8) | o;
        const uint32_t lo = (next4 << 24) | (nav << 21);
        O[i] = ((unsigned long long)hi << 32) | lo;
    }
}

// S'[x] = position of the x-th group start; S'[D] = T

// per read: number of low-complexity q-gram offsets and of maximal runs of
// such offsets (both used by the map-time seed rules), and whether more of
// them lie in the first half of the offsets than in the second (bit 31: a
// hint for the direction of verification's first pass)
__global__ __launch_bounds__(256) void k_read_lc(PnIndexDev ix, uint32_t *lcinfo) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ix.n_reads) return;
    const uint64_t off = ix.offsets[r];
    const uint64_t n = ix.offsets[r + 1] - off;
    const uint64_t nq = n >= (uint64_t)ix.q ? n - ix.q + 1 : 0;
    uint32_t cnt = 0, runs = 0, front = 0;
    bool prev_lc = false;
    for (uint64_t o = 0; o < nq; o++) {
        const uint32_t g = pn_window16(ix.packed, off + o) >> (32 - 2 * ix.q);
        const bool lc = pn_low_complexity(g, ix.q);
        cnt += lc;
        front += lc && 2 * o < nq;
        runs += lc && !prev_lc;
        prev_lc = lc;
    }
    lcinfo[r] = cnt | (runs << 16) | ((2 * front > cnt ? 1u : 0u) << 31);
}

inline unsigned grid_for(uint64_t n, unsigned threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

namespace pn {

void launch_read_nq(const PnIndexDev &ix, uint32_t *nq, uint16_t *len, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_nq, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, nq, len);
}

void launch_qgram_keys(const PnIndexDev &ix, const uint32_t *qoff, unsigned long long *keys,
                       hipStream_t st) {
    if (!ix.n_reads) return;
    const uint64_t threads = (uint64_t)ix.n_reads * 64;  // a wave per read
    if (index_key_carries(ix.q))
        hipLaunchKernelGGL(k_qgram_keys<true>, dim3(grid_for(threads, 256)), dim3(256), 0, st, ix,
                           qoff, keys);
    else
        hipLaunchKernelGGL(k_qgram_keys<false>, dim3(grid_for(threads, 256)), dim3(256), 0, st, ix,
                           qoff, keys);
}

void launch_index_from_sorted(const PnIndexDev &ix, const unsigned long long *keys, uint64_t T,
                              unsigned long long *O, uint8_t *flags, void *I, const uint16_t *len,
                              hipStream_t st) {
    if (!T) return;
    const unsigned blocks = grid_for(T, 256 * kPer);
    const bool c = index_key_carries(ix.q);
    if (ix.log2w == 6 && c)
        hipLaunchKernelGGL((k_index_from_sorted<unsigned long long, true>), dim3(blocks), dim3(256),
                           0, st, ix, keys, T, O, flags, (unsigned long long *)I, len);
    else if (ix.log2w == 6)
        hipLaunchKernelGGL((k_index_from_sorted<unsigned long long, false>), dim3(blocks),
                           dim3(256), 0, st, ix, keys, T, O, flags, (unsigned long long *)I, len);
    else if (c)
        hipLaunchKernelGGL((k_index_from_sorted<uint32_t, true>), dim3(blocks), dim3(256), 0, st, ix,
                           keys, T, O, flags, (uint32_t *)I, len);
    else
        hipLaunchKernelGGL((k_index_from_sorted<uint32_t, false>), dim3(blocks), dim3(256), 0, st,
                           ix, keys, T, O, flags, (uint32_t *)I, len);
}


void launch_read_lc(const PnIndexDev &ix, uint32_t *lcinfo, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_lc, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, lcinfo);
}

}  // namespace pn
