// Algorithm 1: building the q-group index (I, S, S', O) of the read batch
// on the device (Section 2.2).  One thread handles up to 32 consecutive
// q-gram starts of one read; reads are independent, so the six steps are
//   1. I[g / w] |= bit (g mod w)              (k_qgram_bitmap)
//   2-3. S = exclusive scan of popcount(I[i])  (pn_scan.hip)
//   4. count[S[i] + j'] += 1, j' = GROUPRANK   (k_qgram_count)
//   5. S' = exclusive scan of count            (pn_scan.hip)
//   6. O[S'[x] + next free] = position         (k_qgram_scatter)
// followed by ordering each q-gram's slice of O by entry value (small slices
// fully, long slices by preceding letter).  Each O entry also carries the
// letter before its q-gram and the (up to) four letters after it, which the
// filter compares with the reference without touching the reads.
#include "pn_internal.h"

namespace {

constexpr int kChunk = 32;  // q-gram starts per thread

struct QgramIter {
    uint32_t r;
    uint64_t off;
    uint32_t n;       // read length
    uint32_t o0, o1;  // q-gram starts [o0, o1)
};

__device__ __forceinline__ bool qgram_iter(const PnIndexDev &ix, uint32_t nch, QgramIter &it) {
    uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    it.r = (uint32_t)(gid / nch);
    uint32_t c = (uint32_t)(gid % nch);
    if (it.r >= ix.n_reads) return false;
    it.off = ix.offsets[it.r];
    uint64_t n = ix.offsets[it.r + 1] - it.off;
    it.n = (uint32_t)n;
    if (n < (uint64_t)ix.q) return false;
    uint32_t nq = (uint32_t)(n - ix.q + 1);
    it.o0 = c * kChunk;
    it.o1 = min(it.o0 + kChunk, nq);
    return it.o0 < it.o1;
}

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

template <typename TW>
__global__ __launch_bounds__(256) void k_qgram_bitmap(PnIndexDev ix, uint32_t nch, TW *I) {
    QgramIter it;
    if (!qgram_iter(ix, nch, it)) return;
    const uint32_t wmask = (1u << ix.log2w) - 1;
    for (uint32_t o = it.o0; o < it.o1; o++) {
        uint32_t cls;
        uint32_t g = qgram_at(ix, it.off, o, cls);
        TW bit = (TW)1 << (g & wmask);
        TW *p = &I[g >> ix.log2w];
        if (!(*p & bit)) atomicOr(p, bit);
    }
}

template <typename TW>
__device__ __forceinline__ uint32_t group_rank_slot(const PnIndexDev &ix, const TW *I, uint32_t g) {
    const uint32_t wmask = (1u << ix.log2w) - 1;
    uint32_t i = g >> ix.log2w, j = g & wmask;
    TW word = I[i];
    uint32_t jp = (uint32_t)pn_popc<TW>(word & (((TW)1 << j) - 1));  // GROUPRANK
    return ix.S[i] + jp;
}

template <typename TW>
__global__ __launch_bounds__(256) void k_qgram_count(PnIndexDev ix, uint32_t nch, uint32_t *cnt) {
    QgramIter it;
    if (!qgram_iter(ix, nch, it)) return;
    const TW *I = (const TW *)ix.I;
    for (uint32_t o = it.o0; o < it.o1; o++) {
        uint32_t cls;
        uint32_t g = qgram_at(ix, it.off, o, cls);
        atomicAdd(&cnt[group_rank_slot<TW>(ix, I, g)], 1u);
    }
}

template <typename TW>
__global__ __launch_bounds__(256) void k_qgram_scatter(PnIndexDev ix, uint32_t nch,
                                                       uint32_t *cursor, unsigned long long *O) {
    QgramIter it;
    if (!qgram_iter(ix, nch, it)) return;
    const TW *I = (const TW *)ix.I;
    for (uint32_t o = it.o0; o < it.o1; o++) {
        uint32_t cls;
        uint32_t g = qgram_at(ix, it.off, o, cls);
        uint32_t x = group_rank_slot<TW>(ix, I, g);
        uint32_t k = ix.Sp[x] + atomicAdd(&cursor[x], 1u);
        // the letters after the q-gram inside the read (at most four)
        const uint32_t after = it.n - o - (uint32_t)ix.q;
        const uint32_t nav = after < 4u ? after : 4u;
        uint32_t next4 = pn_window16(ix.packed, it.off + o + ix.q) >> 24;
        next4 &= (0xffu << (8 - 2 * nav)) & 0xffu;
        const uint32_t hi = (cls << 29) | (it.r << 8) | o;
        const uint32_t lo = (next4 << 24) | (nav << 21);
        O[k] = ((unsigned long long)hi << 32) | lo;
    }
}

// per read: number of low-complexity q-gram offsets and of maximal runs of
// such offsets (both used by the map-time seed rules)
__global__ __launch_bounds__(256) void k_read_lc(PnIndexDev ix, uint32_t *lcinfo) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ix.n_reads) return;
    const uint64_t off = ix.offsets[r];
    const uint64_t n = ix.offsets[r + 1] - off;
    uint32_t cnt = 0, runs = 0;
    bool prev_lc = false;
    for (uint64_t o = 0; o + (uint64_t)ix.q <= n; o++) {
        const uint32_t g = pn_window16(ix.packed, off + o) >> (32 - 2 * ix.q);
        const bool lc = pn_low_complexity(g, ix.q);
        cnt += lc;
        runs += lc && !prev_lc;
        prev_lc = lc;
    }
    lcinfo[r] = cnt | (runs << 16);
}

// order small slices of O in place; slices longer than 32 go to a list
__global__ __launch_bounds__(256) void k_bucket_sort(const uint32_t *Sp, uint64_t n_slots,
                                                     const uint32_t *n_distinct,
                                                     unsigned long long *O, uint32_t *big_list,
                                                     uint32_t *big_count) {
    uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_slots || x >= *n_distinct) return;
    uint32_t s = Sp[x], e = Sp[x + 1];
    uint32_t m = e - s;
    if (m <= 1) return;
    if (m > 32) {
        big_list[atomicAdd(big_count, 1u)] = (uint32_t)x;
        return;
    }
    for (uint32_t i = s + 1; i < e; i++) {
        unsigned long long v = O[i];
        uint32_t j = i;
        while (j > s && O[j - 1] > v) {
            O[j] = O[j - 1];
            j--;
        }
        O[j] = v;
    }
}

// one block per long slice: stable partition by preceding-letter class
// (the top three bits of an entry) through a scratch copy
__global__ __launch_bounds__(256) void k_bucket_sort_big(const uint32_t *Sp,
                                                         unsigned long long *O,
                                                         unsigned long long *tmp,
                                                         const uint32_t *big_list) {
    uint32_t x = big_list[blockIdx.x];
    uint32_t s = Sp[x], e = Sp[x + 1];
    uint32_t at = s;
    for (uint32_t cls = 0; cls <= PN_CLS_NONE; cls++) {
        for (uint32_t base = s; base < e; base += 256) {
            uint32_t i = base + threadIdx.x;
            unsigned long long v = i < e ? O[i] : 0ull;
            uint32_t f = (i < e) && ((uint32_t)(v >> 61) == cls);
            uint32_t tot;
            uint32_t ex = pn_block_excl_scan(f, &tot);
            if (f) tmp[at + ex] = v;
            at += tot;
        }
    }
    __syncthreads();
    for (uint32_t i = s + threadIdx.x; i < e; i += 256) O[i] = tmp[i];
}

inline unsigned grid_for(uint64_t n, unsigned threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// chunks of kChunk q-gram starts per read, from the longest read
uint32_t nch_for(const PnIndexDev &ix) {
    uint32_t nq = ix.max_len >= (uint32_t)ix.q ? ix.max_len - ix.q + 1 : 1;
    return (nq + kChunk - 1) / kChunk;
}

}  // namespace

namespace pn {

void launch_qgram_bitmap(const PnIndexDev &ix, void *I, hipStream_t st) {
    const uint32_t nch = nch_for(ix);
    uint64_t n = (uint64_t)ix.n_reads * nch;
    if (!n) return;
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_qgram_bitmap<unsigned long long>, dim3(grid_for(n, 256)), dim3(256),
                           0, st, ix, nch, (unsigned long long *)I);
    else
        hipLaunchKernelGGL(k_qgram_bitmap<uint32_t>, dim3(grid_for(n, 256)), dim3(256), 0, st, ix,
                           nch, (uint32_t *)I);
}

void launch_qgram_count(const PnIndexDev &ix, uint32_t *cnt, hipStream_t st) {
    const uint32_t nch = nch_for(ix);
    uint64_t n = (uint64_t)ix.n_reads * nch;
    if (!n) return;
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_qgram_count<unsigned long long>, dim3(grid_for(n, 256)), dim3(256), 0,
                           st, ix, nch, cnt);
    else
        hipLaunchKernelGGL(k_qgram_count<uint32_t>, dim3(grid_for(n, 256)), dim3(256), 0, st, ix,
                           nch, cnt);
}

void launch_qgram_scatter(const PnIndexDev &ix, uint32_t *cursor, unsigned long long *O,
                          hipStream_t st) {
    const uint32_t nch = nch_for(ix);
    uint64_t n = (uint64_t)ix.n_reads * nch;
    if (!n) return;
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_qgram_scatter<unsigned long long>, dim3(grid_for(n, 256)), dim3(256),
                           0, st, ix, nch, cursor, O);
    else
        hipLaunchKernelGGL(k_qgram_scatter<uint32_t>, dim3(grid_for(n, 256)), dim3(256), 0, st, ix,
                           nch, cursor, O);
}

void launch_bucket_sort(const uint32_t *Sp, uint64_t n_slots, const uint32_t *n_distinct,
                        unsigned long long *O, uint32_t *big_list, uint32_t *big_count,
                        hipStream_t st) {
    if (!n_slots) return;
    hipLaunchKernelGGL(k_bucket_sort, dim3(grid_for(n_slots, 256)), dim3(256), 0, st, Sp, n_slots,
                       n_distinct, O, big_list, big_count);
}

void launch_bucket_sort_big(const uint32_t *Sp, unsigned long long *O, unsigned long long *tmp,
                            const uint32_t *big_list, uint32_t n_big, hipStream_t st) {
    if (!n_big) return;
    hipLaunchKernelGGL(k_bucket_sort_big, dim3(n_big), dim3(256), 0, st, Sp, O, tmp, big_list);
}

void launch_read_lc(const PnIndexDev &ix, uint32_t *lcinfo, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_lc, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, lcinfo);
}

}  // namespace pn
