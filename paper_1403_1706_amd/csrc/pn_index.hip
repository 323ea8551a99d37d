// Algorithm 1: building the q-group index (I, S, S', O) of the read batch
// on the device (Section 2.2).  The paper fills O through per-q-gram
// counters and "next free entry" cursors; here the same arrays come from
// one sort, which needs no atomic per occurrence and leaves every slice of
// O ordered:
//   a. one 64-bit key per q-gram occurrence (read r, offset o):
//      (r, o) above (q-gram g, class of the letter before it)   (k_qgram_keys)
//   b. stable LSD radix sort on the low 2q+3 bits: occurrences grouped by
//      g, inside a group by (class, r, o)                         (pn_canon.hip)
//   c. O[i] from the i-th key; the first key of each g sets bit g of I
//      (Algorithm 1 step 1) and marks a group start               (k_index_from_sorted)
//   d. S = exclusive scan of popcount(I[i]) (steps 2-3); the rank of each
//      group start among the starts is its slot x = S[g/w] + GROUPRANK, so
//      S'[x] = its position in O (steps 4-6)                     (pn_scan.hip, k_sp_fill)
// Each O entry also carries the letter before its q-gram and the (up to)
// four letters after it, which the filter compares with the reference
// without touching the reads.
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

// q-gram starts per read (n_r - q + 1, or 0)
__global__ void k_read_nq(PnIndexDev ix, uint32_t *nq) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ix.n_reads) return;
    const uint64_t n = ix.offsets[r + 1] - ix.offsets[r];
    nq[r] = n >= (uint64_t)ix.q ? (uint32_t)(n - ix.q + 1) : 0u;
}

// key of occurrence (r, o): ((r << 8 | o) << (2q + 3)) | (g << 3) | class
__global__ __launch_bounds__(256) void k_qgram_keys(PnIndexDev ix, uint32_t nch,
                                                    const uint32_t *__restrict__ qoff,
                                                    unsigned long long *__restrict__ keys) {
    QgramIter it;
    if (!qgram_iter(ix, nch, it)) return;
    const int sh = 2 * ix.q + 3;
    const uint64_t base = qoff[it.r];
    for (uint32_t o = it.o0; o < it.o1; o++) {
        uint32_t cls;
        const uint32_t g = qgram_at(ix, it.off, o, cls);
        keys[base + o] = ((unsigned long long)((it.r << 8) | o) << sh) |
                         ((unsigned long long)g << 3) | cls;
    }
}

// O entries from the sorted keys, group starts, and the presence bitmap I
template <typename TW>
__global__ __launch_bounds__(256) void k_index_from_sorted(PnIndexDev ix,
                                                           const unsigned long long *__restrict__ keys,
                                                           uint64_t T, unsigned long long *O,
                                                           uint32_t *flags, TW *I) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    const int sh = 2 * ix.q + 3;
    const unsigned long long lowm = (1ull << sh) - 1ull;
    const unsigned long long k = keys[i];
    const uint32_t g = (uint32_t)((k & lowm) >> 3);
    const uint32_t cls = (uint32_t)(k & 7ull);
    const uint32_t ro = (uint32_t)(k >> sh);
    const uint32_t r = ro >> 8, o = ro & 0xffu;
    const bool start = i == 0 || (uint32_t)((keys[i - 1] & lowm) >> 3) != g;
    flags[i] = start;
    if (start) {
        const uint32_t wmask = (1u << ix.log2w) - 1;
        atomicOr(&I[g >> ix.log2w], (TW)1 << (g & wmask));
    }
    // the letters after the q-gram inside the read (at most four)
    const uint64_t off = ix.offsets[r];
    const uint32_t n = (uint32_t)(ix.offsets[r + 1] - off);
    const uint32_t after = n - o - (uint32_t)ix.q;
    const uint32_t nav = after < 4u ? after : 4u;
    uint32_t next4 = pn_window16(ix.packed, off + o + ix.q) >> 24;
    next4 &= (0xffu << (8 - 2 * nav)) & 0xffu;
    const uint32_t hi = (cls << 29) | (r << 8) | o;
    const uint32_t lo = (next4 << 24) | (nav << 21);
    O[i] = ((unsigned long long)hi << 32) | lo;
}

// S'[x] = position of the x-th group start; S'[D] = T
__global__ void k_sp_fill(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                          uint64_t T, uint32_t *Sp) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T && flags[i]) Sp[pos[i]] = (uint32_t)i;
    if (i == T) Sp[pos[T]] = (uint32_t)T;
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

void launch_read_nq(const PnIndexDev &ix, uint32_t *nq, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_nq, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, nq);
}

void launch_qgram_keys(const PnIndexDev &ix, const uint32_t *qoff, unsigned long long *keys,
                       hipStream_t st) {
    const uint32_t nch = nch_for(ix);
    uint64_t n = (uint64_t)ix.n_reads * nch;
    if (!n) return;
    hipLaunchKernelGGL(k_qgram_keys, dim3(grid_for(n, 256)), dim3(256), 0, st, ix, nch, qoff, keys);
}

void launch_index_from_sorted(const PnIndexDev &ix, const unsigned long long *keys, uint64_t T,
                              unsigned long long *O, uint32_t *flags, void *I, hipStream_t st) {
    if (!T) return;
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_index_from_sorted<unsigned long long>, dim3(grid_for(T, 256)),
                           dim3(256), 0, st, ix, keys, T, O, flags, (unsigned long long *)I);
    else
        hipLaunchKernelGGL(k_index_from_sorted<uint32_t>, dim3(grid_for(T, 256)), dim3(256), 0, st,
                           ix, keys, T, O, flags, (uint32_t *)I);
}

void launch_sp_fill(const uint32_t *flags, const uint32_t *pos, uint64_t T, uint32_t *Sp,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_sp_fill, dim3(grid_for(T + 1, 256)), dim3(256), 0, st, flags, pos, T, Sp);
}

void launch_read_lc(const PnIndexDev &ix, uint32_t *lcinfo, hipStream_t st) {
    if (!ix.n_reads) return;
    hipLaunchKernelGGL(k_read_lc, dim3(grid_for(ix.n_reads, 256)), dim3(256), 0, st, ix, lcinfo);
}

}  // namespace pn
