// Algorithm 2: filtration of reference positions through the q-group index
// (Section 3.2).  Both strands come from one pass over the forward 2-bit
// text: the q-gram of strand 1 at position L-q-u is the reverse complement
// of the forward q-gram at u.  For each (position, strand) the occurrences
// of its q-gram are O[k_start .. k_end) (INDEXPAIR), each giving a candidate
// (read r, diagonal d = p - o).
//
// An occurrence pair (p, o) whose left neighbours are equal,
// T[p-1] == read[o-1], is not emitted: the pair (p-1, o-1) lies on the same
// diagonal and is found from position p-1, so the candidate set (read,
// strand, diagonal) is unchanged.  O slices are ordered by the class of the
// letter before each q-gram occurrence, so the skipped pairs form one
// contiguous sub-range [cl, ch) found by a short search.
//
// Two launches share the probe code: a count pass (per-block totals, the
// cumulative sum C of Algorithm 2) and an emit pass writing each block's
// candidates at its exclusive offset, so compaction needs no atomics.
#include "pn_internal.h"

namespace {

constexpr int kT = pn::kFilterThreads;
constexpr int kPPT = pn::kFilterPPT;

// 64 bits of packed reference starting at signed base position B (base B+t
// in bits 63-2t .. 62-2t); packed[-1] and 3 words past the end are readable
__device__ __forceinline__ uint64_t window32(const uint32_t *packed, int64_t B) {
    int64_t wi = B >> 4;
    uint32_t sh = (uint32_t)(B & 15);
    uint64_t hi = ((uint64_t)packed[wi] << 32) | packed[wi + 1];
    if (sh == 0) return hi;
    return (hi << (2 * sh)) | (packed[wi + 2] >> (32 - 2 * sh));
}

struct Probe {
    uint32_t ks, cl, ch, ke;  // survivors: [ks, cl) and [ch, ke)
};

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *O, uint32_t lo, uint32_t hi,
                                                    uint32_t key) {
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (O[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// INDEXPAIR(g) and the sub-range of occurrences preceded by letter `prev`
template <typename TW>
__device__ __forceinline__ Probe probe(const PnIndexDev &ix, uint32_t g, bool has_prev,
                                       uint32_t prev) {
    Probe pr{0, 0, 0, 0};
    const TW *I = (const TW *)ix.I;
    const uint32_t wmask = (1u << ix.log2w) - 1;
    uint32_t i = g >> ix.log2w, j = g & wmask;
    TW word = I[i];
    if (!((word >> j) & 1)) return pr;
    uint32_t jp = (uint32_t)pn_popc<TW>(word & (((TW)1 << j) - 1));  // GROUPRANK
    uint32_t x = ix.S[i] + jp;
    pr.ks = ix.Sp[x];
    pr.ke = ix.Sp[x + 1];
    pr.cl = pr.ch = pr.ke;
    if (!has_prev) return pr;
    const uint32_t key0 = prev << 29, key1 = (prev + 1) << 29;
    uint32_t m = pr.ke - pr.ks;
    if (m <= 8) {
        uint32_t below0 = 0, below1 = 0;
        for (uint32_t t = 0; t < m; t++) {
            uint32_t v = ix.O[pr.ks + t];
            below0 += v < key0;
            below1 += v < key1;
        }
        pr.cl = pr.ks + below0;
        pr.ch = pr.ks + below1;
    } else {
        pr.cl = lower_bound_u32(ix.O, pr.ks, pr.ke, key0);
        pr.ch = lower_bound_u32(ix.O, pr.cl, pr.ke, key1);
    }
    return pr;
}

// the two probes of forward position u (strand 0 at p = u, strand 1 at
// p = L-q-u); returns false past the last q-gram
struct PosQ {
    uint32_t g0, g1, prev0, prev1;
    bool has0, has1;
};

__device__ __forceinline__ bool pos_qgrams(const PnRefDev &ref, int q, uint64_t X, uint64_t u,
                                           int j, PosQ &pq) {
    if (u + q > ref.L) return false;
    pq.g0 = (uint32_t)((X << (2 * (j + 1))) >> (64 - 2 * q));
    pq.prev0 = (uint32_t)(X >> (62 - 2 * j)) & 3u;            // R[u-1]
    uint32_t nxt = (uint32_t)(X >> (62 - 2 * (j + 1 + q))) & 3u;  // R[u+q]
    pq.has0 = u >= 1;
    pq.g1 = pn_revcomp_code(pq.g0, q);
    pq.prev1 = 3u - nxt;  // T1[p-1] = complement of R[u+q]
    pq.has1 = u + q < ref.L;
    return true;
}

template <typename TW>
__global__ __launch_bounds__(kT) void k_filter_count(PnRefDev ref, PnIndexDev ix,
                                                     uint32_t *block_counts,
                                                     unsigned long long *n_seeds) {
    const uint64_t u0 = ((uint64_t)blockIdx.x * kT + threadIdx.x) * kPPT;
    uint32_t cnt = 0;
    unsigned long long seeds = 0;
    if (u0 + ix.q <= ref.L) {
        const uint64_t X = window32(ref.packed, (int64_t)u0 - 1);
#pragma unroll
        for (int j = 0; j < kPPT; j++) {
            PosQ pq;
            if (!pos_qgrams(ref, ix.q, X, u0 + j, j, pq)) break;
            Probe a = probe<TW>(ix, pq.g0, pq.has0, pq.prev0);
            Probe b = probe<TW>(ix, pq.g1, pq.has1, pq.prev1);
            cnt += (a.cl - a.ks) + (a.ke - a.ch) + (b.cl - b.ks) + (b.ke - b.ch);
            seeds += (a.ke - a.ks) + (b.ke - b.ks);
        }
    }
    uint32_t total;
    pn_block_excl_scan(cnt, &total);
    for (int o = 32; o > 0; o >>= 1) seeds += __shfl_xor(seeds, o);
    if ((threadIdx.x & 63) == 0 && seeds) atomicAdd(n_seeds, seeds);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = total;
}

__device__ __forceinline__ void emit_range(const PnIndexDev &ix, uint32_t a, uint32_t b,
                                           int64_t p, uint32_t s, uint2 *out, uint64_t &at) {
    for (uint32_t k = a; k < b; k++) {
        uint32_t e = ix.O[k];
        uint32_t r = (e >> 8) & (PN_MAX_READS - 1);
        int64_t d = p - (int64_t)(e & 0xffu);
        out[at++] = make_uint2(r | (s << 31), (uint32_t)(d + PN_DBIAS));
    }
}

template <typename TW>
__global__ __launch_bounds__(kT) void k_filter_emit(PnRefDev ref, PnIndexDev ix, uint64_t blk0,
                                                    const uint64_t *block_offsets, uint2 *cands) {
    const uint64_t blk = blk0 + blockIdx.x;
    const uint64_t u0 = (blk * kT + threadIdx.x) * kPPT;
    const bool any = u0 + ix.q <= ref.L;
    const uint64_t X = any ? window32(ref.packed, (int64_t)u0 - 1) : 0;
    uint32_t cnt = 0;
    if (any) {
#pragma unroll
        for (int j = 0; j < kPPT; j++) {
            PosQ pq;
            if (!pos_qgrams(ref, ix.q, X, u0 + j, j, pq)) break;
            Probe a = probe<TW>(ix, pq.g0, pq.has0, pq.prev0);
            Probe b = probe<TW>(ix, pq.g1, pq.has1, pq.prev1);
            cnt += (a.cl - a.ks) + (a.ke - a.ch) + (b.cl - b.ks) + (b.ke - b.ch);
        }
    }
    uint32_t total;
    uint32_t ex = pn_block_excl_scan(cnt, &total);
    if (!any || cnt == 0) return;
    uint64_t at = block_offsets[blk] - block_offsets[blk0] + ex;
    for (int j = 0; j < kPPT; j++) {
        PosQ pq;
        const uint64_t u = u0 + j;
        if (!pos_qgrams(ref, ix.q, X, u, j, pq)) break;
        Probe a = probe<TW>(ix, pq.g0, pq.has0, pq.prev0);
        emit_range(ix, a.ks, a.cl, (int64_t)u, 0, cands, at);
        emit_range(ix, a.ch, a.ke, (int64_t)u, 0, cands, at);
        Probe b = probe<TW>(ix, pq.g1, pq.has1, pq.prev1);
        const int64_t p1 = (int64_t)(ref.L - ix.q - u);
        emit_range(ix, b.ks, b.cl, p1, 1, cands, at);
        emit_range(ix, b.ch, b.ke, p1, 1, cands, at);
    }
}

}  // namespace

namespace pn {

void launch_filter_count(const PnRefDev &ref, const PnIndexDev &ix, uint64_t n_blocks,
                         uint32_t *block_counts, unsigned long long *n_seeds, hipStream_t st) {
    if (!n_blocks) return;
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_filter_count<unsigned long long>, dim3((unsigned)n_blocks), dim3(kT),
                           0, st, ref, ix, block_counts, n_seeds);
    else
        hipLaunchKernelGGL(k_filter_count<uint32_t>, dim3((unsigned)n_blocks), dim3(kT), 0, st,
                           ref, ix, block_counts, n_seeds);
}

void launch_filter_emit(const PnRefDev &ref, const PnIndexDev &ix, uint64_t blk0, uint64_t blk1,
                        const uint64_t *block_offsets, uint2 *cands, hipStream_t st) {
    if (blk1 <= blk0) return;
    if (ix.log2w == 6)
        hipLaunchKernelGGL(k_filter_emit<unsigned long long>, dim3((unsigned)(blk1 - blk0)),
                           dim3(kT), 0, st, ref, ix, blk0, block_offsets, cands);
    else
        hipLaunchKernelGGL(k_filter_emit<uint32_t>, dim3((unsigned)(blk1 - blk0)), dim3(kT), 0, st,
                           ref, ix, blk0, block_offsets, cands);
}

}  // namespace pn
