// Exclusive prefix sums (the cumulative sums of Algorithm 1, steps 3 and 5;
// the parallel prefix scans of Section 2.1).  Reduce-then-scan in three
// launches: per-tile sums, one block scanning the tile sums, per-tile scan
// plus carry.  Tiles are 4096 elements (256 lanes x 16); values are uint32.
#include "pn_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;

__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 5); }

struct LoadU32 {
    const uint32_t *p;
    __device__ uint32_t operator()(uint64_t i) const { return p[i]; }
};
template <typename TW>
struct LoadPopc {
    const TW *I;
    __device__ uint32_t operator()(uint64_t i) const { return (uint32_t)pn_popc<TW>(I[i]); }
};

// inclusive scan across the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// exclusive block scan of one value per thread; returns the thread's
// exclusive prefix and writes the block total to *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *total) {
    __shared__ uint32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; w++) {
        uint32_t s = wsum[w];
        before += (w < wave) ? s : 0u;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

template <typename Load>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(Load load, uint64_t n,
                                                          uint32_t *partials) {
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        if (i < n) s += load(i);
    }
    uint32_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// one block: exclusive scan of partials[0..nb) in place, total to partials[nb];
// each thread takes kTopItems consecutive values per round, so a round
// covers 8192 tile sums (each thread reads and writes only its own)
constexpr int kTopItems = 32;

__global__ __launch_bounds__(kThreads) void k_scan_top(uint32_t *partials, uint64_t nb) {
    uint32_t carry = 0;
    for (uint64_t base = 0; base < nb; base += (uint64_t)kThreads * kTopItems) {
        const uint64_t i0 = base + (uint64_t)threadIdx.x * kTopItems;
        uint32_t x[kTopItems];
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < kTopItems; j++) {
            x[j] = i0 + j < nb ? partials[i0 + j] : 0u;
            s += x[j];
        }
        uint32_t total;
        uint32_t run = carry + block_excl_scan(s, &total);
#pragma unroll
        for (int j = 0; j < kTopItems; j++) {
            if (i0 + j < nb) partials[i0 + j] = run;
            run += x[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) partials[nb] = carry;
}

template <typename Load>
__global__ __launch_bounds__(kThreads) void k_scan_down(Load load, uint32_t *out, uint64_t n,
                                                        const uint32_t *partials, uint64_t nb) {
    __shared__ uint32_t tile[kTile + kTile / 32];
    uint64_t base = (uint64_t)blockIdx.x * kTile;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        int li = j * kThreads + threadIdx.x;
        uint64_t i = base + li;
        tile[lds_idx(li)] = i < n ? load(i) : 0u;
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        v[j] = tile[lds_idx(threadIdx.x * kItems + j)];
        s += v[j];
    }
    uint32_t total;
    uint32_t run = block_excl_scan(s, &total) + partials[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        tile[lds_idx(threadIdx.x * kItems + j)] = run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        int li = j * kThreads + threadIdx.x;
        uint64_t i = base + li;
        if (i < n) out[i] = tile[lds_idx(li)];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partials[nb];
}

// The group starts of a sorted q-gram list (Algorithm 1 steps 4-6): for
// every i with flags[i] = 1, Sp[number of flags before i] = i, and
// Sp[number of flags] = n.  The flags are bytes (0 or 1); a thread takes 16
// consecutive ones in one 16-byte load, and counts them as the set bits of
// its four words.  Tiles of kTile flags: per-tile counts, one block scanning
// them, then each tile again with its carry placing its starts (the prefix
// sums are never stored).
__device__ __forceinline__ uint4 load_flags16(const uint8_t *__restrict__ flags, uint64_t n,
                                              uint64_t first) {
    if (first + 16 <= n) return *(const uint4 *)(flags + first);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (uint64_t j = first; j < n && j < first + 16; j++)
        w[(j - first) >> 2] |= (uint32_t)flags[j] << (8 * ((j - first) & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ __launch_bounds__(kThreads) void k_flags_reduce(const uint8_t *__restrict__ flags,
                                                           uint64_t n, uint32_t *partials) {
    const uint64_t first = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    const uint4 v = first < n ? load_flags16(flags, n, first) : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t c = __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    uint32_t total;
    block_excl_scan(c, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_down_sp(const uint8_t *__restrict__ flags,
                                                           uint64_t n,
                                                           const uint32_t *partials, uint64_t nb,
                                                           uint32_t *Sp) {
    const uint64_t first = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    const uint4 v = first < n ? load_flags16(flags, n, first) : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t c = __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    uint32_t total;
    uint32_t run = block_excl_scan(c, &total) + partials[blockIdx.x];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        if ((w[j >> 2] >> (8 * (j & 3))) & 1u) Sp[run++] = (uint32_t)(first + j);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) Sp[partials[nb]] = (uint32_t)n;
}

template <typename Load>
void scan_impl(Load load, uint32_t *out, uint64_t n, uint32_t *partials, hipStream_t st) {
    uint64_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce<Load>, dim3((unsigned)nb), dim3(kThreads), 0, st, load, n,
                       partials);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, st, partials, nb);
    hipLaunchKernelGGL(k_scan_down<Load>, dim3((unsigned)nb), dim3(kThreads), 0, st, load, out, n,
                       (const uint32_t *)partials, nb);
}

// Concatenation of a sharded list: block b copies part b / regions of
// region b % regions to dst at the region's exclusive prefix of counts.
__global__ __launch_bounds__(256) void k_gather_shards(const unsigned long long *__restrict__ src,
                                                       const unsigned long long *__restrict__ counts,
                                                       uint32_t regions, uint64_t region_cap,
                                                       unsigned long long *__restrict__ dst) {
    const uint32_t g = blockIdx.x % regions;
    uint64_t start = 0;
    for (uint32_t t = 0; t < g; t++) start += min((uint64_t)counts[t], region_cap);
    const uint64_t n = min((uint64_t)counts[g], region_cap);
    const uint64_t per = gridDim.x / regions;
    const unsigned long long *s = src + (uint64_t)g * region_cap;
    for (uint64_t i = (blockIdx.x / regions) * 256 + threadIdx.x; i < n; i += per * 256)
        dst[start + i] = s[i];
}

}  // namespace

namespace pn {

uint64_t scan_partials_size(uint64_t n) { return (n + kTile - 1) / kTile + 2; }

void launch_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *partials,
                     hipStream_t st) {
    scan_impl(LoadU32{in}, out, n, partials, st);
}

void launch_starts_to_sp(const uint8_t *flags, uint64_t n, uint32_t *partials, uint32_t *Sp,
                         hipStream_t st) {
    uint64_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_flags_reduce, dim3((unsigned)nb), dim3(kThreads), 0, st, flags, n,
                       partials);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, st, partials, nb);
    hipLaunchKernelGGL(k_scan_down_sp, dim3((unsigned)nb), dim3(kThreads), 0, st, flags, n,
                       (const uint32_t *)partials, nb, Sp);
}

void launch_scan_popc(const void *I, int log2w, uint32_t *out, uint64_t n, uint32_t *partials,
                      hipStream_t st) {
    if (log2w == 6)
        scan_impl(LoadPopc<uint64_t>{(const uint64_t *)I}, out, n, partials, st);
    else
        scan_impl(LoadPopc<uint32_t>{(const uint32_t *)I}, out, n, partials, st);
}

void launch_gather_shards(const unsigned long long *src, const unsigned long long *counts,
                          uint32_t regions, uint64_t region_cap, unsigned long long *dst,
                          hipStream_t st) {
    if (!regions || !region_cap) return;
    uint64_t per = (region_cap + 255) / 256;
    if (per > 64) per = 64;
    hipLaunchKernelGGL(k_gather_shards, dim3((unsigned)(per * regions)), dim3(256), 0, st, src,
                       counts, regions, region_cap, dst);
}

}  // namespace pn
