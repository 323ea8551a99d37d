// Canonical hit list (Section 3.4, postprocessing): records (read, strand,
// end, errors) packed into 64-bit keys are sorted, duplicates of the same
// (read, strand, end) found through several candidates keep the smallest
// error count, and best-stratum mode keeps the hits whose error count is the
// read's minimum.  The sort is a stable LSD radix sort with 8-bit digits:
// per-tile digit histograms (stored tile by tile, 256 counts each), an
// exclusive scan in (digit, tile) order done column by column, and a stable
// scatter that ranks equal digits inside each wave with ballots.
#include "pn_internal.h"
#include "pn_radix.h"

namespace {

constexpr int kThreads = 256;
// Radix tiles: 16 keys per thread; blocks of 512 threads (tiles of 8192
// keys: runs of 32 keys per digit on average, written as longer bursts) for
// large sorts, of 256 threads for smaller ones, where more tiles keep more
// of the chip busy
constexpr int kRadixItems = 16;
constexpr int kThrLarge = 512, kThrSmall = 256;
constexpr uint64_t kLargeSort = 1ull << 24;  // keys from which the large tiles are used
inline int radix_threads(uint64_t n) { return n >= kLargeSort ? kThrLarge : kThrSmall; }

// exclusive scan of one value per digit (threads 0-255) over the 256
// digits; every thread of the block calls it (it synchronises the block)
__device__ __forceinline__ uint32_t digit_excl_scan(uint32_t x) {
    __shared__ uint32_t ws[4];
    const int lane = threadIdx.x & 63, wave = (int)(threadIdx.x >> 6);
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (threadIdx.x < 256 && lane == 63) ws[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave && w < 4; w++) before += ws[w];
    __syncthreads();
    return before + inc - x;
}

inline unsigned grid_for(uint64_t n, unsigned threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// The digit a radix pass sorts by: bits [shift, shift + width) of the key,
// or (osh > 0) the first pass of an index whose slices are ordered by the
// letters after the q-gram (see pn::radix_sort_index_slices): the key's 7
// lowest bits above a piece-start flag.
struct RadixDigit {
    int shift;
    uint32_t dmask;
    int osh;       // where the read offset (8 bits) starts in an index key, or 0
    uint32_t ell;  // piece length
    __device__ __forceinline__ uint32_t operator()(unsigned long long k) const {
        if (osh) {
            const uint32_t o = (uint32_t)(k >> osh) & 0xffu;
            const uint32_t piece = ((uint32_t)k & 511u) < 256u && o % ell == 0u;
            return (((uint32_t)k & 127u) << 1) | piece;
        }
        return (uint32_t)(k >> shift) & dmask;
    }
};

template <int kThr>
__global__ __launch_bounds__(kThr) void k_radix_hist(const unsigned long long *keys, uint64_t n,
                                                     RadixDigit digit, uint32_t *hist,
                                                     uint64_t n_tiles) {
    constexpr int kTile = kThr * kRadixItems;
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int j = 0; j < kRadixItems; j++) {
        uint64_t i = base + (uint64_t)j * kThr + threadIdx.x;
        if (i < n) atomicAdd(&h[digit(keys[i])], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[(uint64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the tile-major counts hist[b][d] in (digit, tile) order:
// offs[b][d] = sum of all counts of digits below d + counts of digit d in
// tiles below b.  Three launches: column sums per group of tiles, a block
// per digit scanning its column over the groups (and its total), then each
// group's columns again with its carries and the digit base.  Sums and
// offsets are 64-bit (pn_radix.h).

// exclusive scan of one 64-bit value per thread over a 256-thread block;
// *total = block sum.  Every thread of the block must call it.
__device__ __forceinline__ pn_roff block_excl_scan64(pn_roff x, pn_roff *total) {
    __shared__ pn_roff ws[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    pn_roff inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const pn_roff y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    pn_roff before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
        before += w < wave ? ws[w] : (pn_roff)0;
        all += ws[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

__global__ __launch_bounds__(256) void k_col_sums(const uint32_t *__restrict__ hist,
                                                  uint64_t n_tiles, uint64_t per,
                                                  pn_roff *colsum) {
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = min(n_tiles, b0 + per);
    colsum[(uint64_t)blockIdx.x * 256 + threadIdx.x] =
        pn_radix_col_sum(hist, b0, b1, threadIdx.x);
}

// a block per digit d, a thread per group: colsum[g][d] -> the column's
// sum over groups below g, dtot[d] -> the column's total
__global__ __launch_bounds__(256) void k_col_top(pn_roff *colsum, uint32_t groups,
                                                 pn_roff *dtot) {
    const uint32_t d = blockIdx.x, g = threadIdx.x;
    const pn_roff v = g < groups ? colsum[(uint64_t)g * 256 + d] : (pn_roff)0;
    pn_roff tot;
    const pn_roff ex = block_excl_scan64(v, &tot);
    if (g < groups) colsum[(uint64_t)g * 256 + d] = ex;
    if (g == 0) dtot[d] = tot;
}

__global__ __launch_bounds__(256) void k_col_down(const uint32_t *__restrict__ hist,
                                                  uint64_t n_tiles, uint64_t per,
                                                  const pn_roff *__restrict__ colsum,
                                                  const pn_roff *__restrict__ dtot,
                                                  pn_roff *offs) {
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = min(n_tiles, b0 + per);
    pn_roff tot;
    const pn_roff base = block_excl_scan64(dtot[threadIdx.x], &tot);  // digits below this one
    pn_radix_col_down(hist, b0, b1, threadIdx.x,
                      colsum[(uint64_t)blockIdx.x * 256 + threadIdx.x] + base, offs);
}

// Stable scatter of one tile.  Wave w owns the tile's keys
// [w * kTile/4, (w + 1) * kTile/4), all loaded up front; each key's rank
// among the equal digits before it in its wave comes from ballots and a
// per-wave digit counter in LDS (no block barrier per step).  One prefix
// over the waves then places every key in digit order in LDS, and the tile
// is written out so that consecutive threads write consecutive addresses of
// one digit's run.
template <int kThr>
__global__ __launch_bounds__(kThr) void k_radix_scatter(const unsigned long long *keys,
                                                        unsigned long long *out, uint64_t n,
                                                        RadixDigit digit,
                                                        const pn_roff *offs,
                                                        const uint32_t *hist, uint64_t n_tiles) {
    constexpr int kItems = kRadixItems;
    constexpr int kTile = kThr * kItems;
    constexpr int kWaves = kThr / 64;
    constexpr int kPerWave = kTile / kWaves;
    __shared__ unsigned long long tile[kTile];
    __shared__ uint32_t local[256];        // start of each digit inside the tile
    __shared__ pn_roff goff[256];          // start of each digit's run in the output
    __shared__ uint32_t wcnt[kWaves][256];  // per wave: keys of each digit (then: before it)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    const uint32_t tile_n = (uint32_t)min((uint64_t)kTile, n - base);
    const uint32_t w0 = (uint32_t)wave * kPerWave;
    unsigned long long key[kItems];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const uint32_t li = w0 + (uint32_t)j * 64 + lane;
        key[j] = li < tile_n ? keys[base + li] : 0ull;
    }
    for (int t = threadIdx.x; t < kWaves * 256; t += kThr) (&wcnt[0][0])[t] = 0;
    {
        const bool dig = threadIdx.x < 256;
        const uint32_t c = dig ? hist[(uint64_t)blockIdx.x * 256 + threadIdx.x] : 0u;
        if (dig) goff[threadIdx.x] = offs[(uint64_t)blockIdx.x * 256 + threadIdx.x];
        const uint32_t ex = digit_excl_scan(c);  // (synchronises the block)
        if (dig) local[threadIdx.x] = ex;
    }
    uint32_t slot[kItems];  // digit | rank inside the wave's run of that digit << 8
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const uint32_t li = w0 + (uint32_t)j * 64 + lane;
        const bool valid = li < tile_n;
        const uint32_t dg = digit(key[j]);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (dg >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t before = wcnt[wave][dg];
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcnt[wave][dg] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        slot[j] = dg | ((before + rank) << 8);
    }
    __syncthreads();
    // per digit: the keys of the waves before each wave
    if (threadIdx.x < 256) {
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) {
            const uint32_t c = wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = acc + local[threadIdx.x];
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const uint32_t li = w0 + (uint32_t)j * 64 + lane;
        if (li < tile_n) tile[wcnt[wave][slot[j] & 255u] + (slot[j] >> 8)] = key[j];
    }
    __syncthreads();
    // the tile in digit order: slot i belongs to digit d with local[d] <= i,
    // and goes to offs[d] + (i - local[d])
    for (uint32_t i = threadIdx.x; i < tile_n; i += kThr) {
        const unsigned long long k = tile[i];
        const uint32_t dg = digit(k);
        out[goff[dg] + (i - local[dg])] = k;
    }
}

// smallest error count per read (over all records; duplicates do not matter)
__global__ void k_read_min(const unsigned long long *keys, uint64_t n, int ebits,
                           uint32_t *minv) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        unsigned long long k = keys[i];
        uint32_t r = (uint32_t)(k >> (6 + ebits));
        atomicMin(&minv[r], (uint32_t)(k & 31u));
    }
}

// smallest error count of the (read, strand, end) run that starts at i (the
// records of a run are adjacent, in no particular order of errors; a run
// holds the few candidates that reached the same end)
__device__ __forceinline__ uint32_t run_min_errors(const unsigned long long *keys, uint64_t n,
                                                   uint64_t i) {
    const unsigned long long k = keys[i];
    uint32_t m = (uint32_t)(k & 31u);
    for (uint64_t j = i + 1; j < n && (keys[j] >> 5) == (k >> 5); j++)
        m = min(m, (uint32_t)(keys[j] & 31u));
    return m;
}

// 1 for the first record of each (read, strand, end) run whose smallest
// error count also passes the stratum filter
__global__ void k_keep_flags(const unsigned long long *keys, uint64_t n, int ebits, int best,
                             const uint32_t *minv, uint32_t *flags) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        unsigned long long k = keys[i];
        uint32_t f = (i == 0) || ((keys[i - 1] >> 5) != (k >> 5));
        if (best && f) f = run_min_errors(keys, n, i) == minv[(uint32_t)(k >> (6 + ebits))];
        flags[i] = f;
    }
}

__device__ __forceinline__ uint4 key_to_hit(unsigned long long k, int ebits) {
    uint32_t v = (uint32_t)(k & 31u);
    uint32_t e = (uint32_t)((k >> 5) & ((1ull << ebits) - 1ull));
    uint32_t s = (uint32_t)((k >> (5 + ebits)) & 1u);
    uint32_t r = (uint32_t)(k >> (6 + ebits));
    return make_uint4(r, e, s | (v << 8), 0u);
}

__global__ void k_write_hits(const unsigned long long *keys, uint64_t n, int ebits,
                             const uint32_t *flags, const uint32_t *pos, uint32_t *out,
                             uint64_t capacity) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!flags[i]) continue;
        uint64_t p = pos[i];
        if (p >= capacity) continue;
        uint4 h = key_to_hit((keys[i] & ~31ull) | run_min_errors(keys, n, i), ebits);
        out[3 * p + 0] = h.x;
        out[3 * p + 1] = h.y;
        out[3 * p + 2] = h.z;
    }
}

__global__ void k_total(const uint32_t *pos, uint64_t n, unsigned long long *n_out) {
    *n_out = pos[n];
}

__global__ void k_records_to_hits(const unsigned long long *keys, uint64_t n, int ebits,
                                  uint32_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint4 h = key_to_hit(keys[i], ebits);
        out[3 * i + 0] = h.x;
        out[3 * i + 1] = h.y;
        out[3 * i + 2] = h.z;
    }
}

// candidate (read | strand << 31, diagonal + bias) -> sortable key
__global__ void k_cand_keys(const uint2 *c, uint64_t n, unsigned long long *keys) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint2 v = c[i];
        const uint32_t r = v.x == PN_CAND_NONE ? 0x7fffffffu : v.x & PN_CAND_READ;
        keys[i] = ((unsigned long long)r << 33) | ((unsigned long long)(v.x >> 31) << 32) | v.y;
    }
}

// sorted candidate key -> pn_candidate {u32 read, u8 strand, pad[3], i64 diag}
__global__ void k_keys_to_cands(const unsigned long long *keys, uint64_t n, uint32_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        unsigned long long k = keys[i];
        long long d = (long long)(k & 0xffffffffull) - (long long)PN_DBIAS;
        out[4 * i + 0] = (uint32_t)(k >> 33);
        out[4 * i + 1] = (uint32_t)((k >> 32) & 1u);
        out[4 * i + 2] = (uint32_t)((unsigned long long)d & 0xffffffffull);
        out[4 * i + 3] = (uint32_t)((unsigned long long)d >> 32);
    }
}

}  // namespace

namespace pn {

uint64_t radix_tile_keys(uint64_t n) { return (uint64_t)radix_threads(n) * kRadixItems; }

static uint64_t tiles_for(uint64_t n) {
    const uint64_t tile = radix_tile_keys(n);
    return (n + tile - 1) / tile;
}

// temp: counts (u32, 256 per tile), offsets (64-bit, 256 per tile), column
// sums (64-bit, 256 per group), digit totals (64-bit, 256)
uint64_t radix_temp_size(uint64_t n) {
    uint64_t nt = tiles_for(n) ? tiles_for(n) : 1;
    uint64_t hist = 256 * nt + 2;
    return hist * sizeof(uint32_t) +
           (hist + 256 * (uint64_t)PN_RADIX_GROUPS + 256) * sizeof(pn_roff) + 256;
}

// one stable pass src -> dst by `digit` (hist_given: its per-tile counts, if
// already made)
static void radix_pass(const unsigned long long *src, unsigned long long *dst, uint64_t n,
                       RadixDigit digit, const uint32_t *hist_given, void *temp, hipStream_t st) {
    const uint64_t nt = tiles_for(n);
    uint32_t *hist = (uint32_t *)temp;
    pn_roff *offs = (pn_roff *)(hist + 256 * nt + 2);  // (8-byte aligned: temp is)
    pn_roff *colsum = offs + 256 * nt + 2;
    pn_roff *dtot = colsum + 256 * (uint64_t)PN_RADIX_GROUPS;
    const uint64_t per = pn_radix_tiles_per_group(nt);  // tiles per group
    const uint32_t groups = (uint32_t)((nt + per - 1) / per);
    const uint32_t *hp = hist_given ? hist_given : hist;
    if (!hist_given && radix_threads(n) == kThrLarge)
        hipLaunchKernelGGL(k_radix_hist<kThrLarge>, dim3((unsigned)nt), dim3(kThrLarge), 0, st,
                           src, n, digit, hist, nt);
    else if (!hist_given)
        hipLaunchKernelGGL(k_radix_hist<kThrSmall>, dim3((unsigned)nt), dim3(kThrSmall), 0, st,
                           src, n, digit, hist, nt);
    hipLaunchKernelGGL(k_col_sums, dim3(groups), dim3(256), 0, st, hp, nt, per, colsum);
    hipLaunchKernelGGL(k_col_top, dim3(256), dim3(256), 0, st, colsum, groups, dtot);
    hipLaunchKernelGGL(k_col_down, dim3(groups), dim3(256), 0, st, hp, nt, per,
                       (const pn_roff *)colsum, (const pn_roff *)dtot, offs);
    if (radix_threads(n) == kThrLarge)
        hipLaunchKernelGGL(k_radix_scatter<kThrLarge>, dim3((unsigned)nt), dim3(kThrLarge), 0, st,
                           src, dst, n, digit, (const pn_roff *)offs, hp, nt);
    else
        hipLaunchKernelGGL(k_radix_scatter<kThrSmall>, dim3((unsigned)nt), dim3(kThrSmall), 0, st,
                           src, dst, n, digit, (const pn_roff *)offs, hp, nt);
}

unsigned long long *radix_sort_u64_any(unsigned long long *keys, unsigned long long *tmp,
                                       uint64_t n, int bits, void *temp, hipStream_t st, int lo,
                                       const uint32_t *hist0) {
    if (n <= 1 || bits <= 0) return keys;
    unsigned long long *src = keys, *dst = tmp;
    const int passes = (bits - lo + 7) / 8;
    for (int p = 0; p < passes; p++) {
        const int shift = lo + 8 * p;
        // the last digit may be narrower: bits above `bits` do not take part
        const uint32_t dmask = bits - shift >= 8 ? 255u : (1u << (bits - shift)) - 1u;
        // the first pass may come with its histogram (made with the keys:
        // the counts of the digit at bit lo)
        radix_pass(src, dst, n, RadixDigit{shift, dmask, 0, 1u}, p == 0 ? hist0 : nullptr, temp,
                   st);
        unsigned long long *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// An index key (q <= 12: read and offset, letter before, q-gram, 9-bit code
// of the letters after) sorted by (q-gram, code, piece start): each slice
// ordered by the letters after its q-gram, and inside one code the entries
// that start a piece (read offset a multiple of q + 4, four letters after
// it) last.  The first pass takes the code's low 7 bits above the piece
// flag, the others bits 7 .. 2q + 9 of the key.
unsigned long long *radix_sort_index_slices(unsigned long long *keys, unsigned long long *tmp,
                                            uint64_t n, int q, void *temp, hipStream_t st) {
    if (n <= 1) return keys;
    radix_pass(keys, tmp, n, RadixDigit{0, 0u, 2 * q + 11, (uint32_t)q + 4u}, nullptr, temp, st);
    return radix_sort_u64_any(tmp, keys, n, 2 * q + 9, temp, st, 7);
}

void radix_sort_u64(unsigned long long *keys, unsigned long long *tmp, uint64_t n, int bits,
                    void *temp, hipStream_t st, int lo) {
    unsigned long long *src = radix_sort_u64_any(keys, tmp, n, bits, temp, st, lo);
    if (src != keys)
        (void)hipMemcpyAsync(keys, src, n * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                             st);
}

void launch_finish_hits(const unsigned long long *sorted, uint64_t n, int ebits, int best,
                        uint32_t n_reads, uint32_t *minv, uint32_t *flags, uint32_t *pos,
                        uint32_t *partials, void *out_hits, uint64_t capacity,
                        unsigned long long *n_out, hipStream_t st) {
    if (best) {
        launch_fill_u32(minv, n_reads, 0xffffffffu, st);
        if (n)
            hipLaunchKernelGGL(k_read_min, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, sorted, n,
                               ebits, minv);
    }
    if (n)
        hipLaunchKernelGGL(k_keep_flags, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, sorted, n,
                           ebits, best, (const uint32_t *)minv, flags);
    launch_scan_u32(flags, pos, n, partials, st);
    if (n)
        hipLaunchKernelGGL(k_write_hits, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, sorted, n,
                           ebits, (const uint32_t *)flags, (const uint32_t *)pos,
                           (uint32_t *)out_hits, capacity);
    hipLaunchKernelGGL(k_total, dim3(1), dim3(1), 0, st, (const uint32_t *)pos, n, n_out);
}

void launch_records_to_hits(const unsigned long long *sorted, uint64_t n, int ebits, void *out,
                            hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_records_to_hits, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, sorted, n,
                       ebits, (uint32_t *)out);
}

void launch_cand_keys(const uint2 *c, uint64_t n, unsigned long long *keys, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_cand_keys, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, c, n, keys);
}

void launch_keys_to_cands(const unsigned long long *keys, uint64_t n, void *out, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_keys_to_cands, dim3(pn_stride_blocks(n, 256)), dim3(256), 0, st, keys, n,
                       (uint32_t *)out);
}

}  // namespace pn
