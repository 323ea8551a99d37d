// Ingest: ASCII -> 2-bit codes, reference bit planes for both strands, read
// metadata and read bit planes.  Base codes follow Section 2.2
// (A=00, C=01, G=10, T=11).
#include "pn_internal.h"

namespace {

// code of an ASCII letter (either case) and whether it is A/C/G/T.
// A 0x41 -> 0, C 0x43 -> 1, G 0x47 -> 2, T 0x54 -> 3 (same for lower case).
__device__ __forceinline__ uint32_t ascii_code(uint32_t c, bool &ok) {
    uint32_t l = c | 0x20u;
    ok = (l == 'a') | (l == 'c') | (l == 'g') | (l == 't');
    return ((c >> 1) ^ (c >> 2)) & 3u;
}

__global__ void k_pack2(const char *__restrict__ ascii, uint64_t n, uint32_t *__restrict__ packed,
                        uint32_t *status, int aligned16) {
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t t0 = w * 16;
    if (t0 >= n) return;
    uint32_t bytes[16];
    if (aligned16 && t0 + 16 <= n) {
        uint4 v = *reinterpret_cast<const uint4 *>(ascii + t0);
        uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 16; i++) bytes[i] = (u[i >> 2] >> (8 * (i & 3))) & 0xffu;
    } else {
#pragma unroll
        for (int i = 0; i < 16; i++) bytes[i] = (t0 + i < n) ? (uint32_t)(uint8_t)ascii[t0 + i] : 'A';
    }
    uint32_t word = 0;
    bool all_ok = true;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        bool ok;
        uint32_t c = ascii_code(bytes[i], ok);
        all_ok &= ok;
        word |= c << (30 - 2 * i);
    }
    packed[w] = word;
    if (!all_ok) atomicOr(status, 1u);
}

__global__ void k_ref_planes(const uint32_t *__restrict__ packed, uint64_t L,
                             uint4 *__restrict__ planes0, uint4 *__restrict__ planes1,
                             uint64_t n_blocks) {
    uint64_t B = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= n_blocks) return;
    int64_t t0 = 32 * ((int64_t)B - PN_PAD_BLOCKS);
    uint32_t h0 = 0, l0 = 0, h1 = 0, l1 = 0, v = 0;
    for (int b = 0; b < 32; b++) {
        int64_t t = t0 + b;
        if (t < 0 || t >= (int64_t)L) continue;
        uint32_t c0 = pn_base_at(packed, (uint64_t)t);
        // strand 1 at t is the complement of strand 0 at L-1-t
        uint32_t c1 = 3u - pn_base_at(packed, L - 1 - (uint64_t)t);
        h0 |= (c0 >> 1) << b;
        l0 |= (c0 & 1u) << b;
        h1 |= (c1 >> 1) << b;
        l1 |= (c1 & 1u) << b;
        v |= 1u << b;
    }
    planes0[B] = make_uint4(h0, l0, v, 0u);
    planes1[B] = make_uint4(h1, l1, v, 0u);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    return x;
}

// stats[0] = max read length, stats[1] = |T| = sum max(0, n_r - q + 1),
// stats[2] = number of malformed reads (decreasing offsets, past n_bases,
// or longer than PN_MAX_READ_LEN)
__global__ __launch_bounds__(256) void k_read_meta(const uint64_t *__restrict__ offsets,
                                                   uint32_t n_reads, int q, uint64_t n_bases,
                                                   unsigned long long *stats) {
    // a grid-stride loop and one atomic per block and figure: the three
    // figures live at three addresses, whose atomics serialise
    unsigned long long mx = 0, tq = 0, bad = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n_reads;
         r += gridDim.x * blockDim.x) {
        const uint64_t a = offsets[r], b = offsets[r + 1];
        if (b < a || b > n_bases) {
            bad++;
        } else {
            const unsigned long long len = b - a;
            mx = len > mx ? len : mx;
            tq += len >= (unsigned long long)q ? len - q + 1 : 0;
            bad += len > PN_MAX_READ_LEN;
        }
    }
    mx = wave_max_u64(mx);
    tq = wave_sum_u64(tq);
    bad = wave_sum_u64(bad);
    __shared__ unsigned long long red[3][4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = mx;
        red[1][wave] = tq;
        red[2][wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            mx = red[0][w] > mx ? red[0][w] : mx;
            tq += red[1][w];
            bad += red[2][w];
        }
        atomicMax(&stats[0], mx);
        if (tq) atomicAdd(&stats[1], tq);
        if (bad) atomicAdd(&stats[2], bad);
    }
}

// the odd (hi = true) or even bits of a 32-bit word packed into 16 bits,
// in order: bit 2t+1 (or 2t) goes to bit t
__device__ __forceinline__ uint32_t compress_bits(uint32_t x, bool hi) {
    x = (hi ? x >> 1 : x) & 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0f0f0f0fu;
    x = (x | (x >> 4)) & 0x00ff00ffu;
    return (x | (x >> 8)) & 0x0000ffffu;
}

// Plane words of one read (a thread per read): word m holds letters
// 32m .. 32m+31, letter b of the word in bit b (H: high code bit, L: low).
// The forward words come from 64-bit windows of the packed text (32
// letters, first letter in the top two bits): the odd bits give H and the
// even bits L, highest first, so a bit reversal puts letter b at bit b.
// Letter j of the reverse complement is the complement (both code bits
// flipped) of forward letter len-1-j, so its words are the forward bit
// vectors read backwards and inverted.  Bits past the read's end are 0.
__global__ __launch_bounds__(256) void k_read_planes(const uint32_t *__restrict__ packed,
                                                     const uint64_t *__restrict__ offsets,
                                                     uint32_t n_reads, uint2 *__restrict__ rplanes,
                                                     uint2 *__restrict__ rplanes_rc) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_reads) return;
    const uint64_t start = offsets[r];
    const int len = (int)min(offsets[r + 1] - start, (uint64_t)PN_MAX_READ_LEN);
    uint32_t H[PN_READ_WORDS], L[PN_READ_WORDS];
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) {
        H[m] = L[m] = 0;
        const int left = len - 32 * m;  // letters of this word inside the read
        if (left > 0) {
            const uint64_t t = start + 32ull * m;
            const uint64_t wi = t >> 4;
            const uint32_t sh = 2 * (uint32_t)(t & 15);
            const uint32_t w0 = packed[wi], w1 = packed[wi + 1], w2 = packed[wi + 2];
            const uint32_t hi = sh ? (w0 << sh) | (w1 >> (32 - sh)) : w0;  // letters 0-15
            const uint32_t lo = sh ? (w1 << sh) | (w2 >> (32 - sh)) : w1;  // letters 16-31
            const uint32_t keep = left >= 32 ? 0xffffffffu : (1u << left) - 1u;
            H[m] = __builtin_bitreverse32((compress_bits(hi, true) << 16) | compress_bits(lo, true)) &
                   keep;
            L[m] = __builtin_bitreverse32((compress_bits(hi, false) << 16) | compress_bits(lo, false)) &
                   keep;
        }
    }
    uint2 *f = rplanes + (uint64_t)r * PN_READ_WORDS;
    uint2 *rc = rplanes_rc + (uint64_t)r * PN_READ_WORDS;
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) f[m] = make_uint2(H[m], L[m]);
    // reverse complement word m: forward bits len-1-32m-b for b = 0..31,
    // i.e. forward bits [e-32, e) read downwards, e = len - 32m
#pragma unroll
    for (int m = 0; m < PN_READ_WORDS; m++) {
        const int e = len - 32 * m;
        uint32_t h = 0, l = 0;
        if (e > 0) {
            // forward bits [e-32, e) as one word (bits below 0 are 0)
            const int lo_bit = e - 32;
            uint32_t vh, vl;
            if (lo_bit >= 0) {
                const int wlo = lo_bit >> 5, s5 = lo_bit & 31;
                const uint32_t h0 = H[wlo], h1 = wlo + 1 < PN_READ_WORDS ? H[wlo + 1] : 0u;
                const uint32_t l0 = L[wlo], l1 = wlo + 1 < PN_READ_WORDS ? L[wlo + 1] : 0u;
                vh = s5 ? (h0 >> s5) | (h1 << (32 - s5)) : h0;
                vl = s5 ? (l0 >> s5) | (l1 << (32 - s5)) : l0;
            } else {
                vh = H[0] << (-lo_bit);
                vl = L[0] << (-lo_bit);
            }
            const uint32_t keep = e >= 32 ? 0xffffffffu : (1u << e) - 1u;
            h = ~__builtin_bitreverse32(vh) & keep;
            l = ~__builtin_bitreverse32(vl) & keep;
        }
        rc[m] = make_uint2(h, l);
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

inline unsigned grid_for(uint64_t n, unsigned threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

namespace pn {

void launch_pack2(const char *ascii, uint64_t n, uint32_t *packed, uint32_t *status,
                  hipStream_t st) {
    uint64_t words = (n + 15) / 16;
    if (!words) return;
    int aligned = ((uintptr_t)ascii % 16) == 0;
    hipLaunchKernelGGL(k_pack2, dim3(grid_for(words, 256)), dim3(256), 0, st, ascii, n, packed,
                       status, aligned);
}

void launch_ref_planes(const uint32_t *packed, uint64_t L, uint4 *planes0, uint4 *planes1,
                       uint64_t n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_ref_planes, dim3(grid_for(n_blocks, 256)), dim3(256), 0, st, packed, L,
                       planes0, planes1, n_blocks);
}

void launch_read_meta(const uint64_t *offsets, uint32_t n_reads, int q, uint64_t n_bases,
                      uint64_t *stats, hipStream_t st) {
    if (!n_reads) return;
    uint64_t g = grid_for(n_reads, 256 * 8);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_read_meta, dim3((unsigned)g), dim3(256), 0, st, offsets, n_reads, q,
                       n_bases, (unsigned long long *)stats);
}

void launch_read_planes(const uint32_t *packed, const uint64_t *offsets, uint32_t n_reads,
                        uint2 *rplanes, hipStream_t st) {
    uint64_t n = (uint64_t)n_reads * PN_READ_WORDS;
    if (!n) return;
    hipLaunchKernelGGL(k_read_planes, dim3(grid_for(n_reads, 256)), dim3(256), 0, st, packed,
                       offsets, n_reads, rplanes, rplanes + n);
}

void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
    if (!n) return;
    uint64_t g = grid_for(n, 256);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
}

}  // namespace pn
