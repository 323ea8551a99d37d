// Validation (Section 3.3): banded bit-parallel semiglobal edit distance,
// one candidate per lane, the band of W = 2k+1 diagonals [d-k, d+k] held in
// one 32-bit word (k <= 15).
//
// The band is processed row by row (one read letter per step).  Bit b of
// row i stands for column c = i + (d-k) + b, so the same bit index is the
// same diagonal in every row.  The words VP/VN hold the horizontal
// differences D[i][c] - D[i][c-1] (+1 / -1) along the row; a step is Myers'
// bit-vector column update (Myers 1999, in the formulation of Hyyro 2003)
// with the roles of text and pattern exchanged: the band's reference
// letters are the "pattern" bits, the read letter x_i is the "text"
// character.  Between rows the previous row's differences move one bit
// down (its column c sits at bit b+1 of the previous row); the column that
// enters on the right has no value in the band and is given the difference
// +1, and the carry into bit 0 is +1 as well — both stand for paths that
// are never better than the in-band diagonal move, so the band values are
// exactly those of the band-restricted recurrence.
//
// Reference positions outside [0, L) never match (validity plane V): with
// a free start on row 0 this reproduces E[i][0] = i at column 0.  The
// value of the right-most band cell is tracked explicitly; every other
// cell follows from the differences.  A lane stops as soon as every cell of
// its row exceeds k (the row minimum never decreases from one row to the
// next; bounded below by R - #(+1 steps)), or after row n, where it reports
// each end column with value <= k.
#include "pn_band.h"

namespace {

__global__ __launch_bounds__(256) void k_verify(PnRefDev ref, PnIndexDev ix,
                                                const uint2 *__restrict__ cands,
                                                const unsigned long long *__restrict__ n_dev,
                                                uint64_t cap, int kglob,
                                                const uint8_t *__restrict__ kpr,
                                                pn::VerifyOut out) {
    const uint64_t n = min((uint64_t)*n_dev, cap);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long rows = 0;
    for (uint64_t ci = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ci < n; ci += stride) {
        const uint2 c = cands[ci];
        if (c.x == PN_CAND_NONE) continue;  // padding slot
        const uint32_t r = c.x & 0x7fffffffu;
        const uint32_t s = c.x >> 31;
        const int64_t d = (int64_t)c.y - (int64_t)PN_DBIAS;
        const int len = (int)(ix.offsets[r + 1] - ix.offsets[r]);
        const int k = kglob >= 0 ? kglob : (int)kpr[r];
        if (k > PN_MAX_K || len < 1 || len > PN_MAX_READ_LEN) continue;
        const unsigned long long head = (((unsigned long long)r << 1) | s) << out.ebits;
        rows += (unsigned long long)pn_band_verify(
            s ? ref.planes[1] : ref.planes[0], ix.rplanes + (uint64_t)r * PN_READ_WORDS, len, k,
            d - k, ref.L, [&](uint32_t e, int v) {
                unsigned long long at = atomicAdd(out.count, 1ull);
                if (at < out.capacity)
                    out.records[at] = ((head | (unsigned long long)e) << 5) | (unsigned long long)v;
            });
    }
    for (int o = 32; o > 0; o >>= 1) rows += __shfl_xor(rows, o);
    if ((threadIdx.x & 63) == 0 && rows) atomicAdd(out.rows, rows);
}

}  // namespace

namespace pn {

void launch_verify(const PnRefDev &ref, const PnIndexDev &ix, const uint2 *cands,
                   const unsigned long long *n_dev, uint64_t cap, int kglob, const uint8_t *kpr,
                   VerifyOut out, hipStream_t st) {
    if (!cap) return;
    // enough resident waves to fill the chip; each thread strides over candidates
    uint64_t blocks = (cap + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_verify, dim3((unsigned)blocks), dim3(256), 0, st, ref, ix, cands, n_dev,
                       cap, kglob, kpr, out);
}

}  // namespace pn
