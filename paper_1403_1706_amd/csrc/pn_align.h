// Start position and alignment of a hit (Section 3.3 runs the verification
// backwards from a hit's end to find where it starts; Section 3.4 makes the
// alignment in postprocessing).
//
// For a hit (read x of length n, strand s, end e, errors v): F[i][j] = edit
// distance (unit costs, no free start) of the read's last i letters and the
// j text letters ending at e, for 0 <= j <= e + 1.  min_j F[n][j] = v (the
// semiglobal value at e), the start is e + 1 - j for the smallest such j,
// and the alignment is read off from (n, j) back to (0, 0): of the
// predecessors that explain a cell, the diagonal one first (a match '=' or
// a substitution 'X'), then the one above (a read letter not in the text,
// 'I'), then the one to the left (a text letter not in the read, 'D').
// Row n holds the read's first letter, so the walk emits the read's first
// operation first.
//
// Only cells of value <= v matter, and such a cell lies within v diagonals
// of the main one (F >= |i - j|), as does every cell of its optimal paths
// (their values never exceed the cell's).  So the band |i - j| <= v with
// values saturated at v + 1 gives every such cell its exact value, and a
// cell above v reads v + 1, which never explains a cell of value <= v.
// The band index b = j - i + v (0 .. 2v) is the bit and array index; from
// row i - 1 to row i the diagonal predecessor keeps its index, the one
// above sits at b + 1, the one to the left at b - 1.
//
// The reversed read against the text read backwards is, letter for letter,
// the read's reverse complement against the other strand read forwards
// (complementing both sides keeps every match): cell (i, j) compares the
// reverse complement's letter i - 1 with the other strand's letter at
// L - 2 - e + j, so a row's match bits come from the other strand's bit
// planes with the funnel shifts the validation kernels use.
#pragma once
#include "pn_band.h"

// One hit, error count K, read length n (its reverse complement's plane
// words rp), end e on a strand whose other strand's planes are pl (text
// length L).  Row i's op codes (2 bits per band cell: 0 '=', 1 'X', 2 'I',
// 3 'D'; cell b in bits 2 (b mod 32) of word b / 32) go to
// bp[((i - 1) * NW + b / 32) * bstride], NW = pn_align_row_words(K).  Writes *start and *err (0xff and
// start 0 when no alignment of K errors ends at e) and, with want_ops, the
// operations into o (at most stride of them; o may be null) and returns
// their number (0 without want_ops).
__host__ __device__ constexpr int pn_align_row_words(int K) { return (2 * (2 * K + 1) + 63) / 64; }

template <int K>
__host__ __device__ inline int pn_align_one(const uint4 *pl, const uint2 *rp, int n, int64_t e,
                                            uint64_t L, unsigned long long *bp, uint64_t bstride,
                                            bool want_ops, uint8_t *o, uint32_t stride,
                                            uint32_t *start, uint8_t *err) {
    constexpr int W = 2 * K + 1;
    constexpr int C = K + 1;  // saturation value
    constexpr int NW = pn_align_row_words(K);
    // other-strand position of cell (i, b): p0 + i + b
    const int64_t p0 = (int64_t)L - 2 - e - K;
    int Fp[W], F[W];
#pragma unroll
    for (int b = 0; b < W; b++) Fp[b] = b >= K ? b - K : C;
    for (int i = 1; i <= n; i++) {
        const uint64_t tp = (uint64_t)(p0 + i + PN_PAD_POS);
        const uint64_t blk = tp >> 5;
        const uint32_t ph = (uint32_t)(tp & 31);
        const uint4 A = pl[blk], B = pl[blk + 1];
        // the W text letters of the row (a second word for W > 32)
        uint64_t H = pn_funnel(B.x, A.x, ph), Lw = pn_funnel(B.y, A.y, ph),
                 V = pn_funnel(B.z, A.z, ph);
        if (W > 32) {
            const uint4 Cb = pl[blk + 2];
            H |= (uint64_t)pn_funnel(Cb.x, B.x, ph) << 32;
            Lw |= (uint64_t)pn_funnel(Cb.y, B.y, ph) << 32;
            V |= (uint64_t)pn_funnel(Cb.z, B.z, ph) << 32;
        }
        const uint2 rw = rp[(i - 1) >> 5];
        const uint32_t sh = (uint32_t)((i - 1) & 31);
        const uint64_t xh = 0ull - ((rw.x >> sh) & 1u), xl = 0ull - ((rw.y >> sh) & 1u);
        const uint64_t eq = ~((H ^ xh) | (Lw ^ xl)) & V;
        unsigned long long row[NW];
#pragma unroll
        for (int q = 0; q < NW; q++) row[q] = 0;
#pragma unroll
        for (int b = 0; b < W; b++) {
            const int j = i - K + b;
            int val, op;
            if (j <= 0) {
                // F[i][0] = i, reached from above; cells left of column 0 do
                // not exist and are never read
                val = j == 0 ? (i < C ? i : C) : C;
                op = 2;
            } else {
                const int sub = ((eq >> b) & 1u) ? 0 : 1;
                const int d = Fp[b] + sub;
                const int u = (b + 1 < W ? Fp[b + 1] : C) + 1;
                const int l = (b > 0 ? F[b - 1] : C) + 1;
                int m = d < u ? d : u;
                m = m < l ? m : l;
                op = m == d ? sub : (m == u ? 2 : 3);
                val = m < C ? m : C;
            }
            F[b] = val;
            row[b >> 5] |= (unsigned long long)op << (2 * (b & 31));
        }
#pragma unroll
        for (int q = 0; q < NW; q++) bp[((uint64_t)(i - 1) * NW + q) * bstride] = row[q];
#pragma unroll
        for (int b = 0; b < W; b++) Fp[b] = F[b];
    }
    // the least value of the last row over columns 0 <= j <= e + 1, the
    // smallest j first
    const int64_t bmax = e + 1 - n + K;
    int best = -1, bv = C;
#pragma unroll
    for (int b = 0; b < W; b++)
        if (b <= bmax && n - K + b >= 0 && Fp[b] < bv) {
            bv = Fp[b];
            best = b;
        }
    if (best < 0) {  // no alignment of K errors ends at e
        *err = 0xff;
        *start = 0;
        return 0;
    }
    *err = (uint8_t)bv;
    *start = (uint32_t)(e + 1 - (n - K + best));
    if (!want_ops) return 0;
    // the walk from (n, best) back to (0, 0)
    int i = n, b = best, m = 0;
    while (i > 0 || i - K + b > 0) {
        const int op =
            i == 0 ? 3
                   : (int)((bp[((uint64_t)(i - 1) * NW + (b >> 5)) * bstride] >> (2 * (b & 31))) &
                           3u);
        if (o && (uint32_t)m < stride) o[m] = (uint8_t)op;
        m++;
        if (op <= 1) {
            i--;
        } else if (op == 2) {
            i--;
            b++;
        } else {
            b--;
        }
    }
    return m;
}
