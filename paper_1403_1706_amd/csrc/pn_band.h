// Per-candidate banded bit-parallel semiglobal edit distance (Section 3.3),
// shared by the verification kernel and by a host-side check of the same
// code.  See pn_verify.hip for the recurrence and its band conventions.
#pragma once

#include "pn_internal.h"

// bits [sh, sh+32) of the 64-bit value hi:lo (0 <= sh < 32)
__host__ __device__ __forceinline__ uint32_t pn_funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, sh);
#else
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
#endif
}

// Verify one candidate.  `pl`: the strand's padded bit planes; `rp`: the
// read's PN_READ_WORDS plane words; the band covers diagonals [lo, lo + 2k]
// (lo = d - k); 1 <= len <= PN_MAX_READ_LEN; 0 <= k <= PN_BAND_K.  Calls
// emit(end, value) for every end column of the last row with value <= k,
// and returns the number of rows computed.  A candidate still alive after
// row_cap rows (a multiple of 8, below len) stops there without emitting
// and -row_cap is returned; the caller runs it again from row 0 without cap.
// The first memory words a candidate needs: plane blocks blk .. blk+3 of
// its stream and the read's first plane word.  Loading them is separate so
// that a kernel can issue one candidate's loads while it computes another.
struct PnBandHead {
    uint4 A, B, C, Dn;
    uint2 rw0;
};

__host__ __device__ __forceinline__ void pn_band_load(const uint4 *__restrict__ pl,
                                                      const uint2 *__restrict__ rp, int64_t lo,
                                                      PnBandHead &h) {
    const uint64_t blk = (uint64_t)(lo + PN_PAD_POS) >> 5;
    h.A = pl[blk];
    h.B = pl[blk + 1];
    h.C = pl[blk + 2];
    h.Dn = pl[blk + 3];
    h.rw0 = rp[0];
}

// The band's state between rows: the candidate's stream of plane words
// (word m covers reference positions [lo + 32m, lo + 32m + 32); h0/l0/v0 the
// current word, h1/l1/v1 the next), the row's differences VP/VN and the count
// Ck of the right-most cell (see below).
struct PnBandState {
    uint32_t h0, l0, v0, h1, l1, v1;
    uint32_t VP, VN;
    int Ck;
};

// Rows 32m+1 .. 32m+32 (read plane word rw).  Returns 0 to go on with the
// next word, else the value pn_band_run returns.  kLast = false: no row of
// this word is the read's last (the caller knows len > 32m + 32).
template <bool kLast, typename Emit>
__host__ __device__ __forceinline__ int pn_band_word(PnBandState &s, uint2 rw, int m, int len,
                                                     int k, int64_t lo, uint64_t L, int row_cap,
                                                     Emit &emit) {
    const int W = 2 * k + 1;
    const uint32_t M = (1u << W) - 1u;
    const uint32_t M2 = M & ~1u;
    const uint32_t TOP = 1u << (W - 1);
#pragma unroll
    for (int t = 0; t < 32; t++) {
        const int i = 32 * m + t + 1;  // row i compares read letter i-1
        const uint32_t H = pn_funnel(s.h1, s.h0, t), Lw = pn_funnel(s.l1, s.l0, t),
                       V = pn_funnel(s.v1, s.v0, t);
        // all ones where read letter i-1 has a 1 bit (a sign-extended bit field)
        const uint32_t xh = (uint32_t)((int32_t)(rw.x << (31 - t)) >> 31),
                       xl = (uint32_t)((int32_t)(rw.y << (31 - t)) >> 31);
        const uint32_t Eq = ~((H ^ xh) | (Lw ^ xl)) & V & M;
        uint32_t VP = (s.VP >> 1) | TOP;  // previous row's differences, moved into this row's frame
        uint32_t VN = s.VN >> 1;
        const uint32_t Xv = Eq | VN;
        const uint32_t Xh = (((Eq & VP) + VP) ^ VP) | Eq;
        uint32_t HP = VN | ~(Xh | VP);
        uint32_t HN = VP & Xh;
        s.Ck += (int)((HN >> (W - 1)) & 1u);
        HP = (HP << 1) | 1u;
        HN <<= 1;
        s.VP = VP = HN | ~(Xv | HP);
        s.VN = VN = HP & Xv;
        if (kLast && i == len) {
            // last row: cell b holds R minus the differences to its right
            int v = i + k - s.Ck;
            for (int b = W - 1; b >= 0; b--) {
                const int64_t c = (int64_t)len + lo + b;
                if (c >= 1 && c <= (int64_t)L && v <= k) emit((uint32_t)(c - 1), v);
                v -= (int)((VP >> b) & 1u) - (int)((VN >> b) & 1u);
            }
            return i;
        }
        // stop when the whole row is above k: R minus the +1 steps bounds
        // the row minimum from below (R - popcount > k), written as one
        // accumulating bit count and a compare
        if (__builtin_popcount(VP & M2) + s.Ck < i) return i;
        if ((t & 7) == 7 && t != 31 && i == row_cap) return -i;  // a cap inside a word
    }
    return 0;
}

// kLast = false: the caller knows that len > row_cap, so no row is the last.
// no_end: no row below it is the read's last (a bound the caller may know
// for a whole wave; words entirely below it skip the last-row test).
template <bool kLast = true, typename Emit>
__host__ __device__ __forceinline__ int pn_band_run(const PnBandHead &hd,
                                                    const uint4 *__restrict__ pl,
                                                    const uint2 *__restrict__ rp, int len, int k,
                                                    int64_t lo, uint64_t L, int row_cap,
                                                    Emit &&emit, int no_end = 0) {
    const uint64_t tp = (uint64_t)(lo + PN_PAD_POS);
    const uint64_t blk = tp >> 5;
    const uint32_t ph = (uint32_t)(tp & 31);
    const uint4 A = hd.A, B = hd.B;
    uint4 C = hd.C, Dn = hd.Dn;
    PnBandState s;
    s.h0 = pn_funnel(B.x, A.x, ph);
    s.l0 = pn_funnel(B.y, A.y, ph);
    s.v0 = pn_funnel(B.z, A.z, ph);
    s.h1 = pn_funnel(C.x, B.x, ph);
    s.l1 = pn_funnel(C.y, B.y, ph);
    s.v1 = pn_funnel(C.z, B.z, ph);
    s.VP = s.VN = 0;  // row 0: every band cell is 0 (free start)
    // The right-most band cell of row i holds R = i - (number of rows whose
    // step left it unchanged, i.e. moved a -1 difference out of the band's
    // top bit); Ck counts those rows plus k, so that R = i + k - Ck.
    s.Ck = k;
    uint2 rw_next = hd.rw0;  // the read's plane word for the next 32 rows, loaded a word ahead
    for (int m = 0;; m++) {
        const uint2 rw = rw_next;
        if (32 * (m + 1) < len && 32 * (m + 1) < row_cap) rw_next = rp[m + 1];
        const int r = !kLast || 32 * (m + 1) < no_end
                          ? pn_band_word<false>(s, rw, m, len, k, lo, L, row_cap, emit)
                          : pn_band_word<kLast>(s, rw, m, len, k, lo, L, row_cap, emit);
        if (r) return r;
        if (32 * (m + 1) >= row_cap) return -32 * (m + 1);
        // advance the stream by 32 positions
        s.h0 = s.h1;
        s.l0 = s.l1;
        s.v0 = s.v1;
        s.h1 = pn_funnel(Dn.x, C.x, ph);
        s.l1 = pn_funnel(Dn.y, C.y, ph);
        s.v1 = pn_funnel(Dn.z, C.z, ph);
        C = Dn;
        Dn = pl[blk + m + 4];
    }
}

// one candidate start to finish (loads, then rows)
template <typename Emit>
__host__ __device__ __forceinline__ int pn_band_verify(const uint4 *__restrict__ pl,
                                                       const uint2 *__restrict__ rp, int len, int k,
                                                       int64_t lo, uint64_t L, int row_cap,
                                                       Emit &&emit) {
    PnBandHead hd;
    pn_band_load(pl, rp, lo, hd);
    return pn_band_run(hd, pl, rp, len, k, lo, L, row_cap, emit);
}

// The same recurrence for PN_BAND_K < k <= PN_MAX_K: the band's 2k + 1 <= 63
// diagonals in one 64-bit word, row by row from row 0 to the end (no cap,
// no tail check).  Row i compares read letter i - 1 with the text from
// position lo + i - 1 on; the four plane blocks the window needs advance by
// one block every 32 rows.  Calls emit(end, value) like pn_band_run and returns
// the number of rows computed.
template <typename Emit>
__host__ __device__ inline int pn_band_verify_wide(const uint4 *__restrict__ pl,
                                                   const uint2 *__restrict__ rp, int len, int k,
                                                   int64_t lo, uint64_t L, Emit &&emit) {
    const int W = 2 * k + 1;
    const uint64_t M = (1ull << W) - 1ull;
    const uint64_t M2 = M & ~1ull;
    const uint64_t TOP = 1ull << (W - 1);
    const uint64_t tp = (uint64_t)(lo + PN_PAD_POS);
    uint64_t blk = tp >> 5;
    const uint32_t ph = (uint32_t)(tp & 31);
    uint4 A = pl[blk], B = pl[blk + 1], C = pl[blk + 2], D = pl[blk + 3];
    uint64_t VP = 0, VN = 0;  // row 0: every band cell is 0 (free start)
    int Ck = k;               // as in pn_band_run: R = i + k - Ck
    uint2 rw = rp[0];
    for (int i = 1; i <= len; i++) {
        const uint32_t t = (uint32_t)(i - 1) & 31u;  // (ph + i - 1) - 32 * (blocks advanced)
        const uint32_t sh = ph + t;
        // bits [sh, sh + 64) of the blocks A .. D (sh < 63)
        const uint32_t s0 = sh & 31u;
        const bool up = sh >= 32;
        const uint4 a0 = up ? B : A, a1 = up ? C : B, a2 = up ? D : C;
        const uint32_t a0x = a0.x, a1x = a1.x, a2x = a2.x;
        const uint32_t a0y = a0.y, a1y = a1.y, a2y = a2.y;
        const uint32_t a0z = a0.z, a1z = a1.z, a2z = a2.z;
        const uint64_t H = (uint64_t)pn_funnel(a1x, a0x, s0) | ((uint64_t)pn_funnel(a2x, a1x, s0) << 32);
        const uint64_t Lw = (uint64_t)pn_funnel(a1y, a0y, s0) | ((uint64_t)pn_funnel(a2y, a1y, s0) << 32);
        const uint64_t V = (uint64_t)pn_funnel(a1z, a0z, s0) | ((uint64_t)pn_funnel(a2z, a1z, s0) << 32);
        const uint64_t xh = 0ull - (uint64_t)((rw.x >> t) & 1u);
        const uint64_t xl = 0ull - (uint64_t)((rw.y >> t) & 1u);
        const uint64_t Eq = ~((H ^ xh) | (Lw ^ xl)) & V & M;
        uint64_t vp = (VP >> 1) | TOP;
        uint64_t vn = VN >> 1;
        const uint64_t Xv = Eq | vn;
        const uint64_t Xh = (((Eq & vp) + vp) ^ vp) | Eq;
        uint64_t HP = vn | ~(Xh | vp);
        uint64_t HN = vp & Xh;
        Ck += (int)((HN >> (W - 1)) & 1ull);
        HP = (HP << 1) | 1ull;
        HN <<= 1;
        VP = HN | ~(Xv | HP);
        VN = HP & Xv;
        if (i == len) {
            int v = i + k - Ck;
            for (int b = W - 1; b >= 0; b--) {
                const int64_t c = (int64_t)len + lo + b;
                if (c >= 1 && c <= (int64_t)L && v <= k) emit((uint32_t)(c - 1), v);
                v -= (int)((VP >> b) & 1ull) - (int)((VN >> b) & 1ull);
            }
            return i;
        }
        if (__builtin_popcountll(VP & M2) + Ck < i) return i;
        if (t == 31) {
            // the next 32 rows: the next read word, the window one block on
            rw = rp[i >> 5];
            blk++;
            A = B;
            B = C;
            C = D;
            D = pl[blk + 3];
        }
    }
    return len;
}

// Count filter (the q-gram lemma of Section 2.2, with the read cut into its
// m = floor(n / 4) disjoint pieces of 4 letters): an edit falls into one
// piece at most (a deletion between two pieces breaks neither), so an
// alignment with at most k errors leaves at least m - k pieces exact, each
// on one diagonal of the alignment; every cell of an alignment through the
// candidate's diagonal d lies within k diagonals of d, so those pieces
// match the text exactly on diagonals of the band [d - k, d + k].
//
// The read is taken 32 letters (8 pieces) at a time and the band one
// diagonal at a time: on diagonal b the match bits of all 32 letters are
// one word, ~((H_b ^ xH) | (L_b ^ xL)) with H_b, L_b the text planes from
// position lo + 32 w + b, and a piece is exact there when its 4 bits are
// all set (two shift-and steps leave that at the piece's first bit).  OR
// over the 2k + 1 diagonals and a population count give the pieces of the
// word found somewhere in the band: about 8 operations per diagonal for 32
// letters, against 8 per letter row by row.  The candidate is dropped as
// soon as the pieces found plus those unchecked fall below m - k, and kept
// once m - k are found (decisions at word ends; the outcome is the same as
// piece by piece).  Short pieces decide sooner against a diverged copy (a
// 4-letter piece of a copy at 72 % identity is exact a quarter of the
// time) while a chance match on one of the band's 2k + 1 diagonals stays
// rare (2k + 1 in 256).  kInside: every band position of the wave's
// candidates lies in [0, L) (no validity plane).  `letters`: 32 per word
// examined (the letters one diagonal-major step covers).
constexpr int kPnPiece = 4;

template <bool kInside>
__host__ __device__ __forceinline__ bool pn_count_pieces(const PnBandHead &hd, const uint4 *__restrict__ pl,
                                             const uint2 *__restrict__ rp, int len, int k,
                                             int64_t lo, int &letters) {
    const int m = len / kPnPiece;
    const int need = m - k;
    letters = 0;
    if (need <= 0) return true;
    const int W = 2 * k + 1;
    const uint64_t tp = (uint64_t)(lo + PN_PAD_POS);
    const uint64_t blk = tp >> 5;
    const uint32_t ph = (uint32_t)(tp & 31);
    uint4 A = hd.A, B = hd.B, C = hd.C, Dn = hd.Dn;
    uint2 rw = hd.rw0;
    int found = 0;
    for (int w = 0;; w++) {
        const int left = m - 8 * w;  // pieces from this word on
        const uint2 rwn = left > 8 ? rp[w + 1] : rw;
        // the 64 text letters from lo + 32 w
        const uint32_t h0 = pn_funnel(B.x, A.x, ph), h1 = pn_funnel(C.x, B.x, ph);
        const uint32_t l0 = pn_funnel(B.y, A.y, ph), l1 = pn_funnel(C.y, B.y, ph);
        uint32_t v0 = 0, v1 = 0;
        if (!kInside) {
            v0 = pn_funnel(B.z, A.z, ph);
            v1 = pn_funnel(C.z, B.z, ph);
        }
        uint32_t F = 0;
        for (int b = 0; b < W; b++) {
            const uint32_t H = pn_funnel(h1, h0, (uint32_t)b), Lw = pn_funnel(l1, l0, (uint32_t)b);
            uint32_t eq = ~((H ^ rw.x) | (Lw ^ rw.y));
            if (!kInside) eq &= pn_funnel(v1, v0, (uint32_t)b);
            const uint32_t y = eq & (eq >> 1);
            F |= y & (y >> 2);
        }
        const uint32_t firsts =
            left >= 8 ? 0x11111111u : (0x11111111u & ((1u << (4 * left)) - 1u));
        found += __builtin_popcount(F & firsts);
        const int now = left < 8 ? left : 8;
        letters += 32;
        const int unchecked = left - now;
        if (found >= need) return true;
        if (found + unchecked < need) return false;
        // the next 32 letters: advance the text stream by 32 positions
        A = B;
        B = C;
        C = Dn;
        Dn = pl[blk + w + 4];
        rw = rwn;
    }
}

// The pieces of one 32-letter read word (plane words rw) found on some
// diagonal of the band, at each piece's first bit, for a band inside the
// reference: A, B, C are the H and L words of the word's plane blocks
// (letters from lo + 32 w on, phase ph inside block A), W = 2k + 1.
__host__ __device__ __forceinline__ uint32_t pn_count_word_hl(uint2 A, uint2 B, uint2 C, uint2 rw,
                                                              uint32_t ph, int W) {
    const uint32_t h0 = pn_funnel(B.x, A.x, ph), h1 = pn_funnel(C.x, B.x, ph);
    const uint32_t l0 = pn_funnel(B.y, A.y, ph), l1 = pn_funnel(C.y, B.y, ph);
    uint32_t F = 0;
    for (int b = 0; b < W; b++) {
        const uint32_t H = pn_funnel(h1, h0, (uint32_t)b), Lw = pn_funnel(l1, l0, (uint32_t)b);
        const uint32_t eq = ~((H ^ rw.x) | (Lw ^ rw.y));
        const uint32_t y = eq & (eq >> 1);
        F |= y & (y >> 2);
    }
    return F;
}

// the first bits of the pieces of a word that has `left` pieces from it on
__host__ __device__ __forceinline__ uint32_t pn_piece_firsts(int left) {
    return left >= 8 ? 0x11111111u : (0x11111111u & ((1u << (4 * left)) - 1u));
}

// The same count for a band that lies inside the reference, from the H and
// L words of the plane blocks only (V is all ones there): `hl` is the
// planes read as uint2 (block i's H, L at hl[2 i]), A..Dn the blocks
// blk .. blk + 3 of the candidate's stream.
__host__ __device__ __forceinline__ bool pn_count_pieces_hl(uint2 A, uint2 B, uint2 C, uint2 Dn,
                                                            uint2 rw0,
                                                            const uint2 *__restrict__ hl,
                                                            const uint2 *__restrict__ rp, int len,
                                                            int k, int64_t lo, int &letters) {
    const int m = len / kPnPiece;
    const int need = m - k;
    letters = 0;
    if (need <= 0) return true;
    const int W = 2 * k + 1;
    const uint64_t tp = (uint64_t)(lo + PN_PAD_POS);
    const uint64_t blk = tp >> 5;
    const uint32_t ph = (uint32_t)(tp & 31);
    uint2 rw = rw0;
    int found = 0;
    for (int w = 0;; w++) {
        const int left = m - 8 * w;
        const uint2 rwn = left > 8 ? rp[w + 1] : rw;
        const uint32_t F = pn_count_word_hl(A, B, C, rw, ph, W);
        found += __builtin_popcount(F & pn_piece_firsts(left));
        const int now = left < 8 ? left : 8;
        letters += 32;
        if (found >= need) return true;
        if (found + (left - now) < need) return false;
        A = B;
        B = C;
        C = Dn;
        Dn = hl[2 * (blk + w + 4)];
        rw = rwn;
    }
}
