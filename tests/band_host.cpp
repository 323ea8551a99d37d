// Host-side driver of the verification device code (pn_band.h): lays out a
// text and a read the way the library does (padded bit planes, read plane
// words) and runs pn_band_verify on the CPU, so the band recurrence can be
// checked against the oracle without a GPU.
#include <cstdint>
#include <vector>

#include "../paper_1403_1706_amd/csrc/pn_align.h"

namespace {

// padded bit planes of a text; with rc, of its reverse complement
std::vector<uint4> text_planes(const uint8_t *text, uint64_t L, bool rc) {
    const uint64_t nb = (L + 31) / 32 + 2 * PN_PAD_BLOCKS + 16;
    std::vector<uint4> pl(nb, make_uint4(0, 0, 0, 0));
    for (uint64_t t = 0; t < L; t++) {
        const uint32_t c = rc ? 3u - text[L - 1 - t] : text[t];
        uint64_t B = t / 32 + PN_PAD_BLOCKS;
        uint32_t b = (uint32_t)(t % 32);
        pl[B].x |= (c >> 1) << b;
        pl[B].y |= (c & 1u) << b;
        pl[B].z |= 1u << b;
    }
    return pl;
}

std::vector<uint2> read_planes(const uint8_t *read, int n, bool rc) {
    std::vector<uint2> rp(PN_READ_WORDS, make_uint2(0, 0));
    for (int o = 0; o < n; o++) {
        const uint32_t c = rc ? 3u - read[n - 1 - o] : read[o];
        rp[o / 32].x |= (c >> 1) << (o % 32);
        rp[o / 32].y |= (c & 1u) << (o % 32);
    }
    return rp;
}

}  // namespace

// The kernel's protocol for one candidate: a first pass of at most 16 rows,
// then (if the candidate is still alive there) from row 0 without a cap.
// With tail != 0 the first pass is the tail check instead: 16 rows of the
// read's reverse complement against the text's reverse complement on the
// mirrored diagonal L - n - d; the forward run follows if it survives.
// Returns the number of hits written, or -3 when the tail check dropped
// the candidate.
extern "C" int band_host(const uint8_t *text, uint64_t L, const uint8_t *read, int n, int64_t d,
                         int k, int tail, int32_t *out_e, int32_t *out_v) {
    if (n < 1 || n > PN_MAX_READ_LEN || k < 0 || k > PN_MAX_K) return -1;
    const std::vector<uint4> pl = text_planes(text, L, false);
    const std::vector<uint2> rp = read_planes(read, n, false);
    int m = 0;
    auto emit = [&](uint32_t e, int v) {
        out_e[m] = (int32_t)e;
        out_v[m] = v;
        m++;
    };
    if (k > PN_BAND_K) {
        // the 64-bit band pass: from row 0 to the end, no first pass
        pn_band_verify_wide(pl.data(), rp.data(), n, k, d - k, L, emit);
        return m;
    }
    if (tail) {
        const std::vector<uint4> plr = text_planes(text, L, true);
        const std::vector<uint2> rpr = read_planes(read, n, true);
        auto none = [&](uint32_t, int) {};
        const int64_t lo = (int64_t)L - n - d - k;
        const int rw = pn_band_verify(plr.data(), rpr.data(), n, k, lo, L, 16, none);
        if (rw > 0 && rw < n) return -3;
        pn_band_verify(pl.data(), rp.data(), n, k, d - k, L, PN_MAX_READ_LEN, emit);
        return m;
    }
    if (pn_band_verify(pl.data(), rp.data(), n, k, d - k, L, 16, emit) < 0) {
        if (m != 0) return -2;  // a capped run must not have emitted
        pn_band_verify(pl.data(), rp.data(), n, k, d - k, L, PN_MAX_READ_LEN, emit);
    }
    return m;
}

// The count filter's per-candidate code (pn_count_pieces) on the host:
// 1 when the candidate is kept for the band pass, 0 when dropped.
extern "C" int count_host(const uint8_t *text, uint64_t L, const uint8_t *read, int n, int64_t d,
                          int k) {
    if (n < 1 || n > PN_MAX_READ_LEN || k < 0 || k > PN_MAX_K) return -1;
    if (k > PN_BAND_K) return 1;  // the kernel hands such bands to the band pass uncounted
    const std::vector<uint4> pl = text_planes(text, L, false);
    const std::vector<uint2> rp = read_planes(read, n, false);
    PnBandHead hd;
    pn_band_load(pl.data(), rp.data(), d - k, hd);
    int letters = 0;
    const bool inside = d - k >= 0 && d - k + n + 2 * k < (int64_t)L;
    const bool keep = inside ? pn_count_pieces<true>(hd, pl.data(), rp.data(), n, k, d - k, letters)
                             : pn_count_pieces<false>(hd, pl.data(), rp.data(), n, k, d - k, letters);
    if (inside) {
        // the H/L-only form the kernel runs for bands inside the reference
        const uint2 *hl = (const uint2 *)pl.data();
        const uint64_t blk = (uint64_t)(d - k + PN_PAD_POS) >> 5;
        int l2 = 0;
        const bool k2 = pn_count_pieces_hl(hl[2 * blk], hl[2 * (blk + 1)], hl[2 * (blk + 2)],
                                           hl[2 * (blk + 3)], rp[0], hl, rp.data(), n, k, d - k, l2);
        if (k2 != keep || l2 != letters) return -2;
    }
    return keep ? 1 : 0;
}

// The count filter's backward order on the host, from the per-word code
// the kernel runs (pn_count_word_hl): the whole read words from the last
// one down to the first, the pieces past the last whole word taken as
// found; for a band inside the reference.  1: kept, 0: dropped, -1: bad
// arguments, -3: outside the reference or fewer than two whole words (the
// kernel counts those forwards).  *words: read words examined.
extern "C" int count_host_backward(const uint8_t *text, uint64_t L, const uint8_t *read, int n,
                                   int64_t d, int k, int *words) {
    if (n < 1 || n > PN_MAX_READ_LEN || k < 0 || k > PN_BAND_K) return -1;
    const int m = n / kPnPiece, wf = m / 8, need = m - k;
    const int64_t lo = d - k;
    if (wf < 2 || !(lo >= 0 && lo + n + 2 * k < (int64_t)L)) return -3;
    *words = 0;
    if (need <= 0) return 1;
    const std::vector<uint4> pl = text_planes(text, L, false);
    const std::vector<uint2> rp = read_planes(read, n, false);
    const uint2 *hl = (const uint2 *)pl.data();
    const uint64_t tp = (uint64_t)(lo + PN_PAD_POS);
    const uint64_t blk = tp >> 5;
    const uint32_t ph = (uint32_t)(tp & 31);
    int found = 0, left = m;
    for (int w = wf - 1; w >= 0; w--) {
        const uint32_t F = pn_count_word_hl(hl[2 * (blk + w)], hl[2 * (blk + w + 1)],
                                            hl[2 * (blk + w + 2)], rp[w], ph, 2 * k + 1);
        found += __builtin_popcount(F & pn_piece_firsts(8));
        left -= 8;
        (*words)++;
        if (found >= need) return 1;
        if (found + left < need) return 0;
    }
    return 1;  // the pieces past the last whole word could make up the rest
}

// The alignment code (pn_align_one) on the host for one hit on `text` (the
// strand's own letters) ending at e with v errors: the other strand's planes
// are those of the text's reverse complement, the read's are those of its
// reverse complement.  Returns the number of ops, with *start and *err.
template <int K>
static int align_k(const std::vector<uint4> &pl, const std::vector<uint2> &rp, int n, uint64_t e,
                   uint64_t L, uint32_t *start, uint8_t *err, uint8_t *ops, uint32_t stride) {
    std::vector<unsigned long long> bp(((size_t)n + 1) * pn_align_row_words(K));
    return pn_align_one<K>(pl.data(), rp.data(), n, (int64_t)e, L, bp.data(), 1, true, ops, stride,
                           start, err);
}

extern "C" int align_host(const uint8_t *text, uint64_t L, const uint8_t *read, int n, uint64_t e,
                          int v, uint32_t *start, uint8_t *err, uint8_t *ops, uint32_t stride) {
    if (n < 1 || n > PN_MAX_READ_LEN || v < 0 || v > PN_MAX_K || e >= L) return -1;
    const std::vector<uint4> pl = text_planes(text, L, true);
    const std::vector<uint2> rp = read_planes(read, n, true);
    switch (v) {
#define ALIGN_CASE(k) \
    case k: return align_k<k>(pl, rp, n, e, L, start, err, ops, stride);
        ALIGN_CASE(0) ALIGN_CASE(1) ALIGN_CASE(2) ALIGN_CASE(3) ALIGN_CASE(4) ALIGN_CASE(5)
        ALIGN_CASE(6) ALIGN_CASE(7) ALIGN_CASE(8) ALIGN_CASE(9) ALIGN_CASE(10) ALIGN_CASE(11)
        ALIGN_CASE(12) ALIGN_CASE(13) ALIGN_CASE(14) ALIGN_CASE(15) ALIGN_CASE(16) ALIGN_CASE(17)
        ALIGN_CASE(18) ALIGN_CASE(19) ALIGN_CASE(20) ALIGN_CASE(21) ALIGN_CASE(22) ALIGN_CASE(23)
        ALIGN_CASE(24) ALIGN_CASE(25) ALIGN_CASE(26) ALIGN_CASE(27) ALIGN_CASE(28) ALIGN_CASE(29)
        ALIGN_CASE(30) ALIGN_CASE(31)
#undef ALIGN_CASE
    }
    return -1;
}
