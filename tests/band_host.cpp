// Host-side driver of the verification device code (pn_band.h): lays out a
// text and a read the way the library does (padded bit planes, read plane
// words) and runs pn_band_verify on the CPU, so the band recurrence can be
// checked against the oracle without a GPU.
#include <cstdint>
#include <vector>

#include "../paper_1403_1706_amd/csrc/pn_band.h"

extern "C" int band_host(const uint8_t *text, uint64_t L, const uint8_t *read, int n, int64_t d,
                         int k, int32_t *out_e, int32_t *out_v) {
    if (n < 1 || n > PN_MAX_READ_LEN || k < 0 || k > PN_MAX_K) return -1;
    const uint64_t nb = (L + 31) / 32 + 2 * PN_PAD_BLOCKS + 16;
    std::vector<uint4> pl(nb, make_uint4(0, 0, 0, 0));
    for (uint64_t t = 0; t < L; t++) {
        uint64_t B = t / 32 + PN_PAD_BLOCKS;
        uint32_t b = (uint32_t)(t % 32);
        pl[B].x |= (uint32_t)(text[t] >> 1) << b;
        pl[B].y |= (uint32_t)(text[t] & 1) << b;
        pl[B].z |= 1u << b;
    }
    std::vector<uint2> rp(PN_READ_WORDS, make_uint2(0, 0));
    for (int o = 0; o < n; o++) {
        rp[o / 32].x |= (uint32_t)(read[o] >> 1) << (o % 32);
        rp[o / 32].y |= (uint32_t)(read[o] & 1) << (o % 32);
    }
    // the kernel's two passes: at most 16 rows first, then (if the candidate
    // is still alive there) from row 0 without a cap
    int m = 0;
    auto emit = [&](uint32_t e, int v) {
        out_e[m] = (int32_t)e;
        out_v[m] = v;
        m++;
    };
    if (pn_band_verify(pl.data(), rp.data(), n, k, d - k, L, 16, emit) < 0) {
        if (m != 0) return -2;  // a capped run must not have emitted
        pn_band_verify(pl.data(), rp.data(), n, k, d - k, L, PN_MAX_READ_LEN, emit);
    }
    return m;
}
