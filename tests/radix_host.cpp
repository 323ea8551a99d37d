// Host-side driver of the radix sort's offset arithmetic (pn_radix.h): the
// three column passes of pn_canon.hip done with the same functions on the
// CPU, so that the widths of the sums and offsets can be checked on key
// counts past 2^32 without a GPU.  Built twice by the test: with the
// library's offset type and with 32-bit offsets (-DPN_ROFF_T=uint32_t).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "../paper_1403_1706_amd/csrc/pn_radix.h"

extern "C" int radix_offsets_host(const uint32_t *hist, uint64_t n_tiles, uint64_t *offs_out) {
    const uint64_t per = pn_radix_tiles_per_group(n_tiles);
    const uint64_t groups = (n_tiles + per - 1) / per;
    std::vector<pn_roff> colsum(groups * 256), dtot(256), base(256);
    for (uint64_t g = 0; g < groups; g++)
        for (uint32_t d = 0; d < 256; d++)
            colsum[g * 256 + d] =
                pn_radix_col_sum(hist, g * per, std::min(n_tiles, (g + 1) * per), d);
    for (uint32_t d = 0; d < 256; d++) {  // each column over the groups
        pn_roff run = 0;
        for (uint64_t g = 0; g < groups; g++) {
            const pn_roff v = colsum[g * 256 + d];
            colsum[g * 256 + d] = run;
            run += v;
        }
        dtot[d] = run;
    }
    pn_roff run = 0;
    for (uint32_t d = 0; d < 256; d++) {  // digits below each digit
        base[d] = run;
        run += dtot[d];
    }
    std::vector<pn_roff> offs(n_tiles * 256);
    for (uint64_t g = 0; g < groups; g++)
        for (uint32_t d = 0; d < 256; d++)
            pn_radix_col_down(hist, g * per, std::min(n_tiles, (g + 1) * per), d,
                              colsum[g * 256 + d] + base[d], offs.data());
    for (uint64_t i = 0; i < n_tiles * 256; i++) offs_out[i] = (uint64_t)offs[i];
    return (int)sizeof(pn_roff);
}
