// Offset arithmetic of the LSD radix sort (pn_canon.hip), shared by its
// kernels and by a host-side unit test.
//
// The sort keeps, per tile of at most 8192 keys, the count of each 8-bit
// digit (32 bits suffice), and turns them into output offsets by an
// exclusive scan in (digit, tile) order: column sums over groups of tiles,
// a scan of those sums over the groups, then each group's columns again.
// The sums and offsets reach the key count itself, which passes 2^32 for
// the position set of a reference longer than 2^31 bases (both strands),
// so they are 64-bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef PN_ROFF_T
#define PN_ROFF_T uint64_t
#endif
typedef PN_ROFF_T pn_roff;

// groups of tiles scanned by one block each in the column passes
#define PN_RADIX_GROUPS 256

__host__ __device__ inline uint64_t pn_radix_tiles_per_group(uint64_t n_tiles) {
    return (n_tiles + PN_RADIX_GROUPS - 1) / PN_RADIX_GROUPS;
}

// sum of column d of the tile-major counts hist[b][d] over tiles [b0, b1)
__host__ __device__ inline pn_roff pn_radix_col_sum(const uint32_t *hist, uint64_t b0, uint64_t b1,
                                                    uint32_t d) {
    pn_roff acc = 0;
#pragma unroll 8
    for (uint64_t b = b0; b < b1; b++) acc += hist[b * 256 + d];
    return acc;
}

// offsets of column d over tiles [b0, b1): offs[b][d] = run + the counts of
// column d in tiles b0 .. b-1
__host__ __device__ inline void pn_radix_col_down(const uint32_t *hist, uint64_t b0, uint64_t b1,
                                                  uint32_t d, pn_roff run, pn_roff *offs) {
#pragma unroll 8
    for (uint64_t b = b0; b < b1; b++) {
        offs[b * 256 + d] = run;
        run += hist[b * 256 + d];
    }
}
