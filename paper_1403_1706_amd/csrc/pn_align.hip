// Start positions and alignments of hits, one thread per hit; the per-hit
// recurrence and walk are in pn_align.h.
#include "pn_align.h"

namespace {

constexpr int kAlignThreads = 64;

// The launch covers the hits of one error count K.  hw: the chunk's hit
// records (3 words each: read, end, strand | errors << 8); perm: the
// chunk-local indices of this launch's hits; bp: cnt words per op-code word
// of a row (pn_align_row_words(K) of them per row).
template <int K>
__global__ __launch_bounds__(kAlignThreads) void k_align(PnRefDev ref, PnIndexDev ix,
                                                         const uint32_t *__restrict__ hw,
                                                         const uint32_t *__restrict__ perm,
                                                         uint32_t cnt,
                                                         unsigned long long *__restrict__ bp,
                                                         uint32_t *__restrict__ starts,
                                                         uint8_t *__restrict__ errs,
                                                         uint8_t *__restrict__ ops,
                                                         uint32_t stride,
                                                         uint16_t *__restrict__ n_ops) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const uint32_t h = perm[t];
    const uint32_t r = hw[3 * (uint64_t)h], s = hw[3 * (uint64_t)h + 2] & 0xffu;
    const int64_t e = hw[3 * (uint64_t)h + 1];
    const int n = (int)(ix.offsets[r + 1] - ix.offsets[r]);
    uint32_t st;
    uint8_t er;
    const int m = pn_align_one<K>(s ? ref.planes[0] : ref.planes[1],
                                  ix.rplanes_rc + (uint64_t)r * PN_READ_WORDS, n, e, ref.L,
                                  bp + t, cnt, n_ops != nullptr,
                                  ops ? ops + (uint64_t)h * stride : nullptr, stride, &st, &er);
    starts[h] = st;
    errs[h] = er;
    if (n_ops) n_ops[h] = (uint16_t)m;
}

template <int K>
void launch_k(const PnRefDev &ref, const PnIndexDev &ix, const uint32_t *hw, const uint32_t *perm,
              uint32_t cnt, unsigned long long *bp, uint32_t *starts, uint8_t *errs, uint8_t *ops,
              uint32_t stride, uint16_t *n_ops, hipStream_t st) {
    hipLaunchKernelGGL(k_align<K>, dim3((cnt + kAlignThreads - 1) / kAlignThreads),
                       dim3(kAlignThreads), 0, st, ref, ix, hw, perm, cnt, bp, starts, errs, ops,
                       stride, n_ops);
}

}  // namespace

namespace pn {

static_assert(PN_MAX_K == 31, "one instance per error count 0 .. PN_MAX_K");

void launch_align(const PnRefDev &ref, const PnIndexDev &ix, int v, const uint32_t *hw,
                  const uint32_t *perm, uint32_t cnt, unsigned long long *bp, uint32_t *starts,
                  uint8_t *errs, uint8_t *ops, uint32_t stride, uint16_t *n_ops, hipStream_t st) {
    if (!cnt) return;
    switch (v) {
#define PN_ALIGN_CASE(k) \
    case k: launch_k<k>(ref, ix, hw, perm, cnt, bp, starts, errs, ops, stride, n_ops, st); break;
        PN_ALIGN_CASE(0) PN_ALIGN_CASE(1) PN_ALIGN_CASE(2) PN_ALIGN_CASE(3)
        PN_ALIGN_CASE(4) PN_ALIGN_CASE(5) PN_ALIGN_CASE(6) PN_ALIGN_CASE(7)
        PN_ALIGN_CASE(8) PN_ALIGN_CASE(9) PN_ALIGN_CASE(10) PN_ALIGN_CASE(11)
        PN_ALIGN_CASE(12) PN_ALIGN_CASE(13) PN_ALIGN_CASE(14) PN_ALIGN_CASE(15)
        PN_ALIGN_CASE(16) PN_ALIGN_CASE(17) PN_ALIGN_CASE(18) PN_ALIGN_CASE(19)
        PN_ALIGN_CASE(20) PN_ALIGN_CASE(21) PN_ALIGN_CASE(22) PN_ALIGN_CASE(23)
        PN_ALIGN_CASE(24) PN_ALIGN_CASE(25) PN_ALIGN_CASE(26) PN_ALIGN_CASE(27)
        PN_ALIGN_CASE(28) PN_ALIGN_CASE(29) PN_ALIGN_CASE(30) PN_ALIGN_CASE(31)
#undef PN_ALIGN_CASE
        default: break;
    }
}

}  // namespace pn
