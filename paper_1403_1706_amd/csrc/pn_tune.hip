// Autotuning of the index parameters for a read batch: q (Section 2.2; a
// larger q gives fewer random q-gram hits but a weaker lemma) and the group
// width w of I (Section 2.2, GROUPBIT/GROUPRANK).  Every candidate that the
// q-gram lemma admits for every read of the batch is timed (build + map,
// best of a few runs) on the batch's first m and first m/2 reads.  A mapping
// costs a part that does not depend on the reads (the scan of the
// reference) plus a part per read (index, candidates, verification), so the
// two times give a line that is evaluated at the whole batch; the fastest
// prediction wins.  The hit list does not depend on the choice (the filter
// is lossless for every admitted q), so the tuner only changes time.
#include <algorithm>
#include <chrono>
#include <vector>

#include "pn_runtime.h"

namespace {

// largest q with (k_r + 1) q <= n_r for every read: min over reads of
// floor(n_r / (k_r + 1))
__global__ void k_batch_qmax(const uint64_t *__restrict__ offsets, uint32_t n_reads, int kglob,
                             const uint8_t *__restrict__ kpr, uint32_t *qmax) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = 0xffffffffu;
    if (r < n_reads) {
        const uint64_t n = offsets[r + 1] - offsets[r];
        const uint32_t k = kglob >= 0 ? (uint32_t)kglob : kpr[r];
        v = (uint32_t)std::min<uint64_t>(n / (k + 1), 0xffffffffull);
    }
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    if ((threadIdx.x & 63) == 0 && v != 0xffffffffu) atomicMin(qmax, v);
}

// the calling thread's current device, restored on scope exit
struct KeepDevice {
    int prev = 0;
    KeepDevice() { (void)hipGetDevice(&prev); }
    ~KeepDevice() { (void)hipSetDevice(prev); }
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int pn_autotune(pn_ctx *ctx, const pn_ref *ref, const char *d_reads, const uint64_t *d_offsets,
                uint32_t n_reads, uint64_t n_bases, int k, const uint8_t *d_k_per_read,
                pn_mode mode, uint32_t sample_reads, pn_tune_result *results, int *n_results,
                int *best_q, int *best_w) {
    if (!ctx || !ref || !n_results || !best_q || !best_w || !results) return PN_EINVAL;
    if (!n_reads || !d_offsets || !d_reads || (k < 0 && !d_k_per_read) || k > PN_MAX_K)
        return PN_EINVAL;
    if (mode != PN_ALL_HITS && mode != PN_BEST_STRATUM) return PN_EINVAL;
    void *sv = nullptr;
    int rc = pn_ctx_stream(ctx, &sv);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)sv;
    KeepDevice keep;
    if (hipSetDevice(pnrt::ctx_device(ctx)) != hipSuccess) return PN_EDEVICE;
    // q admitted by the lemma for the whole batch
    uint32_t *d_qmax = nullptr;
    if (hipMalloc((void **)&d_qmax, 4) != hipSuccess) return PN_ENOMEM;
    uint32_t qmax = 0xffffffffu;
    hipError_t e = hipMemcpyAsync(d_qmax, &qmax, 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_batch_qmax, dim3((n_reads + 255) / 256), dim3(256), 0, st, d_offsets,
                           n_reads, k, d_k_per_read, d_qmax);
        e = hipMemcpyAsync(&qmax, d_qmax, 4, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_qmax);
    if (e != hipSuccess) return PN_EDEVICE;
    // the sample: the batch's first m reads, whose letters end at offsets[m]
    const uint32_t m = std::max<uint32_t>(1, std::min(sample_reads ? sample_reads : n_reads, n_reads));
    uint64_t sample_bases = 0;
    e = hipMemcpyAsync(&sample_bases, d_offsets + m, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    uint64_t half_bases = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&half_bases, d_offsets + std::max<uint32_t>(1, m / 2), 8,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess || sample_bases > n_bases) return e != hipSuccess ? PN_EDEVICE : PN_EINVAL;
    // device output for the sample's hits (sized after a first run)
    pn_hit *d_hits = nullptr;
    uint64_t cap = 0;
    const int qs[] = {10, 11, 12};
    const int ws[] = {32, 64};
    int nres = 0;
    double best = 1e300;
    *best_q = *best_w = 0;
    for (int q : qs) {
        for (int w : ws) {
            pn_tune_result &res = results[nres++];
            res.q = q;
            res.w = w;
            res.ms = -1.0;
            res.status = PN_OK;
            if ((uint32_t)q > qmax) {
                res.status = PN_ELEMMA;
                continue;
            }
            double t_at[2] = {1e300, 1e300};
            for (int half = 0; half < 2 && res.status == PN_OK; half++) {
                const uint32_t mm = half ? std::max<uint32_t>(1, m / 2) : m;
                const uint64_t bb = half ? half_bases : sample_bases;
                for (int rep = 0; rep < 3 && res.status == PN_OK; rep++) {
                    const double t0 = now_ms();
                    pn_index *x = nullptr;
                    int s = pn_index_build_dev(ctx, d_reads, d_offsets, mm, bb, q, w, st, &x);
                    uint64_t n_hits = 0;
                    if (!s) {
                        s = pn_map_dev(ctx, ref, x, k, d_k_per_read, mode, d_hits, cap, &n_hits, st);
                        if (s == PN_ETRUNC) {  // size the output once, then time again
                            if (d_hits) (void)hipFree(d_hits);
                            cap = n_hits + n_hits / 4 + 1;
                            d_hits = nullptr;
                            s = hipMalloc((void **)&d_hits, cap * sizeof(pn_hit)) == hipSuccess
                                    ? PN_OK
                                    : PN_ENOMEM;
                            if (!s)
                                s = pn_map_dev(ctx, ref, x, k, d_k_per_read, mode, d_hits, cap,
                                               &n_hits, st);
                            rep = -1;  // this run paid for sizing: not timed
                        }
                        pn_index_free(x);
                    }
                    if (s == PN_OK && hipStreamSynchronize(st) != hipSuccess) s = PN_EDEVICE;
                    if (s) {
                        res.status = s;
                        break;
                    }
                    if (rep >= 1) t_at[half] = std::min(t_at[half], now_ms() - t0);  // after a warm-up
                }
            }
            // the line through (m/2, t_half) and (m, t_m), at n_reads
            const double mh = std::max<uint32_t>(1, m / 2);
            const double slope = m > mh ? std::max(0.0, (t_at[0] - t_at[1]) / (m - mh)) : 0.0;
            const double t_best = t_at[0] + slope * ((double)n_reads - m);
            if (res.status == PN_OK) {
                res.ms = t_best;
                if (t_best < best) {
                    best = t_best;
                    *best_q = q;
                    *best_w = w;
                }
            }
        }
    }
    if (d_hits) (void)hipFree(d_hits);
    *n_results = nres;
    return *best_q ? PN_OK : PN_ELEMMA;
}

}  // extern "C"
