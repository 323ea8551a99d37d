// Host runtime of libpeanut: the C ABI of include/peanut.h, a per-context
// caching device allocator, and the ordering of the kernels of the mapping
// path on one stream.  No call aborts or prints; HIP failures become status
// codes.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "pn_runtime.h"
#include "pn_internal.h"

// ---------------------------------------------------------------------------
// context, allocator, workspace

namespace {

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
};

// an index orders its slices by the letters after the q-gram as well when
// at least 1/kOrderNextShare of its occurrences lie in slices longer than
// pn::kLongSlice
constexpr uint64_t kOrderNextShare = 128;

enum MiscSlot {  // 64-bit words of the context's device scratch block
    kStatus = 0,
    kStatMaxLen = 1,
    kStatT = 2,
    kStatBad = 3,
    kOutCount = 6,
    kVerifyRows = 8,
    kVerifyRowsLong = 9,
    kCountLetters = 10,
    kCandCounts = 16,                        // pn::kShards words each
    kRecCounts = kCandCounts + pn::kShards,
    kLongCounts = kRecCounts + pn::kShards,
    kFilterStats = kLongCounts + pn::kShards,  // 4 x pn::kShards words
    kHeavyCounts = kFilterStats + 4 * pn::kShards,
    kLaxCount = kHeavyCounts + pn::kShards,
    kLongEntries = kLaxCount + 1,
    kMiscWords = kLongEntries + 1
};

// the mapping path's grow-only buffers and output-region capacities
// (pn::kShards regions each; they grow on demand)
struct Workspace {
    Buf cands, longc, heavy, keys, keys_tmp, sort_temp, flags, pos, partials, minv, rinfo, side,
        side_meta, out_hits, out_best, lax, laxO;
    uint64_t cand_rcap = 1ull << 18;
    uint64_t rec_rcap = 1ull << 14;
    uint64_t heavy_rcap = 1ull << 12;  // per region: items of occurrence lists set aside
};

struct PendingStage {
    int stage;
    hipEvent_t a, b;
    int launches;
};

}  // namespace

int pnrt_noalloc_setup(int device);  // once per device (pn_ctx_create)

struct pn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::multimap<size_t, void *> cache;  // free device blocks by size
    std::map<void *, size_t> live;        // allocated device blocks
    uint64_t *misc = nullptr;             // device scratch words (MiscSlot)
    uint64_t *hmisc = nullptr;            // pinned host mirror
    // grow-only workspace of the mapping path
    Workspace ws;
    bool sub_on = false;  // lax lists made for the current mapping call
    bool wide_k = false;  // some read of the current mapping call has k > PN_BAND_K
    // stage timing and counters
    bool timing = false;
    pn_stats stats{};
    std::vector<hipEvent_t> ev_pool;
    std::vector<PendingStage> pending;
};

struct pn_ref {
    pn_ctx *ctx;
    uint64_t L;
    uint32_t *packed_base;  // one front word, then the text, then 4 words
    uint4 *planes0, *planes1;
    uint64_t n_blocks;
    // position sets sorted by q-gram, built on first use per q (any context
    // on the device may map against the reference: guarded by prep_mu)
    std::mutex prep_mu;
    unsigned long long *pkeys[PN_MAX_Q + 1] = {};
    uint16_t *pctx[PN_MAX_Q + 1] = {};
    uint64_t pn[PN_MAX_Q + 1] = {};
    // repeat masking per q: 4^q bits, set for the q-grams left out (null: off)
    uint32_t *pmask[PN_MAX_Q + 1] = {};
};

struct pn_index {
    pn_ctx *ctx;
    uint32_t n_reads;
    uint64_t n_bases, n_qgrams, n_distinct, n_groups, n_slots;
    int q, w, max_len;
    bool after_sorted = false;  // slices of O ordered by the letters after the q-gram first
    uint32_t *packed;
    uint64_t *offsets;
    uint2 *rplanes;
    void *I;
    uint32_t *S, *Sp;
    unsigned long long *O;
    uint32_t *lcinfo;
    uint32_t *tab_id = nullptr, *tabs = nullptr;  // slice tables (ordered index)
    uint32_t n_tabs = 0;
    bool s_half = false;  // S sampled at even groups
    uint32_t lc_size[pn::kLcPatterns];  // slice sizes of the low-complexity q-grams
    uint64_t lc_total;
};

namespace {

int map_err(hipError_t e) {
    if (e == hipSuccess) return PN_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return PN_ENOMEM;
    return PN_EDEVICE;
}

#define PN_TRY(expr)                          \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return map_err(e_); \
    } while (0)

#define PN_CHECK(st)                  \
    do {                              \
        int s_ = (st);                \
        if (s_ != PN_OK) return s_;   \
    } while (0)

size_t round_size(size_t n) {
    if (n < 256) return 256;
    if (n < (1u << 20)) return (n + 255) & ~(size_t)255;
    return (n + (2u << 20) - 1) & ~(size_t)((2u << 20) - 1);
}

int dalloc(pn_ctx *c, size_t bytes, void **out) {
    size_t n = round_size(bytes);
    auto it = c->cache.lower_bound(n);
    if (it != c->cache.end() && it->first <= 2 * n) {
        void *p = it->second;
        c->live[p] = it->first;
        c->cache.erase(it);
        *out = p;
        return PN_OK;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give cached blocks back to the driver and try once more
        PN_TRY(hipStreamSynchronize(c->stream));
        for (auto &kv : c->cache) (void)hipFree(kv.second);
        c->cache.clear();
        e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return PN_ENOMEM;
        }
    }
    c->live[p] = n;
    *out = p;
    return PN_OK;
}

void dfree(pn_ctx *c, void *p) {
    if (!p) return;
    auto it = c->live.find(p);
    if (it == c->live.end()) return;
    c->cache.emplace(it->second, p);
    c->live.erase(it);
}

template <typename T>
int dalloc_t(pn_ctx *c, size_t count, T **out) {
    void *p = nullptr;
    PN_CHECK(dalloc(c, count * sizeof(T) ? count * sizeof(T) : 1, &p));
    *out = (T *)p;
    return PN_OK;
}

// grow-only workspace buffer (contents are not preserved)
int ensure(pn_ctx *c, Buf &b, size_t bytes) {
    if (b.cap >= bytes && b.p) return PN_OK;
    dfree(c, b.p);
    b.p = nullptr;
    b.cap = 0;
    size_t want = std::max(bytes + bytes / 4, (size_t)4096);
    PN_CHECK(dalloc(c, want, &b.p));
    b.cap = want;
    return PN_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int bitlen(uint64_t x) {
    int b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

hipStream_t pick_stream(pn_ctx *c, void *s) { return s ? (hipStream_t)s : c->stream; }

// ---- stage timing: hipEvents on the stream the stage runs on ----

hipEvent_t take_event(pn_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

int stage_begin(pn_ctx *c, hipStream_t st, int stage) {
    if (!c->timing) return -1;
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return -1;
    (void)hipEventRecord(a, st);
    c->pending.push_back({stage, a, b, 0});
    return (int)c->pending.size() - 1;
}

void stage_end(pn_ctx *c, hipStream_t st, int tok, int launches) {
    if (tok < 0) return;
    (void)hipEventRecord(c->pending[tok].b, st);
    c->pending[tok].launches = launches;
}

// after a synchronisation: fold finished stage events into the statistics
void collect_stages(pn_ctx *c) {
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->stats.ms[p.stage] += ms;
            c->stats.launches[p.stage] += (uint64_t)p.launches;
        } else {
            (void)hipGetLastError();
        }
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    c->pending.clear();
}

// read the misc words back to the host (synchronises the stream)
int read_misc(pn_ctx *c, hipStream_t st) {
    PN_TRY(hipMemcpyAsync(c->hmisc, c->misc, kMiscWords * sizeof(uint64_t), hipMemcpyDeviceToHost,
                          st));
    PN_TRY(hipStreamSynchronize(st));
    collect_stages(c);
    return PN_OK;
}

void zero_misc(pn_ctx *c, hipStream_t st) {
    pn::launch_fill_u32((uint32_t *)c->misc, 2 * kMiscWords, 0u, st);
}

PnRefDev ref_desc(const pn_ref *r) {
    PnRefDev d;
    d.packed = r->packed_base + 1;
    d.planes[0] = r->planes0;
    d.planes[1] = r->planes1;
    d.L = r->L;
    d.n_plane_blocks = r->n_blocks;
    return d;
}

// the q-gram-sorted position set of `r` for q (Section 3.2), built on first
// use: keys of both strands, a stable radix sort by q-gram, then each
// entry's context.  Owned by the reference (plain device allocations).
int ref_prepare(pn_ref *r, int q, hipStream_t st, pn::RefQDev *out) {
    std::lock_guard<std::mutex> lk(r->prep_mu);
    const uint64_t n = r->L >= (uint64_t)q ? 2 * (r->L - q + 1) : 0;
    // a key holds (position << 1 | strand) beside the q-gram's 2q bits
    if (bitlen(2 * r->L) + 2 * q > 64) return PN_EINVAL;
    if (r->pkeys[q] || n == 0) {
        *out = pn::RefQDev{r->pkeys[q], r->pctx[q], r->pkeys[q] ? r->pn[q] : 0, r->pmask[q]};
        return PN_OK;
    }
    unsigned long long *keys = nullptr, *tmp = nullptr;
    uint16_t *ctx = nullptr;
    void *temp = nullptr;
    const bool packed = pn::refq_packs(r->L, q);
    hipError_t e = hipMalloc((void **)&keys, n * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&tmp, n * 8);
    if (e == hipSuccess && !packed) e = hipMalloc((void **)&ctx, n * 2);
    if (e == hipSuccess) e = hipMalloc(&temp, pn::radix_temp_size(n));
    if (e == hipSuccess) {
        const PnRefDev rd = ref_desc(r);
        pn::launch_refq_keys(rd, q, keys, st);
        unsigned long long *sorted = pn::radix_sort_u64_any(
            keys, tmp, n, 2 * q + 2 * pn::refq_sort_letters(r->L, q), temp, st);
        if (sorted != keys) std::swap(keys, tmp);
        pn::launch_refq_ctx(rd, q, keys, n, ctx, st);
        e = hipStreamSynchronize(st);
    }
    if (tmp) (void)hipFree(tmp);
    if (temp) (void)hipFree(temp);
    if (e != hipSuccess) {
        if (keys) (void)hipFree(keys);
        if (ctx) (void)hipFree(ctx);
        return map_err(e);
    }
    r->pkeys[q] = keys;
    r->pctx[q] = ctx;
    r->pn[q] = n;
    *out = pn::RefQDev{keys, ctx, n, nullptr};
    return PN_OK;
}

PnIndexDev index_desc(const pn_index *x) {
    PnIndexDev d;
    d.packed = x->packed;
    d.offsets = x->offsets;
    d.rplanes = x->rplanes;
    d.rplanes_rc = x->rplanes + (uint64_t)x->n_reads * PN_READ_WORDS;
    d.I = x->I;
    d.S = x->S;
    d.Sp = x->Sp;
    d.O = x->O;
    d.lcinfo = x->lcinfo;
    d.tab_id = x->tab_id;
    d.tabs = x->tabs;
    d.n_reads = x->n_reads;
    d.max_len = (uint32_t)x->max_len;
    d.q = x->q;
    d.log2w = x->w == 64 ? 6 : 5;
    d.n_groups = x->n_groups;
    d.after_sorted = x->after_sorted ? 1 : 0;
    d.s_half = x->s_half ? 1 : 0;
    return d;
}

void free_index_arrays(pn_index *x) {
    pn_ctx *c = x->ctx;
    dfree(c, x->packed);
    dfree(c, x->offsets);
    dfree(c, x->rplanes);
    dfree(c, x->I);
    dfree(c, x->S);
    dfree(c, x->Sp);
    dfree(c, x->O);
    dfree(c, x->lcinfo);
    dfree(c, x->tab_id);
    dfree(c, x->tabs);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *pn_strerror(int status) {
    switch (status) {
        case PN_OK: return "ok";
        case PN_EINVAL: return "invalid argument or limit exceeded";
        case PN_EALPHABET: return "letter other than A/C/G/T";
        case PN_ENOMEM: return "out of memory";
        case PN_EDEVICE: return "HIP device error";
        case PN_ELEMMA: return "q-gram lemma violated: (k+1)*q > read length";
        case PN_ETRUNC: return "output capacity too small";
        case PN_EBUDGET: return "request exceeds the memory budget";
        default: return "unknown status";
    }
}

int pn_ctx_create(int device, pn_ctx **out) {
    if (!out) return PN_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return PN_EDEVICE;
    }
    DeviceGuard g(device);
    pn_ctx *c = new (std::nothrow) pn_ctx();
    if (!c) return PN_ENOMEM;
    c->device = device;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void **)&c->misc, kMiscWords * sizeof(uint64_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->hmisc, kMiscWords * sizeof(uint64_t), 0);
    // the device array of pn_validate_noalloc: its address on this device
    const int s = e == hipSuccess ? pnrt_noalloc_setup(device) : map_err(e);
    if (s) {
        if (c->hmisc) (void)hipHostFree(c->hmisc);
        if (c->misc) (void)hipFree(c->misc);
        if (c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return s;
    }
    *out = c;
    return PN_OK;
}

void pn_ctx_destroy(pn_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->cache) (void)hipFree(kv.second);
    for (auto &kv : c->live) (void)hipFree(kv.first);
    collect_stages(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(c->misc);
    (void)hipHostFree(c->hmisc);
    (void)hipStreamDestroy(c->stream);
    delete c;
}

int pn_ctx_stream(pn_ctx *c, void **stream) {
    if (!c || !stream) return PN_EINVAL;
    *stream = (void *)c->stream;
    return PN_OK;
}

int pn_ctx_set_timing(pn_ctx *c, int enable) {
    if (!c) return PN_EINVAL;
    c->timing = enable != 0;
    return PN_OK;
}

int pn_ctx_get_stats(pn_ctx *c, pn_stats *out, int reset) {
    if (!c || !out) return PN_EINVAL;
    *out = c->stats;
    if (reset) c->stats = pn_stats{};
    return PN_OK;
}

// ---- reference --------------------------------------------------------------

int pn_ref_load_dev(pn_ctx *c, const char *d_seq, uint64_t len, void *stream, pn_ref **out) {
    if (!c || !out || !d_seq || len == 0 || len >= (1ull << 32) - (1ull << 16)) return PN_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t st = pick_stream(c, stream);
    pn_ref *r = new (std::nothrow) pn_ref();
    if (!r) return PN_ENOMEM;
    r->ctx = c;
    r->L = len;
    const uint64_t words = (len + 15) / 16;
    r->n_blocks = (len + 31) / 32 + 2 * PN_PAD_BLOCKS + 16;
    int s = dalloc_t(c, words + 5, &r->packed_base);
    if (!s) s = dalloc_t(c, r->n_blocks, &r->planes0);
    if (!s) s = dalloc_t(c, r->n_blocks, &r->planes1);
    if (s) {
        dfree(c, r->packed_base);
        dfree(c, r->planes0);
        dfree(c, r->planes1);
        delete r;
        return s;
    }
    zero_misc(c, st);
    pn::launch_fill_u32(r->packed_base, 1, 0u, st);
    pn::launch_fill_u32(r->packed_base + 1 + words, 4, 0u, st);
    pn::launch_pack2(d_seq, len, r->packed_base + 1, (uint32_t *)&c->misc[kStatus], st);
    pn::launch_ref_planes(r->packed_base + 1, len, r->planes0, r->planes1, r->n_blocks, st);
    s = read_misc(c, st);
    if (!s && (c->hmisc[kStatus] & 1)) s = PN_EALPHABET;
    if (s) {
        pn_ref_free(r);
        return s;
    }
    *out = r;
    return PN_OK;
}

int pn_ref_load(pn_ctx *c, const char *seq, uint64_t len, pn_ref **out) {
    if (!c || !out || !seq || len == 0 || len >= (1ull << 32) - (1ull << 16)) return PN_EINVAL;
    DeviceGuard g(c->device);
    char *d = nullptr;
    PN_CHECK(dalloc_t(c, len, &d));
    hipError_t e = hipMemcpyAsync(d, seq, len, hipMemcpyHostToDevice, c->stream);
    int s = e == hipSuccess ? pn_ref_load_dev(c, d, len, c->stream, out) : map_err(e);
    (void)hipStreamSynchronize(c->stream);
    dfree(c, d);
    return s;
}

void pn_ref_free(pn_ref *r) {
    if (!r) return;
    pn_ctx *c = r->ctx;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    dfree(c, r->packed_base);
    dfree(c, r->planes0);
    dfree(c, r->planes1);
    for (int q = 0; q <= PN_MAX_Q; q++) {
        if (r->pkeys[q]) (void)hipFree(r->pkeys[q]);
        if (r->pctx[q]) (void)hipFree(r->pctx[q]);
        if (r->pmask[q]) (void)hipFree(r->pmask[q]);
    }
    delete r;
}

int pn_ref_mask(pn_ref *r, int q, uint32_t max_occ) {
    if (!r || q < 1 || q > PN_MAX_Q) return PN_EINVAL;
    DeviceGuard g(r->ctx->device);
    hipStream_t st = r->ctx->stream;
    pn::RefQDev P;
    PN_CHECK(ref_prepare(r, q, st, &P));
    std::lock_guard<std::mutex> lk(r->prep_mu);
    if (r->pmask[q]) {
        PN_TRY(hipStreamSynchronize(st));
        (void)hipFree(r->pmask[q]);
        r->pmask[q] = nullptr;
    }
    if (!max_occ || !P.n) return PN_OK;
    const uint64_t words = ((1ull << (2 * q)) + 31) / 32;
    uint32_t *bits = nullptr;
    PN_TRY(hipMalloc((void **)&bits, words * 4));
    pn::launch_fill_u32(bits, words, 0u, st);
    pn::launch_mask_runs(P, q, max_occ, bits, st);
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(bits);
        return map_err(e);
    }
    r->pmask[q] = bits;
    return PN_OK;
}

int pn_ref_prepare(pn_ref *r, int q) {
    if (!r || q < 1 || q > PN_MAX_Q) return PN_EINVAL;
    DeviceGuard g(r->ctx->device);
    pn::RefQDev P;
    return ref_prepare(r, q, r->ctx->stream, &P);
}

uint64_t pn_ref_length(const pn_ref *r) { return r ? r->L : 0; }

// ---- index (Algorithm 1) ------------------------------------------------------

int pn_index_build_dev(pn_ctx *c, const char *d_reads, const uint64_t *d_offsets,
                       uint32_t n_reads, uint64_t n_bases, int q, int w, void *stream,
                       pn_index **out) {
    if (!c || !out || (n_reads && !d_offsets) || (n_bases && !d_reads)) return PN_EINVAL;
    if (q < 1 || q > PN_MAX_Q || (w != 32 && w != 64) || n_reads > PN_MAX_READS ||
        n_bases >= (1ull << 32))
        return PN_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t st = pick_stream(c, stream);
    pn_index *x = new (std::nothrow) pn_index();
    if (!x) return PN_ENOMEM;
    x->ctx = c;
    x->n_reads = n_reads;
    x->n_bases = n_bases;
    x->q = q;
    x->w = w;
    const uint64_t G = 1ull << (2 * q);
    x->n_groups = (G + w - 1) / w;
    const uint64_t words = (n_bases + 15) / 16;
    int s = dalloc_t(c, words + 4, &x->packed);
    if (!s) s = dalloc_t(c, (uint64_t)n_reads + 1, &x->offsets);
    if (s) {
        free_index_arrays(x);
        delete x;
        return s;
    }
    zero_misc(c, st);
    int tok = stage_begin(c, st, PN_STAGE_INGEST);
    pn::launch_fill_u32(x->packed + words, 4, 0u, st);
    pn::launch_pack2(d_reads, n_bases, x->packed, (uint32_t *)&c->misc[kStatus], st);
    hipError_t e = n_reads ? hipMemcpyAsync(x->offsets, d_offsets, ((uint64_t)n_reads + 1) * 8,
                                            hipMemcpyDeviceToDevice, st)
                           : hipSuccess;
    if (!n_reads) pn::launch_fill_u32((uint32_t *)x->offsets, 2, 0u, st);
    pn::launch_read_meta(x->offsets, n_reads, q, n_bases, &c->misc[kStatMaxLen], st);
    stage_end(c, st, tok, 3);
    if (e == hipSuccess) s = read_misc(c, st);
    else s = map_err(e);
    if (!s && (c->hmisc[kStatus] & 1)) s = PN_EALPHABET;
    if (!s && c->hmisc[kStatBad]) s = PN_EINVAL;
    if (s) {
        free_index_arrays(x);
        delete x;
        return s;
    }
    x->max_len = (int)c->hmisc[kStatMaxLen];
    x->n_qgrams = c->hmisc[kStatT];
    x->n_slots = std::min<uint64_t>(G, x->n_qgrams);
    const uint64_t T = x->n_qgrams, U = x->n_slots;
    uint32_t *nq = nullptr, *partials = nullptr, *lcs = nullptr, *first_read = nullptr,
             *hist0 = nullptr;
    const uint64_t tile = pn::radix_tile_keys(T);
    const uint64_t tiles = (T + tile - 1) / tile;
    uint8_t *flags = nullptr;
    unsigned long long *keys = nullptr, *tmp = nullptr;
    void *sort_temp = nullptr;
    s = dalloc_t(c, 2 * (uint64_t)n_reads * PN_READ_WORDS + 1, &x->rplanes);
    if (!s) s = dalloc(c, x->n_groups * (w / 8), &x->I);
    if (!s) s = dalloc_t(c, x->n_groups + 1, &x->S);
    if (!s) s = dalloc_t(c, U + 1, &x->Sp);
    if (!s) s = dalloc_t(c, T + 1, &x->O);
    if (!s) s = dalloc_t(c, (uint64_t)n_reads + 1, &x->lcinfo);
    if (!s) s = dalloc_t(c, pn::kLcPatterns, &lcs);
    if (!s) s = dalloc_t(c, (uint64_t)n_reads + 1, &nq);
    if (!s) s = dalloc_t(c, T + 1, &keys);
    if (!s) s = dalloc_t(c, T + 1, &tmp);
    if (!s) s = dalloc_t(c, T + 1, &flags);
    if (!s) s = dalloc_t(c, tiles + 1, &first_read);
    if (!s) s = dalloc_t(c, 256 * tiles + 1, &hist0);
    if (!s) s = dalloc(c, pn::radix_temp_size(T), &sort_temp);
    if (!s)
        s = dalloc_t(c,
                     pn::scan_partials_size(
                         std::max<uint64_t>(std::max<uint64_t>(x->n_groups, T + 1), n_reads + 1)),
                     &partials);
    if (!s) {
        PnIndexDev ix = index_desc(x);
        tok = stage_begin(c, st, PN_STAGE_INGEST);
        pn::launch_read_planes(x->packed, x->offsets, n_reads, x->rplanes, st);
        pn::launch_read_lc(ix, x->lcinfo, st);
        stage_end(c, st, tok, 2);
        tok = stage_begin(c, st, PN_STAGE_INDEX);
        // q-gram occurrences -> keys at their read's offset in O
        pn::launch_read_nq(ix, nq, st);
        pn::launch_scan_u32(nq, nq, n_reads, partials, st);
        pn::launch_qgram_keys(ix, nq, T, tile, first_read, keys, hist0, st);
        const int glo = pn::index_gram_lo(q);
        unsigned long long *sorted =
            pn::radix_sort_u64_any(keys, tmp, T, glo + 2 * q, sort_temp, st, glo, hist0);
        pn::launch_fill_u32((uint32_t *)x->I, x->n_groups * (w / 32), 0u, st);
        pn::launch_index_from_sorted(ix, sorted, T, x->O, flags, x->I, st);  // step 1, O
        pn::launch_scan_popc(x->I, ix.log2w, x->S, x->n_groups, partials, st);  // steps 2-3
        pn::launch_starts_to_sp(flags, T, partials, x->Sp, st);  // steps 4-6
        // occurrences in long slices decide whether the slices are ordered
        // by the letters after the q-gram as well
        pn::launch_fill_u32((uint32_t *)&c->misc[kLongEntries], 2, 0u, st);
        pn::launch_long_entries(x->S + x->n_groups, x->Sp, pn::kLongSlice,
                                (unsigned long long *)&c->misc[kLongEntries], st);
        stage_end(c, st, tok, 7 + 3 * ((2 * q + 7) / 8) + 3 + 3);
        pn::launch_lc_sizes(ix, lcs, st);
        uint32_t n_distinct = 0;
        e = hipMemcpyAsync(&n_distinct, x->S + x->n_groups, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(x->lc_size, lcs, sizeof(x->lc_size), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&c->hmisc[kLongEntries], &c->misc[kLongEntries], 8,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = map_err(e);
        if (!s) {
            x->n_distinct = n_distinct;
            x->lc_total = 0;
            for (int i = 0; i < pn::kLcPatterns; i++) x->lc_total += x->lc_size[i];
            collect_stages(c);
            // Repeat families in the reads give long slices whose entries
            // differ in the letters that follow; ordering those letters too
            // (and, inside one set of letters, the piece starts last) lets
            // filtration visit only the entries that can pair with a text
            // position (one more sort, worth it when a notable share of all
            // occurrences lies in long slices)
            if (glo && c->hmisc[kLongEntries] * kOrderNextShare >= T) {
                tok = stage_begin(c, st, PN_STAGE_INDEX);
                unsigned long long *other = sorted == keys ? tmp : keys;
                sorted = pn::radix_sort_index_slices(sorted, other, T, q, sort_temp, st);
                pn::launch_index_from_sorted(ix, sorted, T, x->O, flags, x->I, st);
                stage_end(c, st, tok, 5 * (1 + (2 * q + 9) / 8) + 1);
                x->after_sorted = true;
                // a table per long slice: where each set of letters after the
                // q-gram starts (filtration's searches become two loads)
                const uint64_t D = x->n_distinct;
                uint32_t *tflags = nullptr, *tnum = nullptr;
                s = dalloc_t(c, D + 1, &tnum);
                if (!s) s = dalloc_t(c, D + 1, &tflags);
                if (!s) {
                    pn::launch_tab_flags(x->Sp, D, pn::kTabMin, tflags, st);
                    pn::launch_scan_u32(tflags, tnum, D, partials, st);
                    uint32_t nt = 0;
                    e = hipMemcpyAsync(&nt, tnum + D, 4, hipMemcpyDeviceToHost, st);
                    if (e == hipSuccess) e = hipStreamSynchronize(st);
                    s = map_err(e);
                    if (!s) {
                        x->n_tabs = nt;
                        s = dalloc_t(c, D + 1, &x->tab_id);
                        if (!s) s = dalloc_t(c, (uint64_t)nt * pn::kTabWidth + 1, &x->tabs);
                        if (!s) {
                            // (the flags' buffer then takes the list of table slots)
                            pn::launch_tab_build(x->O, x->Sp, D, pn::kTabMin, tnum, nt, x->tab_id,
                                                 tflags, x->tabs, st);
                            e = hipStreamSynchronize(st);
                            s = map_err(e);
                        }
                    }
                }
                dfree(c, tnum);
                dfree(c, tflags);
                if (!s) collect_stages(c);
            }
        }
    }
    dfree(c, nq);
    dfree(c, keys);
    dfree(c, tmp);
    dfree(c, flags);
    dfree(c, first_read);
    dfree(c, hist0);
    dfree(c, sort_temp);
    dfree(c, partials);
    dfree(c, lcs);
    if (s) {
        free_index_arrays(x);
        delete x;
        return s;
    }
    *out = x;
    return PN_OK;
}

int pn_index_build(pn_ctx *c, const char *reads, const uint64_t *offsets, uint32_t n_reads, int q,
                   int w, pn_index **out) {
    if (!c || !out || (n_reads && (!offsets || !reads))) return PN_EINVAL;
    uint64_t n_bases = n_reads ? offsets[n_reads] : 0;
    for (uint32_t r = 0; r < n_reads; r++)
        if (offsets[r + 1] < offsets[r]) return PN_EINVAL;
    DeviceGuard g(c->device);
    char *dr = nullptr;
    uint64_t *doff = nullptr;
    int s = dalloc_t(c, n_bases + 1, &dr);
    if (!s) s = dalloc_t(c, (uint64_t)n_reads + 1, &doff);
    if (!s && n_bases)
        s = map_err(hipMemcpyAsync(dr, reads, n_bases, hipMemcpyHostToDevice, c->stream));
    if (!s && n_reads)
        s = map_err(hipMemcpyAsync(doff, offsets, ((uint64_t)n_reads + 1) * 8,
                                   hipMemcpyHostToDevice, c->stream));
    if (!s) s = pn_index_build_dev(c, dr, doff, n_reads, n_bases, q, w, c->stream, out);
    (void)hipStreamSynchronize(c->stream);
    dfree(c, dr);
    dfree(c, doff);
    return s;
}

void pn_index_free(pn_index *x) {
    if (!x) return;
    DeviceGuard g(x->ctx->device);
    (void)hipStreamSynchronize(x->ctx->stream);
    free_index_arrays(x);
    delete x;
}

int pn_index_get_info(const pn_index *x, pn_index_info *out) {
    if (!x || !out) return PN_EINVAL;
    pn_index_info i{};
    i.n_reads = x->n_reads;
    i.n_bases = x->n_bases;
    i.n_qgrams = x->n_qgrams;
    i.n_distinct = x->n_distinct;
    i.n_groups = x->n_groups;
    i.q = x->q;
    i.w = x->w;
    i.max_len = x->max_len;
    i.after_sorted = x->after_sorted ? 1 : 0;
    i.s_sample = x->s_half ? 2 : 1;
    *out = i;
    return PN_OK;
}

int pn_index_sample_s(pn_index *x) {
    if (!x) return PN_EINVAL;
    if (x->s_half) return PN_OK;
    pn_ctx *c = x->ctx;
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    uint32_t *half = nullptr;
    PN_CHECK(dalloc_t(c, x->n_groups / 2 + 1, &half));
    pn::launch_sample_s(x->S, x->n_groups, half, st);
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        dfree(c, half);
        return map_err(e);
    }
    dfree(c, x->S);
    x->S = half;
    x->s_half = true;
    return PN_OK;
}

int pn_index_export(const pn_index *x, void *I, uint32_t *S, uint32_t *Sp, uint64_t *O) {
    if (!x) return PN_EINVAL;
    pn_ctx *c = x->ctx;
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    if (I) PN_TRY(hipMemcpyAsync(I, x->I, x->n_groups * (x->w / 8), hipMemcpyDeviceToHost, st));
    const uint64_t ns = x->s_half ? x->n_groups / 2 + 1 : x->n_groups + 1;
    if (S) PN_TRY(hipMemcpyAsync(S, x->S, ns * 4, hipMemcpyDeviceToHost, st));
    if (Sp) PN_TRY(hipMemcpyAsync(Sp, x->Sp, (x->n_distinct + 1) * 4, hipMemcpyDeviceToHost, st));
    if (O && x->n_qgrams)
        PN_TRY(hipMemcpyAsync(O, x->O, x->n_qgrams * 8, hipMemcpyDeviceToHost, st));
    PN_TRY(hipStreamSynchronize(st));
    return PN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// mapping path

namespace {

int key_ebits(uint64_t L) { return std::max(1, bitlen(L - 1)); }
int key_rbits(uint32_t n) { return std::max(1, bitlen(n ? n - 1 : 0)); }

// per-read seed rules (with the k / lemma check) and the low-complexity side
// lists; synchronises once to report a bad k or a lemma violation
// plain: the position set is masked (every read gets the plain rule byte)
int prepare_rules(pn_ctx *c, const pn_index *x, int kglob, const uint8_t *d_k, bool plain,
                  hipStream_t st) {
    // the rule bytes, then (256-byte aligned) the stamp words
    const uint64_t rinfo_bytes = ((uint64_t)x->n_reads + 1 + 255) & ~255ull;
    PN_CHECK(ensure(c, c->ws.rinfo, rinfo_bytes + 2 * ((uint64_t)x->n_reads + 1)));
    uint16_t *rstamp = (uint16_t *)((uint8_t *)c->ws.rinfo.p + rinfo_bytes);
    PN_CHECK(ensure(c, c->ws.side, std::max<uint64_t>(x->lc_total, 1) * 8));
    PN_CHECK(ensure(c, c->ws.side_meta, 17 * pn::kLcPatterns * 4));
    uint32_t starts[pn::kLcPatterns];
    uint64_t at = 0;
    for (int i = 0; i < pn::kLcPatterns; i++) {
        starts[i] = (uint32_t)at;
        at += x->lc_size[i];
    }
    zero_misc(c, st);
    PN_TRY(hipMemcpyAsync(c->ws.side_meta.p, starts, sizeof(starts), hipMemcpyHostToDevice, st));
    PnIndexDev ix = index_desc(x);
    const int tok = stage_begin(c, st, PN_STAGE_RULES);
    pn::launch_read_rules(ix, kglob, d_k, (uint8_t *)c->ws.rinfo.p, rstamp,
                          (uint32_t *)&c->misc[kStatus], plain, st);
    pn::launch_stamp_rules(x->O, x->n_qgrams, rstamp, st);
    // 16 region starts, 16 x 6 class bounds, then scratch for the side lists
    uint32_t *meta = (uint32_t *)c->ws.side_meta.p;
    pn::launch_fill_u32(meta + pn::kLcPatterns, 6 * pn::kLcPatterns, 0u, st);
    if (x->n_reads)
        pn::launch_lc_side(ix, (const uint8_t *)c->ws.rinfo.p, (unsigned long long *)c->ws.side.p, meta,
                           meta + pn::kLcPatterns, meta + 7 * pn::kLcPatterns, st);
    // lax lists: an index whose slices are ordered by the letters after the
    // q-gram is searched in its long slices (see pn::Lists)
    c->sub_on = x->after_sorted && x->n_reads && x->n_distinct;
    if (c->sub_on) {
        PN_CHECK(ensure(c, c->ws.lax, (x->n_distinct + 1) * sizeof(uint2)));
        PN_CHECK(ensure(c, c->ws.laxO, std::max<uint64_t>(x->n_qgrams, 1) * 8));
        pn::launch_fill_u32((uint32_t *)&c->misc[kLaxCount], 2, 0u, st);
        pn::launch_lax_lists(ix, x->n_distinct, pn::kSearchMin, (uint2 *)c->ws.lax.p,
                             (unsigned long long *)c->ws.laxO.p,
                             (unsigned long long *)&c->misc[kLaxCount], st);
    }
    stage_end(c, st, tok, (x->n_reads ? 7 : 3) + (c->sub_on ? 2 : 0));
    PN_CHECK(read_misc(c, st));
    const uint32_t status = (uint32_t)c->hmisc[kStatus];
    c->wide_k = (status & 16u) != 0;
    if (status & 2u) return PN_EINVAL;
    if (status & 4u) return PN_ELEMMA;
    return PN_OK;
}

pn::Lists lists_of(const pn_ctx *c) {
    const uint32_t *meta = (const uint32_t *)c->ws.side_meta.p;
    return pn::Lists{(const unsigned long long *)c->ws.side.p, meta + pn::kLcPatterns,
                     (const unsigned long long *)c->ws.laxO.p, (const uint2 *)c->ws.lax.p, pn::kSearchMin,
                     c->sub_on ? 1 : 0};
}

// filtration of the entries [a, b) of the reference's position set P
int launch_filter_into(pn_ctx *c, const pn_ref *ref, const pn_index *x, const pn::RefQDev &Pall,
                       uint64_t a, uint64_t b, hipStream_t st) {
    pn::RefQDev P{Pall.keys + a, Pall.ctx ? Pall.ctx + a : nullptr, b - a, Pall.mask};
    PN_CHECK(ensure(c, c->ws.heavy, pn::kShards * c->ws.heavy_rcap * 2 * sizeof(uint4)));
    pn::launch_fill_u32((uint32_t *)&c->misc[kHeavyCounts], 2 * pn::kShards, 0u, st);
    pn::FilterOut fo{(uint2 *)c->ws.cands.p,
                     {(unsigned long long *)&c->misc[kCandCounts], c->ws.cand_rcap},
                     (uint4 *)c->ws.heavy.p,
                     {(unsigned long long *)&c->misc[kHeavyCounts], c->ws.heavy_rcap},
                     pn::filter_heavy_min(x->n_qgrams, x->q),
                     (unsigned long long *)&c->misc[kFilterStats]};
    int tok = stage_begin(c, st, PN_STAGE_FILTER_EMIT);
    const pn::Lists ls = lists_of(c);
    pn::launch_filter(ref_desc(ref), P, index_desc(x), ls, fo, st);
    stage_end(c, st, tok, 1);
    tok = stage_begin(c, st, PN_STAGE_FILTER_HEAVY);
    pn::launch_filter_heavy(index_desc(x), ls, fo, st);
    stage_end(c, st, tok, 1);
    return PN_OK;
}

// largest and total count of a sharded list (host mirror)
void region_counts(const pn_ctx *c, int slot, uint32_t regions, uint64_t *mx, uint64_t *total) {
    *mx = *total = 0;
    for (uint32_t g = 0; g < regions; g++) {
        *mx = std::max<uint64_t>(*mx, c->hmisc[slot + g]);
        *total += c->hmisc[slot + g];
    }
}

// after a filtration: the largest heavy-item region count (items asked for)
uint64_t heavy_max(const pn_ctx *c) {
    uint64_t mx, tot;
    region_counts(c, kHeavyCounts, pn::kShards, &mx, &tot);
    return mx;
}

// occurrence pairs seen and index entries read by the last filtration
struct FilterWork {
    uint64_t seeds = 0, visited = 0, set_aside = 0, written = 0, items = 0;
};

FilterWork filter_stats(const pn_ctx *c) {
    FilterWork f;
    for (uint32_t g = 0; g < pn::kShards; g++) {
        f.seeds += c->hmisc[kFilterStats + 4 * g];
        f.visited += c->hmisc[kFilterStats + 4 * g + 1];
        f.set_aside += c->hmisc[kFilterStats + 4 * g + 2];
        f.written += c->hmisc[kFilterStats + 4 * g + 3];
        f.items += c->hmisc[kHeavyCounts + g];
    }
    return f;
}

void zero_counts(pn_ctx *c, int slot, hipStream_t st) {
    pn::launch_fill_u32((uint32_t *)&c->misc[slot], 2 * pn::kShards, 0u, st);
}

// Candidate and hand-off buffers of one filtration stay below these sizes
// (per region: kShards regions each); a part of the position set whose
// output would not fit is split in two and each half is run on its own.
constexpr uint64_t kMaxCandRegion = (1ull << 28) / pn::kShards;   // 2 GiB of candidates
constexpr uint64_t kMaxHeavyRegion = (1ull << 26) / pn::kShards;  // 2 GiB of items

// grow-only buffer whose first `keep` bytes survive the growth
int ensure_keep(pn_ctx *c, Buf &b, size_t bytes, size_t keep, hipStream_t st) {
    if (b.cap >= bytes && b.p) return PN_OK;
    size_t want = std::max(bytes + bytes / 4, (size_t)4096);
    void *p = nullptr;
    PN_CHECK(dalloc(c, want, &p));
    if (keep && b.p) {
        hipError_t e = hipMemcpyAsync(p, b.p, keep, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) {
            dfree(c, p);
            return map_err(e);
        }
    }
    dfree(c, b.p);
    b.p = p;
    b.cap = want;
    return PN_OK;
}

// Validation (both passes) of candidates, records into the sharded
// c->ws.keys_tmp.  With `filter`, the candidates come from filtration of the
// reference's position set, part by part: each part is filtered (and its
// candidate counts checked: a buffer that overflowed is grown, or the part
// split when its output would pass the bounds above, and the part filtered
// again), verified (records that overflowed: grown, verified again) and its
// records gathered into c->ws.keys before the next part, so that candidate
// buffers stay bounded however many candidates the whole reference yields.
// Without `filter`, the n_in candidates already in c->ws.cands are verified.
// Leaves all records, sorted, in c->ws.keys and their count in *n_rec.
constexpr uint64_t kFirstPart = 1ull << 30;  // position-set entries filtered at once at first

int validate_sorted(pn_ctx *c, const pn_ref *ref, const pn_index *x, int kglob, const uint8_t *d_k,
                    bool filter, uint64_t n_in, hipStream_t st, uint64_t *n_rec) {
    const int ebits = key_ebits(ref->L);
    c->ws.rec_rcap = std::max<uint64_t>(c->ws.rec_rcap, (16ull * x->n_reads) / pn::kShards + 4096);
    pn::RefQDev P{nullptr, nullptr, 0, nullptr};
    if (filter) PN_CHECK(ref_prepare(const_cast<pn_ref *>(ref), x->q, st, &P));
    const uint32_t regions = filter ? pn::kShards : 1;
    const uint64_t end = filter ? P.n : (n_in ? 1 : 0);
    uint64_t a = 0, part = std::min<uint64_t>(std::max<uint64_t>(end, 1), kFirstPart), total = 0;
    int attempts = 0;
    while (a < end) {
        if (++attempts > 64) return PN_ENOMEM;
        const uint64_t b = filter ? std::min(end, a + part) : end;
        uint64_t cand_total = filter ? 0 : n_in;
        const uint64_t in_rcap = filter ? c->ws.cand_rcap : std::max<uint64_t>(n_in, 1);
        PN_CHECK(ensure(c, c->ws.cands, regions * in_rcap * sizeof(uint2)));
        PN_CHECK(ensure(c, c->ws.longc, regions * in_rcap * sizeof(uint2)));
        // the count filter before the band pass when the reads come from
        // repeat families (below)
        const bool count_first = filter && x->after_sorted;
        zero_counts(c, kCandCounts, st);
        FilterWork fw;
        if (filter) {
            pn::launch_fill_u32((uint32_t *)&c->misc[kFilterStats], 8 * pn::kShards, 0u, st);
            PN_CHECK(launch_filter_into(c, ref, x, P, a, b, st));
            PN_CHECK(read_misc(c, st));
            uint64_t cand_max;
            region_counts(c, kCandCounts, regions, &cand_max, &cand_total);
            const uint64_t hmax = heavy_max(c);
            bool again = false;
            if ((cand_max > kMaxCandRegion || hmax > kMaxHeavyRegion) && b - a > 1) {
                part = std::max<uint64_t>(1, (b - a) / 2);
                again = true;
            } else {
                if (cand_max > c->ws.cand_rcap) {
                    c->ws.cand_rcap = cand_max + cand_max / 4;
                    again = true;
                }
                if (hmax > c->ws.heavy_rcap) {
                    c->ws.heavy_rcap = hmax + hmax / 4;
                    again = true;
                }
            }
            if (again) continue;
            fw = filter_stats(c);
            // parts that came out small may grow again
            if (cand_max < kMaxCandRegion / 4 && hmax < kMaxHeavyRegion / 4 && part < kFirstPart)
                part *= 2;
        } else {
            pn::launch_fill_u32((uint32_t *)&c->misc[kCandCounts], 1, (uint32_t)n_in, st);
        }
        uint64_t got = 0;
        for (int vattempt = 0;; vattempt++) {
            if (vattempt >= 8) return PN_ENOMEM;
            PN_CHECK(ensure(c, c->ws.keys_tmp, pn::kShards * c->ws.rec_rcap * 8));
            pn::launch_fill_u32((uint32_t *)&c->misc[kVerifyRows], 6, 0u, st);
            zero_counts(c, kRecCounts, st);
            zero_counts(c, kLongCounts, st);
            pn::VerifyIn in{(const uint2 *)c->ws.cands.p,
                            (const unsigned long long *)&c->misc[kCandCounts], regions, in_rcap};
            pn::VerifyOut vo{(unsigned long long *)c->ws.keys_tmp.p,
                             {(unsigned long long *)&c->misc[kRecCounts], c->ws.rec_rcap},
                             (unsigned long long *)&c->misc[kVerifyRows], ebits};
            uint2 *last_in = (uint2 *)c->ws.longc.p;
            unsigned long long *last_n = (unsigned long long *)&c->misc[kLongCounts];
            if (count_first) {
                // Reads from repeat families: most candidates pair a read with
                // another copy of its family, diverged far beyond k but sharing
                // an exact window; the count filter drops them for a few
                // operations per letter, and the band pass takes the rest
                // from row 0.
                const int tok = stage_begin(c, st, PN_STAGE_COUNT);
                pn::launch_count(ref_desc(ref), index_desc(x), in, kglob, d_k, last_in, last_n,
                                 (unsigned long long *)&c->misc[kCountLetters], st);
                stage_end(c, st, tok, 1);
            } else {
                const int tok = stage_begin(c, st, PN_STAGE_VERIFY);
                pn::launch_verify(ref_desc(ref), index_desc(x), in, kglob, d_k, vo, last_in, last_n,
                                  true, st);
                stage_end(c, st, tok, 1);
            }
            vo.rows = (unsigned long long *)&c->misc[kVerifyRowsLong];
            const int tok = stage_begin(c, st, PN_STAGE_VERIFY_LONG);
            pn::launch_verify(ref_desc(ref), index_desc(x), in, kglob, d_k, vo, last_in, last_n,
                              false, st);
            // reads with k > PN_BAND_K: their candidates are all in the
            // survivor list
            if (c->wide_k)
                pn::launch_verify_wide(ref_desc(ref), index_desc(x),
                                       pn::VerifyIn{last_in, last_n, in.regions, in.region_cap},
                                       kglob, d_k, vo, st);
            stage_end(c, st, tok, c->wide_k ? 2 : 1);
            PN_CHECK(read_misc(c, st));
            uint64_t rec_max;
            region_counts(c, kRecCounts, pn::kShards, &rec_max, &got);
            if (rec_max <= c->ws.rec_rcap) break;
            c->ws.rec_rcap = rec_max + rec_max / 4;
        }
        if (filter) {
            c->stats.n_seeds += fw.seeds;
            c->stats.n_visited += fw.visited;
            c->stats.n_candidates += cand_total;
            c->stats.n_visited_heavy += fw.set_aside;
            c->stats.n_heavy_items += fw.items;
            c->stats.n_candidates_heavy += cand_total - std::min(cand_total, fw.written);
        }
        c->stats.verify_rows += c->hmisc[kVerifyRows] + c->hmisc[kVerifyRowsLong];
        c->stats.verify_rows_long += c->hmisc[kVerifyRowsLong];
        c->stats.count_letters += c->hmisc[kCountLetters];
        c->stats.n_records += got;
        PN_CHECK(ensure_keep(c, c->ws.keys, std::max<uint64_t>(total + got, 1) * 8, total * 8, st));
        const int tok = stage_begin(c, st, PN_STAGE_SORT);
        pn::launch_gather_shards((const unsigned long long *)c->ws.keys_tmp.p,
                                 (const unsigned long long *)&c->misc[kRecCounts], pn::kShards,
                                 c->ws.rec_rcap, (unsigned long long *)c->ws.keys.p + total, st);
        stage_end(c, st, tok, 1);
        total += got;
        a = b;
        attempts = 0;
    }
    *n_rec = total;
    const int bits = 6 + ebits + key_rbits(x->n_reads);
    PN_CHECK(ensure_keep(c, c->ws.keys, std::max<uint64_t>(total, 1) * 8, total * 8, st));
    PN_CHECK(ensure(c, c->ws.keys_tmp, std::max<uint64_t>(total, 1) * 8));
    PN_CHECK(ensure(c, c->ws.sort_temp, pn::radix_temp_size(total)));
    const int tok = stage_begin(c, st, PN_STAGE_SORT);
    // mapping: records need only be grouped by (read, strand, end), the
    // finishing pass takes each group's smallest error count; the records
    // pn_validate returns are sorted whole
    const int lo = filter ? 5 : 0;
    pn::radix_sort_u64((unsigned long long *)c->ws.keys.p, (unsigned long long *)c->ws.keys_tmp.p, total,
                       bits, c->ws.sort_temp.p, st, lo);
    stage_end(c, st, tok, 5 * ((bits - lo + 7) / 8));
    return PN_OK;
}

// filtration + validation; leaves the sorted record keys in c->ws.keys and
// their count in *n_rec
int map_records(pn_ctx *c, const pn_ref *ref, const pn_index *x, int kglob, const uint8_t *d_k,
                hipStream_t st, uint64_t *n_rec) {
    PN_CHECK(prepare_rules(c, x, kglob, d_k, ref->pmask[x->q] != nullptr, st));
    return validate_sorted(c, ref, x, kglob, d_k, true, 0, st, n_rec);
}

// duplicate removal + strata + output of the sorted records
int finish(pn_ctx *c, const pn_ref *ref, const pn_index *x, uint64_t n_rec, int best, void *d_out,
           uint64_t cap, hipStream_t st, uint64_t *n_out) {
    // (hit positions are 32-bit prefix sums over the records)
    if (n_rec >= 0xffffffffull) return PN_ENOMEM;
    const int ebits = key_ebits(ref->L);
    PN_CHECK(ensure(c, c->ws.flags, (n_rec + 1) * 4));
    PN_CHECK(ensure(c, c->ws.pos, (n_rec + 1) * 4));
    PN_CHECK(ensure(c, c->ws.partials, pn::scan_partials_size(n_rec + 1) * 4));
    PN_CHECK(ensure(c, c->ws.minv, ((uint64_t)x->n_reads + 1) * 4));
    int tok = stage_begin(c, st, PN_STAGE_FINISH);
    pn::launch_finish_hits((const unsigned long long *)c->ws.keys.p, n_rec, ebits, best, x->n_reads,
                           (uint32_t *)c->ws.minv.p, (uint32_t *)c->ws.flags.p, (uint32_t *)c->ws.pos.p,
                           (uint32_t *)c->ws.partials.p, d_out, cap,
                           (unsigned long long *)&c->misc[kOutCount], st);
    stage_end(c, st, tok, best ? 7 : 5);
    PN_CHECK(read_misc(c, st));
    *n_out = c->hmisc[kOutCount];
    c->stats.n_hits += *n_out;
    return PN_OK;
}

int check_map_args(pn_ctx *c, const pn_ref *ref, const pn_index *x, int k, const uint8_t *kpr,
                   pn_mode mode) {
    // the reference may come from any context on the same device
    if (!c || !ref || !x || ref->ctx->device != c->device || x->ctx != c) return PN_EINVAL;
    if (mode != PN_ALL_HITS && mode != PN_BEST_STRATUM) return PN_EINVAL;
    if (k > PN_MAX_K) return PN_EINVAL;
    if (k < 0 && !kpr && x->n_reads) return PN_EINVAL;
    return PN_OK;
}

}  // namespace

namespace pnrt {

int ctx_device(const pn_ctx *c) { return c->device; }
int ref_device(const pn_ref *r) { return r->ctx->device; }

int map_to_workspace(pn_ctx *c, const pn_ref *ref, const pn_index *x, const uint8_t *d_k,
                     bool want_all, bool want_best, const pn_hit **d_all, uint64_t *n_all,
                     const pn_hit **d_best, uint64_t *n_best, hipStream_t st) {
    PN_CHECK(check_map_args(c, ref, x, -1, d_k, PN_ALL_HITS));
    DeviceGuard g(c->device);
    uint64_t n_rec = 0;
    PN_CHECK(map_records(c, ref, x, -1, d_k, st, &n_rec));
    // each output holds at most one hit per record
    const uint64_t cap = std::max<uint64_t>(n_rec, 1);
    *n_all = *n_best = 0;
    if (want_all) {
        PN_CHECK(ensure(c, c->ws.out_hits, cap * sizeof(pn_hit)));
        PN_CHECK(finish(c, ref, x, n_rec, 0, c->ws.out_hits.p, cap, st, n_all));
        *d_all = (const pn_hit *)c->ws.out_hits.p;
    }
    if (want_best) {
        PN_CHECK(ensure(c, c->ws.out_best, cap * sizeof(pn_hit)));
        PN_CHECK(finish(c, ref, x, n_rec, 1, c->ws.out_best.p, cap, st, n_best));
        *d_best = (const pn_hit *)c->ws.out_best.p;
    }
    return PN_OK;
}

}  // namespace pnrt

extern "C" {

int pn_map_dev(pn_ctx *c, const pn_ref *ref, const pn_index *x, int k, const uint8_t *d_kpr,
               pn_mode mode, pn_hit *d_hits, uint64_t capacity, uint64_t *n_hits, void *stream) {
    PN_CHECK(check_map_args(c, ref, x, k, d_kpr, mode));
    if (!n_hits || (capacity && !d_hits)) return PN_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t st = pick_stream(c, stream);
    uint64_t n_rec = 0, n_out = 0;
    PN_CHECK(map_records(c, ref, x, k < 0 ? -1 : k, d_kpr, st, &n_rec));
    PN_CHECK(finish(c, ref, x, n_rec, mode == PN_BEST_STRATUM, d_hits, capacity, st, &n_out));
    *n_hits = n_out;
    return n_out > capacity ? PN_ETRUNC : PN_OK;
}

int pn_map(pn_ctx *c, const pn_ref *ref, const pn_index *x, int k, const uint8_t *kpr,
           pn_mode mode, pn_hit **hits, uint64_t *n_hits) {
    PN_CHECK(check_map_args(c, ref, x, k, kpr, mode));
    if (!hits || !n_hits) return PN_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    uint8_t *dk = nullptr;
    if (k < 0 && x->n_reads) {
        PN_CHECK(dalloc_t(c, x->n_reads, &dk));
        hipError_t e = hipMemcpyAsync(dk, kpr, x->n_reads, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            dfree(c, dk);
            return map_err(e);
        }
    }
    uint64_t n_rec = 0, n_out = 0;
    int s = map_records(c, ref, x, k < 0 ? -1 : k, dk, st, &n_rec);
    // the output can hold at most one hit per record
    if (!s) s = ensure(c, c->ws.out_hits, std::max<uint64_t>(n_rec, 1) * sizeof(pn_hit));
    if (!s)
        s = finish(c, ref, x, n_rec, mode == PN_BEST_STRATUM, c->ws.out_hits.p,
                   c->ws.out_hits.cap / sizeof(pn_hit), st, &n_out);
    pn_hit *h = nullptr;
    if (!s) {
        h = (pn_hit *)std::malloc(std::max<uint64_t>(n_out, 1) * sizeof(pn_hit));
        if (!h) s = PN_ENOMEM;
    }
    if (!s && n_out) {
        hipError_t e = hipMemcpyAsync(h, c->ws.out_hits.p, n_out * sizeof(pn_hit),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        s = map_err(e);
    }
    (void)hipStreamSynchronize(st);
    dfree(c, dk);
    if (s) {
        std::free(h);
        return s;
    }
    *hits = h;
    *n_hits = n_out;
    return PN_OK;
}

void pn_hits_free(pn_hit *h) { std::free(h); }

// ---- batching: a read set of any size in memory-sized sub-batches -----------

namespace {

// q and w from the cache file, or -1
void tune_cache_lookup(const char *path, const std::string &key, int *q, int *w) {
    *q = *w = -1;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char k[400];
        int a = 0, b = 0;
        if (std::sscanf(line, "%399s %d %d", k, &a, &b) == 3 && key == k) {
            *q = a;
            *w = b;
        }
    }
    std::fclose(f);
}

void tune_cache_store(const char *path, const std::string &key, int q, int w) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;  // an unwritable cache only costs a new tuning next time
    std::fprintf(f, "%s %d %d\n", key.c_str(), q, w);
    std::fclose(f);
}

}  // namespace

int pn_map_batched(pn_ctx *c, const pn_ref *ref, const char *reads, const uint64_t *offsets,
                   uint32_t n_reads, const uint8_t *k_per_read, pn_mode mode,
                   const char *tune_cache, pn_hit **hits, uint64_t *n_hits) {
    if (!c || !ref || !hits || !n_hits || (n_reads && (!offsets || !k_per_read)))
        return PN_EINVAL;
    if (mode != PN_ALL_HITS && mode != PN_BEST_STRATUM) return PN_EINVAL;
    if (ref->ctx->device != c->device) return PN_EINVAL;
    uint32_t len_lo = PN_MAX_READ_LEN, len_hi = 0, k_lo = 255, k_hi = 0;
    int q_lemma = 12;  // largest q the lemma admits for every read, at most 12
    for (uint32_t r = 0; r < n_reads; r++) {
        if (offsets[r + 1] < offsets[r]) return PN_EINVAL;
        const uint64_t n = offsets[r + 1] - offsets[r];
        const uint32_t k = k_per_read[r];
        if (n < 1 || n > PN_MAX_READ_LEN || k > PN_MAX_K) return PN_EINVAL;
        len_lo = std::min<uint32_t>(len_lo, (uint32_t)n);
        len_hi = std::max<uint32_t>(len_hi, (uint32_t)n);
        k_lo = std::min(k_lo, k);
        k_hi = std::max(k_hi, k);
        q_lemma = std::min<int>(q_lemma, (int)(n / (k + 1)));
    }
    if (n_reads && q_lemma < 1) return PN_ELEMMA;
    if (reads == nullptr && n_reads && offsets[n_reads] > offsets[0]) return PN_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    // sub-batches: at most PN_MAX_READS reads (one index) and a share of the
    // free device memory (about 48 bytes per base while an index is built
    // and mapped)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = 8ull << 30;
    }
    const uint64_t max_bases = std::max<uint64_t>(std::min<uint64_t>(free_b / 2 / 48, (1ull << 31)),
                                                  PN_MAX_READ_LEN);
    std::vector<uint32_t> cut{0};
    for (uint32_t r = 0; r < n_reads;) {
        const uint32_t r0 = r;
        while (r < n_reads && r - r0 < PN_MAX_READS &&
               offsets[r + 1] - offsets[r0] <= max_bases)
            r++;
        cut.push_back(r);
    }
    std::vector<pn_hit> out;
    int q = q_lemma, w = 64;
    bool tuned = tune_cache == nullptr;
    std::string key;
    if (!tuned) {
        char buf[400];
        int lg = 0;
        while ((1ull << (lg + 1)) <= (uint64_t)std::max<uint32_t>(n_reads, 1)) lg++;
        std::snprintf(buf, sizeof(buf), "L=%llu;reads=2^%d;len=%u-%u;k=%u-%u;mode=%d",
                      (unsigned long long)ref->L, lg, len_lo, len_hi, k_lo, k_hi, (int)mode);
        key = buf;
        int cq = -1, cw = -1;
        tune_cache_lookup(tune_cache, key, &cq, &cw);
        if (cq >= 1 && cq <= q_lemma && (cw == 32 || cw == 64)) {
            q = cq;
            w = cw;
            tuned = true;
        }
    }
    int s = PN_OK;
    for (size_t b = 0; b + 1 < cut.size() && !s; b++) {
        const uint32_t r0 = cut[b], r1 = cut[b + 1], m = r1 - r0;
        const uint64_t base = offsets[r0], nb = offsets[r1] - base;
        std::vector<uint64_t> offs(m + 1);
        for (uint32_t i = 0; i <= m; i++) offs[i] = offsets[r0 + i] - base;
        char *dr = nullptr;
        uint64_t *doff = nullptr;
        uint8_t *dk = nullptr;
        pn_index *x = nullptr;
        s = dalloc_t(c, nb + 1, &dr);
        if (!s) s = dalloc_t(c, (uint64_t)m + 1, &doff);
        if (!s) s = dalloc_t(c, (uint64_t)m + 1, &dk);
        if (!s && nb) s = map_err(hipMemcpyAsync(dr, reads + base, nb, hipMemcpyHostToDevice, st));
        if (!s)
            s = map_err(hipMemcpyAsync(doff, offs.data(), ((uint64_t)m + 1) * 8,
                                       hipMemcpyHostToDevice, st));
        if (!s) s = map_err(hipMemcpyAsync(dk, k_per_read + r0, m, hipMemcpyHostToDevice, st));
        if (!s && !tuned) {
            // the autotuner times each admitted (q, w) on a sample of this
            // first sub-batch and predicts the whole batch
            pn_tune_result res[6];
            int nres = 0, bq = 0, bw = 0;
            s = pn_autotune(c, ref, dr, doff, m, nb, -1, dk, mode, std::min<uint32_t>(m, 1u << 16),
                            res, &nres, &bq, &bw);
            if (!s) {
                q = bq;
                w = bw;
                tuned = true;
                tune_cache_store(tune_cache, key, q, w);
            }
        }
        if (!s) s = pn_index_build_dev(c, dr, doff, m, nb, q, w, st, &x);
        uint64_t n_rec = 0, n_out = 0;
        if (!s) s = map_records(c, ref, x, -1, dk, st, &n_rec);
        if (!s) s = ensure(c, c->ws.out_hits, std::max<uint64_t>(n_rec, 1) * sizeof(pn_hit));
        if (!s)
            s = finish(c, ref, x, n_rec, mode == PN_BEST_STRATUM, c->ws.out_hits.p,
                       c->ws.out_hits.cap / sizeof(pn_hit), st, &n_out);
        if (!s && n_out) {
            const size_t at = out.size();
            out.resize(at + n_out);
            s = map_err(hipMemcpyAsync(out.data() + at, c->ws.out_hits.p, n_out * sizeof(pn_hit),
                                       hipMemcpyDeviceToHost, st));
            if (!s) s = map_err(hipStreamSynchronize(st));
            for (size_t i = at; !s && i < out.size(); i++) out[i].read_id += r0;
        }
        (void)hipStreamSynchronize(st);
        if (x) pn_index_free(x);
        dfree(c, dr);
        dfree(c, doff);
        dfree(c, dk);
    }
    if (s) return s;
    pn_hit *h = (pn_hit *)std::malloc(std::max<size_t>(out.size(), 1) * sizeof(pn_hit));
    if (!h) return PN_ENOMEM;
    if (!out.empty()) std::memcpy(h, out.data(), out.size() * sizeof(pn_hit));
    *hits = h;
    *n_hits = out.size();
    return PN_OK;
}

int pn_filter(pn_ctx *c, const pn_ref *ref, const pn_index *x, int k, const uint8_t *kpr,
              pn_candidate **cands, uint64_t *n_cands, uint64_t *n_seeds) {
    PN_CHECK(check_map_args(c, ref, x, k, kpr, PN_ALL_HITS));
    if (!cands || !n_cands) return PN_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    uint8_t *dk = nullptr;
    if (k < 0 && x->n_reads) {
        PN_CHECK(dalloc_t(c, x->n_reads, &dk));
        hipError_t e = hipMemcpyAsync(dk, kpr, x->n_reads, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            dfree(c, dk);
            return map_err(e);
        }
    }
    int s = prepare_rules(c, x, k < 0 ? -1 : k, dk, ref->pmask[x->q] != nullptr, st);
    pn::RefQDev P{nullptr, nullptr, 0, nullptr};
    if (!s) s = ref_prepare(const_cast<pn_ref *>(ref), x->q, st, &P);
    uint64_t n = 0;
    // (the whole position set at once: this call returns every candidate)
    for (int attempt = 0; !s && attempt < 8; attempt++) {
        s = ensure(c, c->ws.cands, pn::kShards * c->ws.cand_rcap * sizeof(uint2));
        if (s) break;
        pn::launch_fill_u32((uint32_t *)&c->misc[kFilterStats], 8 * pn::kShards, 0u, st);
        zero_counts(c, kCandCounts, st);
        s = launch_filter_into(c, ref, x, P, 0, P.n, st);
        if (!s) s = read_misc(c, st);
        if (s) break;
        uint64_t mx;
        region_counts(c, kCandCounts, pn::kShards, &mx, &n);
        const uint64_t hmax = heavy_max(c);
        if (mx <= c->ws.cand_rcap && hmax <= c->ws.heavy_rcap) break;
        if (mx > c->ws.cand_rcap) c->ws.cand_rcap = mx + mx / 4;
        if (hmax > c->ws.heavy_rcap) c->ws.heavy_rcap = hmax + hmax / 4;
        n = 0;
    }
    uint64_t seeds = 0;
    if (!s) seeds = filter_stats(c).seeds;
    if (!s) s = ensure(c, c->ws.keys, std::max<uint64_t>(n, 1) * 8);
    if (!s) s = ensure(c, c->ws.keys_tmp, std::max<uint64_t>(n, 1) * 8);
    if (!s) s = ensure(c, c->ws.sort_temp, pn::radix_temp_size(n));
    if (!s) s = ensure(c, c->ws.out_hits, std::max<uint64_t>(n, 1) * sizeof(pn_candidate));
    pn_candidate *h = nullptr;
    if (!s) {
        if (n) {
            pn::launch_gather_shards((const unsigned long long *)c->ws.cands.p,
                                     (const unsigned long long *)&c->misc[kCandCounts],
                                     pn::kShards, c->ws.cand_rcap,
                                     (unsigned long long *)c->ws.keys_tmp.p, st);
            pn::launch_cand_keys((const uint2 *)c->ws.keys_tmp.p, n, (unsigned long long *)c->ws.keys.p,
                                 st);
            pn::radix_sort_u64((unsigned long long *)c->ws.keys.p, (unsigned long long *)c->ws.keys_tmp.p,
                               n, 33 + key_rbits(x->n_reads), c->ws.sort_temp.p, st);
            pn::launch_keys_to_cands((const unsigned long long *)c->ws.keys.p, n, c->ws.out_hits.p, st);
        }
        h = (pn_candidate *)std::malloc(std::max<uint64_t>(n, 1) * sizeof(pn_candidate));
        if (!h) s = PN_ENOMEM;
    }
    if (!s && n)
        s = map_err(hipMemcpyAsync(h, c->ws.out_hits.p, n * sizeof(pn_candidate),
                                   hipMemcpyDeviceToHost, st));
    if (!s) s = map_err(hipStreamSynchronize(st));
    dfree(c, dk);
    if (s) {
        std::free(h);
        return s;
    }
    // padding slots (read id all ones) sort last
    while (n && h[n - 1].read_id == 0x7fffffffu) n--;
    *cands = h;
    *n_cands = n;
    if (n_seeds) *n_seeds = seeds;
    return PN_OK;
}

int pn_validate(pn_ctx *c, const pn_ref *ref, const pn_index *x, const pn_candidate *cands,
                uint64_t n, int k, const uint8_t *kpr, pn_hit **records, uint64_t *n_records) {
    PN_CHECK(check_map_args(c, ref, x, k, kpr, PN_ALL_HITS));
    if (!records || !n_records || (n && !cands) || n >= (1ull << 32)) return PN_EINVAL;
    std::vector<uint2> host(n);
    for (uint64_t i = 0; i < n; i++) {
        const pn_candidate &cd = cands[i];
        if (cd.read_id >= x->n_reads || cd.strand > 1 || cd.diagonal < -(int64_t)PN_MAX_READ_LEN ||
            cd.diagonal > (int64_t)ref->L)
            return PN_EINVAL;
        host[i] = make_uint2(cd.read_id | ((uint32_t)cd.strand << 31),
                             (uint32_t)(cd.diagonal + (int64_t)PN_DBIAS));
    }
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    uint8_t *dk = nullptr;
    if (k < 0 && x->n_reads) {
        PN_CHECK(dalloc_t(c, x->n_reads, &dk));
        hipError_t e = hipMemcpyAsync(dk, kpr, x->n_reads, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            dfree(c, dk);
            return map_err(e);
        }
    }
    int s = prepare_rules(c, x, k < 0 ? -1 : k, dk, false, st);
    if (!s) s = ensure(c, c->ws.cands, std::max<uint64_t>(n, 1) * sizeof(uint2));
    if (!s && n)
        s = map_err(hipMemcpyAsync(c->ws.cands.p, host.data(), n * sizeof(uint2),
                                   hipMemcpyHostToDevice, st));
    if (!s) pn::launch_cands_len((uint2 *)c->ws.cands.p, n, x->offsets, st);
    uint64_t got = 0;
    const int ebits = key_ebits(ref->L);
    if (!s) s = validate_sorted(c, ref, x, k < 0 ? -1 : k, dk, false, n, st, &got);
    if (!s) s = ensure(c, c->ws.out_hits, std::max<uint64_t>(got, 1) * sizeof(pn_hit));
    pn_hit *h = nullptr;
    if (!s) {
        pn::launch_records_to_hits((const unsigned long long *)c->ws.keys.p, got, ebits, c->ws.out_hits.p,
                                   st);
        h = (pn_hit *)std::malloc(std::max<uint64_t>(got, 1) * sizeof(pn_hit));
        if (!h) s = PN_ENOMEM;
    }
    if (!s && got)
        s = map_err(hipMemcpyAsync(h, c->ws.out_hits.p, got * sizeof(pn_hit), hipMemcpyDeviceToHost,
                                   st));
    if (!s) s = map_err(hipStreamSynchronize(st));
    dfree(c, dk);
    if (s) {
        std::free(h);
        return s;
    }
    *records = h;
    *n_records = got;
    return PN_OK;
}

int pn_align(pn_ctx *c, const pn_ref *ref, const pn_index *x, const pn_hit *hits, uint64_t n,
             uint32_t *starts, uint8_t *errors, uint8_t *ops, uint32_t stride, uint16_t *n_ops) {
    if (!c || !ref || !x || ref->ctx->device != c->device || x->ctx != c) return PN_EINVAL;
    if (n && (!hits || !starts || !errors)) return PN_EINVAL;
    for (uint64_t h = 0; h < n; h++) {
        const pn_hit &t = hits[h];
        if (t.read_id >= x->n_reads || t.strand > 1 || t.end_pos >= ref->L || t.errors > PN_MAX_K)
            return PN_EINVAL;
    }
    if (!n) return PN_OK;
    static_assert(sizeof(pn_hit) == 12, "hit records are three words");
    const bool want_ops = n_ops != nullptr;
    const uint32_t ost = want_ops && ops ? stride : 0;
    // chunks whose op-code rows fit 512 MiB (two words per row for bands of
    // more than 32 diagonals)
    uint32_t vmax = 0;
    for (uint64_t h = 0; h < n; h++) vmax = std::max<uint32_t>(vmax, hits[h].errors);
    const uint64_t rows =
        (uint64_t)std::max(x->max_len, 1) * (vmax > PN_BAND_K ? 2ull : 1ull);
    const uint64_t chunk = std::min<uint64_t>(n, std::max<uint64_t>(64, (512ull << 20) / (rows * 8)));
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    uint32_t *dh = nullptr, *dperm = nullptr, *dstart = nullptr;
    unsigned long long *bp = nullptr;
    uint8_t *derr = nullptr, *dops = nullptr;
    uint16_t *dnops = nullptr;
    int s = dalloc_t(c, chunk * 3, &dh);
    if (!s) s = dalloc_t(c, chunk, &dperm);
    if (!s) s = dalloc_t(c, chunk * rows, &bp);
    if (!s) s = dalloc_t(c, chunk, &dstart);
    if (!s) s = dalloc_t(c, chunk, &derr);
    if (!s && ost) s = dalloc_t(c, chunk * ost, &dops);
    if (!s && want_ops) s = dalloc_t(c, chunk, &dnops);
    std::vector<uint32_t> perm(chunk);
    const PnRefDev rd = ref_desc(ref);
    const PnIndexDev xd = index_desc(x);
    for (uint64_t c0 = 0; !s && c0 < n; c0 += chunk) {
        const uint64_t m = std::min(chunk, n - c0);
        // the chunk's hits grouped by error count (one launch per count)
        uint32_t cnt[PN_MAX_K + 1] = {}, off[PN_MAX_K + 2] = {};
        for (uint64_t h = 0; h < m; h++) cnt[hits[c0 + h].errors]++;
        for (int v = 0; v <= PN_MAX_K; v++) off[v + 1] = off[v] + cnt[v];
        uint32_t at[PN_MAX_K + 1];
        for (int v = 0; v <= PN_MAX_K; v++) at[v] = off[v];
        for (uint64_t h = 0; h < m; h++) perm[at[hits[c0 + h].errors]++] = (uint32_t)h;
        s = map_err(hipMemcpyAsync(dh, hits + c0, m * sizeof(pn_hit), hipMemcpyHostToDevice, st));
        if (!s)
            s = map_err(hipMemcpyAsync(dperm, perm.data(), m * 4, hipMemcpyHostToDevice, st));
        const int tok = s ? -1 : stage_begin(c, st, PN_STAGE_ALIGN);
        int launches = 0;
        for (int v = 0; !s && v <= PN_MAX_K; v++) {
            if (!cnt[v]) continue;
            pn::launch_align(rd, xd, v, dh, dperm + off[v], cnt[v], bp, dstart, derr, dops, ost,
                             dnops, st);
            launches++;
        }
        stage_end(c, st, tok, launches);
        if (!s) s = map_err(hipGetLastError());
        if (!s)
            s = map_err(hipMemcpyAsync(starts + c0, dstart, m * 4, hipMemcpyDeviceToHost, st));
        if (!s) s = map_err(hipMemcpyAsync(errors + c0, derr, m, hipMemcpyDeviceToHost, st));
        if (!s && ost)
            s = map_err(hipMemcpyAsync(ops + c0 * ost, dops, m * ost, hipMemcpyDeviceToHost, st));
        if (!s && want_ops)
            s = map_err(hipMemcpyAsync(n_ops + c0, dnops, m * 2, hipMemcpyDeviceToHost, st));
        if (!s) s = map_err(hipStreamSynchronize(st));
        if (!s) collect_stages(c);
    }
    if (s) (void)hipStreamSynchronize(st);
    dfree(c, dh);
    dfree(c, dperm);
    dfree(c, bp);
    dfree(c, dstart);
    dfree(c, derr);
    dfree(c, dops);
    dfree(c, dnops);
    return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// validation without allocation: a fixed device array per device

namespace {

// Limits of pn_validate_noalloc and the layout of its array (byte offsets,
// each a multiple of 256).
constexpr uint64_t kNaMaxCands = 1ull << 16;
constexpr uint64_t kNaRegionCap = 1ull << 15;  // records per output region
constexpr uint64_t kNaMaxRecords = 1ull << 20;
constexpr uint64_t kNaTempBytes = 2ull << 20;  // radix sort counts and offsets
constexpr uint64_t kNaRinfo = 0;
constexpr uint64_t kNaCands = kNaRinfo + (((uint64_t)PN_MAX_READS + 1 + 255) & ~255ull);
constexpr uint64_t kNaLong = kNaCands + kNaMaxCands * 8;
constexpr uint64_t kNaRegions = kNaLong + kNaMaxCands * 8;
constexpr uint64_t kNaKeys = kNaRegions + pn::kShards * kNaRegionCap * 8;
constexpr uint64_t kNaTmp = kNaKeys + kNaMaxRecords * 8;
constexpr uint64_t kNaTemp = kNaTmp + kNaMaxRecords * 8;
constexpr uint64_t kNaBytes = kNaTemp + kNaTempBytes;  // 37 MiB
constexpr int kNaMaxDevices = 64;

// Its device copy (one per device, at a device address that the host
// learns from hipGetSymbolAddress; host code never passes the name itself).
__device__ __align__(256) unsigned char scratch[kNaBytes];

std::mutex g_na_mu;
unsigned char *g_na_ptr[kNaMaxDevices] = {};

// Once per device, with that device current: the array's device address.
int noalloc_setup(int device) {
    if (device < 0 || device >= kNaMaxDevices) return PN_EDEVICE;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (g_na_ptr[device]) return PN_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return PN_EDEVICE;
    }
    g_na_ptr[device] = (unsigned char *)p;
    return PN_OK;
}

unsigned char *noalloc_ptr(int device) {
    if (device < 0 || device >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_na_mu);
    return g_na_ptr[device];
}

// the context's misc words back to the host (no stage bookkeeping)
int na_sync_misc(pn_ctx *c, hipStream_t st) {
    PN_TRY(hipMemcpyAsync(c->hmisc, c->misc, kMiscWords * sizeof(uint64_t), hipMemcpyDeviceToHost,
                          st));
    PN_TRY(hipStreamSynchronize(st));
    return PN_OK;
}

}  // namespace

int pnrt_noalloc_setup(int device) { return noalloc_setup(device); }

extern "C" {

int pn_validate_noalloc(pn_ctx *c, const pn_ref *ref, const pn_index *x,
                        const pn_candidate *d_cands, uint64_t n, int k,
                        const uint8_t *d_k_per_read, pn_hit *d_records, uint64_t capacity,
                        uint64_t *n_records, void *stream) {
    PN_CHECK(check_map_args(c, ref, x, k, d_k_per_read, PN_ALL_HITS));
    if (!n_records || (n && !d_cands) || (capacity && !d_records) || n > kNaMaxCands)
        return PN_EINVAL;
    DeviceGuard g(c->device);
    unsigned char *base = noalloc_ptr(c->device);
    if (!base) return PN_EDEVICE;
    hipStream_t st = pick_stream(c, stream);
    const int kglob = k < 0 ? -1 : k;
    uint2 *cands = (uint2 *)(base + kNaCands);
    uint2 *longc = (uint2 *)(base + kNaLong);
    unsigned long long *regions = (unsigned long long *)(base + kNaRegions);
    unsigned long long *keys = (unsigned long long *)(base + kNaKeys);
    unsigned long long *tmp = (unsigned long long *)(base + kNaTmp);
    const PnIndexDev ix = index_desc(x);
    // k and the lemma per read (as the mapping checks them), the candidates
    // converted and range-checked
    zero_misc(c, st);
    pn::launch_read_rules(ix, kglob, d_k_per_read, base + kNaRinfo, nullptr,
                          (uint32_t *)&c->misc[kStatus], false, st);
    pn::launch_cands_in(d_cands, n, x->n_reads, ref->L, x->offsets, cands,
                        (uint32_t *)&c->misc[kStatus], st);
    pn::launch_fill_u32((uint32_t *)&c->misc[kCandCounts], 1, (uint32_t)n, st);
    PN_CHECK(na_sync_misc(c, st));
    const uint32_t status = (uint32_t)c->hmisc[kStatus];
    if (status & (2u | 8u)) return PN_EINVAL;
    if (status & 4u) return PN_ELEMMA;
    // both verification passes, records into the array's regions
    const int ebits = key_ebits(ref->L);
    const uint64_t in_cap = std::max<uint64_t>(n, 1);
    pn::VerifyIn in{cands, (const unsigned long long *)&c->misc[kCandCounts], 1, in_cap};
    pn::VerifyOut vo{regions, {(unsigned long long *)&c->misc[kRecCounts], kNaRegionCap},
                     (unsigned long long *)&c->misc[kVerifyRows], ebits};
    if (n) {
        pn::launch_verify(ref_desc(ref), ix, in, kglob, d_k_per_read, vo, longc,
                          (unsigned long long *)&c->misc[kLongCounts], true, st);
        pn::launch_verify(ref_desc(ref), ix, in, kglob, d_k_per_read, vo, longc,
                          (unsigned long long *)&c->misc[kLongCounts], false, st);
        if (status & 16u)
            pn::launch_verify_wide(ref_desc(ref), ix,
                                   pn::VerifyIn{longc, (const unsigned long long *)&c->misc[kLongCounts],
                                                1, in_cap},
                                   kglob, d_k_per_read, vo, st);
    }
    PN_CHECK(na_sync_misc(c, st));
    uint64_t rmax = 0, total = 0;
    region_counts(c, kRecCounts, pn::kShards, &rmax, &total);
    if (rmax > kNaRegionCap || total > kNaMaxRecords) return PN_EINVAL;
    if (total > capacity) {
        *n_records = total;
        return PN_ETRUNC;
    }
    if (pn::radix_temp_size(total) > kNaTempBytes) return PN_EINVAL;
    if (total) {
        pn::launch_gather_shards(regions, (const unsigned long long *)&c->misc[kRecCounts],
                                 pn::kShards, kNaRegionCap, keys, st);
        unsigned long long *sorted = pn::radix_sort_u64_any(
            keys, tmp, total, 6 + ebits + key_rbits(x->n_reads), base + kNaTemp, st);
        pn::launch_records_to_hits(sorted, total, ebits, d_records, st);
    }
    PN_TRY(hipStreamSynchronize(st));
    *n_records = total;
    return PN_OK;
}

}  // extern "C"
