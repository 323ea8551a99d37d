// Serving: continuous batching of mapping requests over a resident
// reference (the queued, layered pipeline of Fig. 2; reads buffered into
// batches that share one q-group index, Section 3.1).
//
// Requests wait in a FIFO queue.  Each slot (a worker thread with its own
// pn_ctx, hence its own HIP stream and workspace) takes the queued requests
// that fit one batch, concatenates their reads in pinned host memory,
// copies them to the device, builds one index, maps it (all hits and/or the
// best stratum from one set of records), copies the hits back and splits
// them per request by read-id range.  Mapping is per read, so a request's
// hits are those it would get alone.  Admission is by an estimate of each
// batch's working set against the HBM budget; a batch's estimate is held
// until it completes.  Stream priorities stay at the default.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pn_runtime.h"

#define SV_CHECK(st)                \
    do {                            \
        const int s_ = (st);        \
        if (s_ != PN_OK) return s_; \
    } while (0)

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

uint64_t estimate_bytes(uint64_t n_reads, uint64_t n_bases) {
    return 12ull * n_bases + 4096ull * n_reads + (16ull << 20);
}

struct Request {
    uint64_t ticket = 0;
    std::vector<char> reads;
    std::vector<uint64_t> offsets;  // n_reads + 1, from 0
    std::vector<uint8_t> k;         // per read
    bool best = false;
    uint64_t est = 0;
    double t_submit = 0, t_done = 0;
    int status = PN_OK;
    bool done = false;
    std::vector<pn_hit> hits;
    uint32_t n_reads() const { return (uint32_t)(offsets.size() - 1); }
};

// grow-only buffers of one slot
struct Slot {
    pn_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    std::thread th;
    char *h_reads = nullptr, *d_reads = nullptr;
    uint64_t *h_offs = nullptr, *d_offs = nullptr;
    uint8_t *h_k = nullptr, *d_k = nullptr;
    pn_hit *h_all = nullptr, *h_best = nullptr;
    size_t cap_reads = 0, cap_offs = 0, cap_k = 0, cap_all = 0, cap_best = 0;
};

template <typename T>
int grow_pinned(T **p, size_t *cap, size_t count) {
    if (*cap >= count && *p) return PN_OK;
    size_t n = std::max<size_t>(count, 1);
    n += n / 4;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipHostMalloc((void **)p, n * sizeof(T), 0) != hipSuccess) return PN_ENOMEM;
    *cap = n;
    return PN_OK;
}

template <typename T>
int grow_device(T **p, size_t *cap, size_t count) {
    if (*cap >= count && *p) return PN_OK;
    size_t n = std::max<size_t>(count, 1);
    n += n / 4;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) return PN_ENOMEM;
    *cap = n;
    return PN_OK;
}

}  // namespace

struct pn_server {
    int device = 0;
    const pn_ref *ref = nullptr;
    pn_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_ticket = 1;
    uint64_t in_use = 0;  // estimated bytes of batches in flight
    bool stop = false;
    std::vector<Slot *> slots;
    pn_server_stats stats{};
};

namespace {

// capacities of a slot's device input buffers
struct DevCaps {
    size_t reads = 0, offs = 0, k = 0;
};

int run_batch(pn_server *s, Slot *sl, DevCaps &dc, const std::vector<Request *> &batch,
              uint64_t *n_delivered) {
    uint64_t nr = 0, nb = 0;
    bool want_all = false, want_best = false;
    for (Request *r : batch) {
        nr += r->n_reads();
        nb += r->offsets.back();
        (r->best ? want_best : want_all) = true;
    }
    SV_CHECK(grow_pinned(&sl->h_reads, &sl->cap_reads, nb));
    SV_CHECK(grow_pinned(&sl->h_offs, &sl->cap_offs, nr + 1));
    SV_CHECK(grow_pinned(&sl->h_k, &sl->cap_k, nr));
    uint64_t rb = 0, ro = 0;
    sl->h_offs[0] = 0;
    for (Request *r : batch) {
        std::memcpy(sl->h_reads + rb, r->reads.data(), r->offsets.back());
        for (uint32_t i = 0; i < r->n_reads(); i++) sl->h_offs[ro + i + 1] = rb + r->offsets[i + 1];
        std::memcpy(sl->h_k + ro, r->k.data(), r->n_reads());
        rb += r->offsets.back();
        ro += r->n_reads();
    }
    SV_CHECK(grow_device(&sl->d_reads, &dc.reads, nb));
    SV_CHECK(grow_device(&sl->d_offs, &dc.offs, nr + 1));
    SV_CHECK(grow_device(&sl->d_k, &dc.k, nr));
    hipStream_t st = sl->stream;
    if (nb && hipMemcpyAsync(sl->d_reads, sl->h_reads, nb, hipMemcpyHostToDevice, st) != hipSuccess)
        return PN_EDEVICE;
    if (hipMemcpyAsync(sl->d_offs, sl->h_offs, (nr + 1) * 8, hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return PN_EDEVICE;
    if (nr && hipMemcpyAsync(sl->d_k, sl->h_k, nr, hipMemcpyHostToDevice, st) != hipSuccess)
        return PN_EDEVICE;
    pn_index *x = nullptr;
    SV_CHECK(pn_index_build_dev(sl->ctx, sl->d_reads, sl->d_offs, (uint32_t)nr, nb, s->cfg.q,
                                s->cfg.w, st, &x));
    const pn_hit *d_all = nullptr, *d_best = nullptr;
    uint64_t n_all = 0, n_best = 0;
    int rc = pnrt::map_to_workspace(sl->ctx, s->ref, x, sl->d_k, want_all, want_best, &d_all,
                                    &n_all, &d_best, &n_best, st);
    if (!rc && want_all) rc = grow_pinned(&sl->h_all, &sl->cap_all, n_all);
    if (!rc && want_best) rc = grow_pinned(&sl->h_best, &sl->cap_best, n_best);
    if (!rc && n_all &&
        hipMemcpyAsync(sl->h_all, d_all, n_all * sizeof(pn_hit), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
        rc = PN_EDEVICE;
    if (!rc && n_best &&
        hipMemcpyAsync(sl->h_best, d_best, n_best * sizeof(pn_hit), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
        rc = PN_EDEVICE;
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = PN_EDEVICE;
    pn_index_free(x);
    if (rc) return rc;
    // hits are sorted by read id: each request owns one contiguous range
    uint32_t r0 = 0;
    *n_delivered = 0;
    for (Request *r : batch) {
        const pn_hit *h = r->best ? sl->h_best : sl->h_all;
        const uint64_t n = r->best ? n_best : n_all;
        const uint32_t r1 = r0 + r->n_reads();
        auto lo = std::lower_bound(h, h + n, r0,
                                   [](const pn_hit &a, uint32_t v) { return a.read_id < v; });
        auto hi = std::lower_bound(lo, h + n, r1,
                                   [](const pn_hit &a, uint32_t v) { return a.read_id < v; });
        r->hits.assign(lo, hi);
        for (pn_hit &e : r->hits) e.read_id -= r0;
        *n_delivered += r->hits.size();
        r0 = r1;
    }
    return PN_OK;
}

void worker(pn_server *s, Slot *sl) {
    (void)hipSetDevice(s->device);
    DevCaps dc;
    for (;;) {
        std::vector<Request *> batch;
        uint64_t est = 0, reads = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return (s->stop && s->queue.empty()) ||
                       (!s->queue.empty() && s->in_use + s->queue.front()->est <= s->cfg.hbm_budget);
            });
            if (s->queue.empty()) return;  // stopping
            uint64_t bases = 0;
            while (!s->queue.empty()) {
                Request *r = s->queue.front();
                const uint64_t nb = r->offsets.back();
                if (!batch.empty() &&
                    (reads + r->n_reads() > s->cfg.max_batch_reads || bases + nb >= (1ull << 32) ||
                     s->in_use + est + r->est > s->cfg.hbm_budget))
                    break;
                batch.push_back(r);
                s->queue.pop_front();
                reads += r->n_reads();
                bases += nb;
                est += r->est;
            }
            s->in_use += est;
        }
        uint64_t delivered = 0;
        const int rc = run_batch(s, sl, dc, batch, &delivered);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->in_use -= est;
            const double t = now_ms();
            for (Request *r : batch) {
                r->status = rc;
                if (rc) r->hits.clear();
                r->done = true;
                r->t_done = t;
            }
            s->stats.requests += batch.size();
            s->stats.batches += 1;
            s->stats.reads += reads;
            s->stats.hits += rc ? 0 : delivered;
            s->stats.max_batch_reads = std::max<uint64_t>(s->stats.max_batch_reads, reads);
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

void free_slot(Slot *sl) {
    if (sl->h_reads) (void)hipHostFree(sl->h_reads);
    if (sl->h_offs) (void)hipHostFree(sl->h_offs);
    if (sl->h_k) (void)hipHostFree(sl->h_k);
    if (sl->h_all) (void)hipHostFree(sl->h_all);
    if (sl->h_best) (void)hipHostFree(sl->h_best);
    if (sl->d_reads) (void)hipFree(sl->d_reads);
    if (sl->d_offs) (void)hipFree(sl->d_offs);
    if (sl->d_k) (void)hipFree(sl->d_k);
    if (sl->ctx) pn_ctx_destroy(sl->ctx);
    delete sl;
}

}  // namespace

extern "C" {

int pn_server_create(pn_ctx *ctx, const pn_ref *ref, const pn_server_config *cfg,
                     pn_server **out) {
    if (!ctx || !ref || !cfg || !out) return PN_EINVAL;
    if (pnrt::ctx_device(ctx) != pnrt::ref_device(ref)) return PN_EINVAL;
    if (cfg->q < 1 || cfg->q > PN_MAX_Q || (cfg->w != 32 && cfg->w != 64) || cfg->slots < 1 ||
        cfg->slots > 8 || cfg->max_batch_reads < 1 || cfg->max_batch_reads > PN_MAX_READS ||
        cfg->hbm_budget == 0)
        return PN_EINVAL;
    // the reference's q-gram-sorted position set, before the first request
    const int prc = pn_ref_prepare(const_cast<pn_ref *>(ref), cfg->q);
    if (prc) return prc;
    pn_server *s = new (std::nothrow) pn_server();
    if (!s) return PN_ENOMEM;
    s->device = pnrt::ref_device(ref);
    s->ref = ref;
    s->cfg = *cfg;
    int rc = PN_OK;
    for (int i = 0; i < cfg->slots && !rc; i++) {
        Slot *sl = new (std::nothrow) Slot();
        if (!sl) {
            rc = PN_ENOMEM;
            break;
        }
        rc = pn_ctx_create(s->device, &sl->ctx);
        if (!rc) rc = pn_ctx_stream(sl->ctx, (void **)&sl->stream);
        if (rc) {
            free_slot(sl);
            break;
        }
        s->slots.push_back(sl);
    }
    if (rc) {
        for (Slot *sl : s->slots) free_slot(sl);
        delete s;
        return rc;
    }
    for (Slot *sl : s->slots) sl->th = std::thread(worker, s, sl);
    *out = s;
    return PN_OK;
}

int pn_server_submit(pn_server *s, const char *reads, const uint64_t *offsets, uint32_t n_reads,
                     int k, const uint8_t *k_per_read, pn_mode mode, uint64_t *ticket) {
    if (!s || !ticket || !offsets || (k < 0 && !k_per_read && n_reads)) return PN_EINVAL;
    if (mode != PN_ALL_HITS && mode != PN_BEST_STRATUM) return PN_EINVAL;
    if (k > PN_MAX_K) return PN_EINVAL;
    const uint64_t base = offsets[0];
    const uint64_t nb = offsets[n_reads] - base;
    if (offsets[n_reads] < base || (nb && !reads) || nb >= (1ull << 32)) return PN_EINVAL;
    if (n_reads > PN_MAX_READS) return PN_EBUDGET;  // one index holds at most this many
    const uint64_t est = estimate_bytes(n_reads, nb);
    if (est > s->cfg.hbm_budget) return PN_EBUDGET;
    Request *r = new (std::nothrow) Request();
    if (!r) return PN_ENOMEM;
    r->best = mode == PN_BEST_STRATUM;
    r->est = est;
    r->offsets.resize((size_t)n_reads + 1);
    r->k.resize(n_reads);
    r->reads.assign(reads + base, reads + base + nb);
    bool ok[256] = {};
    for (const char *c = "ACGTacgt"; *c; c++) ok[(uint8_t)*c] = true;
    int rc = PN_OK;
    for (uint32_t i = 0; i < n_reads && !rc; i++) {
        if (offsets[i + 1] < offsets[i]) {
            rc = PN_EINVAL;
            break;
        }
        const uint64_t n = offsets[i + 1] - offsets[i];
        const int kr = k >= 0 ? k : (int)k_per_read[i];
        r->offsets[i] = offsets[i] - base;
        r->k[i] = (uint8_t)kr;
        if (n < 1 || n > PN_MAX_READ_LEN || kr > PN_MAX_K) rc = PN_EINVAL;
        else if ((uint64_t)(kr + 1) * s->cfg.q > n) rc = PN_ELEMMA;
    }
    r->offsets[n_reads] = nb;
    for (uint64_t i = 0; i < nb && !rc; i++)
        if (!ok[(uint8_t)r->reads[i]]) rc = PN_EALPHABET;
    if (rc) {
        delete r;
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        r->t_submit = now_ms();
        if (n_reads == 0) {
            r->done = true;
            r->t_done = r->t_submit;
            s->stats.requests += 1;
        } else {
            s->queue.push_back(r);
        }
        s->reqs[r->ticket] = r;
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return PN_OK;
}

namespace {

// hand a finished request's hits to the caller and delete it
int redeem(Request *r, pn_hit **hits, uint64_t *n_hits, double *latency_ms) {
    const int rc = r->status;
    if (latency_ms) *latency_ms = r->t_done - r->t_submit;
    *hits = nullptr;
    *n_hits = 0;
    if (!rc) {
        pn_hit *h = (pn_hit *)std::malloc(std::max<size_t>(r->hits.size(), 1) * sizeof(pn_hit));
        if (!h) {
            delete r;
            return PN_ENOMEM;
        }
        if (!r->hits.empty()) std::memcpy(h, r->hits.data(), r->hits.size() * sizeof(pn_hit));
        *hits = h;
        *n_hits = r->hits.size();
    }
    delete r;
    return rc;
}

}  // namespace

int pn_server_wait(pn_server *s, uint64_t ticket, pn_hit **hits, uint64_t *n_hits,
                   double *latency_ms) {
    if (!s || !hits || !n_hits) return PN_EINVAL;
    Request *r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return PN_EINVAL;
        r = it->second;
        s->cv_done.wait(lk, [&] { return r->done; });
        s->reqs.erase(it);
    }
    return redeem(r, hits, n_hits, latency_ms);
}

int pn_poll(pn_server *s, uint64_t ticket, pn_hit **hits, uint64_t *n_hits, double *latency_ms) {
    if (!s || !hits || !n_hits) return PN_EINVAL;
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return PN_EINVAL;
        if (!it->second->done) return PN_PENDING;
        r = it->second;
        s->reqs.erase(it);
    }
    return redeem(r, hits, n_hits, latency_ms);
}

int pn_server_get_stats(pn_server *s, pn_server_stats *out) {
    if (!s || !out) return PN_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return PN_OK;
}

void pn_server_destroy(pn_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (Slot *sl : s->slots)
        if (sl->th.joinable()) sl->th.join();
    for (Slot *sl : s->slots) free_slot(sl);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
}

}  // extern "C"
