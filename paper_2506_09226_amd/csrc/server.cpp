// Request loop of the served form: footprint admission, continuous batching
// of same-template queries into shared scans, batches in flight on several
// HIP streams, completion by event polling, per-query latency and status.
//
// Errors.  Each stream slot has its own context, so its own device status
// word; the word is copied to pinned host memory at the end of every batch
// and read when the batch retires.  A batch of several queries that reports
// an error is not charged to all of them: each query is run again alone.  A
// query alone that overflows its group table (GQ_ERR_CAPACITY) is run again
// with twice the group bound, up to its output capacity; past that, the
// query reports GQ_ERR_CAPACITY (the caller may retry with larger outputs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_serve.h"
#include "gq_serve_policy.h"

namespace {

using clk = std::chrono::steady_clock;

struct pending {
    uint64_t ticket;
    gq_serve_query q;
    clk::time_point submitted;
    bool solo = false;                    // run alone (a re-run after a batch error)
};

struct done_state {
    bool done = false;
    gq_status status = GQ_OK;
    double latency = 0.0;
    clk::time_point submitted;
};

struct slot_t {
    gq_ctx *ctx = nullptr;                // its own device status word
    uint32_t *status_host = nullptr;      // pinned copy of that word, per batch
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<pending> items;
    size_t off = 0, bytes = 0;
    gq_status launch_status = GQ_OK;
};

// First-fit allocator over the pool (offsets, 256-byte granules).
struct pool_alloc {
    std::map<size_t, size_t> free_;       // offset -> size
    void init(size_t bytes) { free_ = {{0, bytes & ~size_t(255)}}; }
    bool take(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void give(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct gq_server {
    int device = 0;
    gq_serve_tables tables{};
    char *pool = nullptr;
    size_t pool_bytes = 0;
    int max_batch = 1;
    bool serial = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<pending> queue;
    std::unordered_map<uint64_t, done_state> states;
    std::vector<slot_t> slots;
    pool_alloc alloc;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t n_done = 0, n_batches = 0, max_seen = 0, n_reruns = 0;

    // A shared scan pays for itself only from a few queries of one template
    // on (measured on MI355X over 1.6 billion rows): with fewer queued, the
    // head query runs alone as the plain operator chain.
    static int min_shared(int kind)
    {
        switch (kind) {
        case GQ_QUERY_JOIN_AGG: return 2;
        case GQ_QUERY_FILTER_TOPK: return 9;         // above the top-k batch limit: never shared
        default: return 4;
        }
    }
    bool shared(const gq_serve_query *q, int nq) const { return !serial && nq >= min_shared(q[0].kind); }
    static bool short_kind(int kind) { return kind == GQ_QUERY_FILTER_AGG || kind == GQ_QUERY_FILTER_TOPK; }
    size_t bytes_of(const gq_serve_query *q, int nq) const
    {
        if (shared(q, nq)) return gq_serve_batch_bytes(tables, q, nq);
        size_t b = 0;
        for (int i = 0; i < nq; ++i) b = std::max(b, gq_serve_single_bytes(tables, q[i]));
        return b;
    }
    // Launch a batch on slot sl: its operators, then a copy of the slot's
    // status word to pinned memory and a clear of the word, all on its stream.
    gq_status run(slot_t &sl, const gq_serve_query *q, int nq, void *ws, size_t bytes)
    {
        gq_status st = GQ_OK;
        if (shared(q, nq)) {
            st = gq_serve_batch(sl.ctx, tables, q, nq, ws, bytes, sl.stream);
        } else {
            for (int i = 0; i < nq && st == GQ_OK; ++i)   // (one query, unless the pool cut a shared batch short)
                st = gq_serve_single(sl.ctx, tables, q[i], ws, bytes, sl.stream);
        }
        if (hipMemcpyAsync(sl.status_host, sl.ctx->status_dev, sizeof(uint32_t), hipMemcpyDeviceToHost,
                           sl.stream) != hipSuccess && st == GQ_OK)
            st = GQ_ERR_HIP;
        const gq_status z = gq_zero(sl.ctx, sl.ctx->status_dev, 1, sl.stream);
        return st != GQ_OK ? st : z;
    }
    void retire(slot_t &sl, hipError_t q);
    void loop();
};

// A finished batch: its queries complete, or go back to the head of the
// queue to run again alone (see the error policy at the top of the file).
void gq_server::retire(slot_t &sl, hipError_t q)
{
    gq_status st = sl.launch_status;
    if (st == GQ_OK) st = q == hipSuccess ? gq_status_of_bits(*sl.status_host) : GQ_ERR_HIP;
    std::vector<pending> again;
    const auto now = clk::now();
    for (pending &p : sl.items) {
        gq_retire_case rc{};
        rc.batch_status = st;
        rc.batch_queries = static_cast<int>(sl.items.size());
        rc.aggregate = p.q.kind != GQ_QUERY_FILTER_TOPK;
        rc.max_groups = p.q.max_groups;
        rc.capacity = p.q.out.groups.capacity;
        gq_serve_query doubled = p.q;
        if (st == GQ_ERR_CAPACITY && rc.aggregate) {
            doubled.max_groups = gq_doubled_groups(p.q.max_groups, rc.capacity);
            rc.doubled_fits =
                ((gq_serve_single_bytes(tables, doubled) + 255) & ~size_t(255)) <= (pool_bytes & ~size_t(255));
        }
        const gq_retire_action act = gq_retire_decide(rc);
        if (act != gq_retire_action::complete) {
            if (act == gq_retire_action::rerun_doubled) p.q = doubled;
            p.solo = true;
            again.push_back(p);
            continue;
        }
        done_state &d = states[p.ticket];
        d.done = true;
        d.status = st;
        d.latency = std::chrono::duration<double>(now - d.submitted).count();
        ++n_done;
    }
    for (size_t i = again.size(); i-- > 0;) queue.push_front(again[i]);
    n_reruns += static_cast<int64_t>(again.size());
    alloc.give(sl.off, sl.bytes);
    sl.busy = false;
    sl.items.clear();
    cv_done.notify_all();
}

void gq_server::loop()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        bool progress = false;
        // retire finished batches (a failed batch still retires)
        for (auto &sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            retire(sl, q);
            progress = true;
        }
        // admit and launch
        bool any_busy = false;
        for (auto &sl : slots) any_busy |= sl.busy;
        for (size_t si = 0; si < slots.size(); ++si) {
            slot_t &sl = slots[si];
            if (sl.busy || queue.empty()) continue;
            if (serial && any_busy) break;
            // stream 0 takes the oldest query; the others only short templates,
            // so that long joins never time-share the GPU with each other
            size_t h = 0;
            while (h < queue.size() && si > 0 && !short_kind(queue[h].q.kind)) ++h;
            if (h == queue.size()) continue;
            std::vector<size_t> pick;                     // indices into queue
            const gq_serve_query head = queue[h].q;
            const int limit = (serial || queue[h].solo) ? 1 : max_batch;
            for (size_t i = h; i < queue.size() && static_cast<int>(pick.size()) < limit; ++i) {
                const gq_serve_query &x = queue[i].q;
                if (x.kind == head.kind && !queue[i].solo && (x.kind != GQ_QUERY_FILTER_TOPK || x.k == head.k))
                    pick.push_back(i);
                else if (i == h)
                    pick.push_back(i);                    // a solo head runs by itself
            }
            if (head.kind == GQ_QUERY_FILTER_TOPK && pick.size() > 8) pick.resize(8);
            if (static_cast<int>(pick.size()) < min_shared(head.kind)) pick.resize(1);   // no shared scan: one query
            std::vector<gq_serve_query> qs;
            size_t bytes = 0, off = 0;
            while (!pick.empty()) {                       // largest prefix that fits the free pool
                qs.clear();
                for (size_t i : pick) qs.push_back(queue[i].q);
                bytes = bytes_of(qs.data(), static_cast<int>(qs.size()));
                if (alloc.take(bytes, &off)) break;
                pick.pop_back();
            }
            if (pick.empty()) break;                       // wait for memory to free up
            std::vector<pending> items;
            for (size_t i : pick) items.push_back(queue[i]);
            for (size_t k = pick.size(); k-- > 0;) queue.erase(queue.begin() + static_cast<long>(pick[k]));
            sl.busy = true;
            any_busy = true;
            sl.items = items;
            sl.off = off;
            sl.bytes = bytes;
            ++n_batches;
            if (static_cast<int64_t>(qs.size()) > max_seen) max_seen = static_cast<int64_t>(qs.size());
            lk.unlock();
            gq_status st = run(sl, qs.data(), static_cast<int>(qs.size()), pool + off, bytes);
            if (hipEventRecord(sl.done, sl.stream) != hipSuccess && st == GQ_OK) st = GQ_ERR_HIP;
            lk.lock();
            sl.launch_status = st;
            progress = true;
            if (serial) break;
        }
        bool busy = false;
        for (auto &sl : slots) busy |= sl.busy;
        if (stop && queue.empty() && !busy) break;
        if (!progress) cv_work.wait_for(lk, std::chrono::microseconds(busy ? 20 : 2000));
    }
}

extern "C" {

gq_status gq_server_create(gq_ctx *ctx, const gq_server_cfg *cfg, gq_server **out)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (!cfg || !out) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_server_create: NULL argument");
    *out = nullptr;
    const gq_server_tables &t = cfg->tables;
    if (t.n < 0 || t.n > GQ_MAX_ROWS || (t.n > 0 && (!t.fk || !t.fk2 || !t.date || !t.qty || !t.price || !t.disc)) ||
        !t.dim1_table || !t.dim2_table || !cfg->pool || cfg->pool_bytes < 4096 ||
        reinterpret_cast<uintptr_t>(cfg->pool) % 256 != 0 || cfg->streams < 1 || cfg->streams > 8 ||
        cfg->max_batch < 1 || cfg->max_batch > SV_MAX_BATCH)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_server_create: bad tables, pool or limits");
    gq_server *s = new gq_server();
    s->device = ctx->device;
    auto log2_of = [](size_t bytes) {
        int L = 6;
        while (L < 40 && 256 + (size_t(2) << L) * 16 <= bytes) ++L;
        return L;
    };
    s->tables = {t.fk, t.fk2, t.date, t.qty, t.price, t.disc, t.n, t.dim1_table, t.dim2_table,
                 log2_of(t.dim1_table_bytes), log2_of(t.dim2_table_bytes)};
    s->pool = static_cast<char *>(cfg->pool);
    s->pool_bytes = cfg->pool_bytes;
    s->alloc.init(cfg->pool_bytes);
    s->serial = cfg->serial != 0;
    s->max_batch = s->serial ? 1 : cfg->max_batch;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    s->slots.resize(s->serial ? 1 : cfg->streams);
    gq_status rc = GQ_OK;
    for (auto &sl : s->slots) {
        if (gq_ctx_create(s->device, &sl.ctx) != GQ_OK ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.status_host), sizeof(uint32_t), hipHostMallocDefault) !=
                hipSuccess ||
            hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            rc = GQ_ERR_HIP;
            break;
        }
        *sl.status_host = 0;
    }
    (void)hipSetDevice(prev);
    if (rc != GQ_OK) {
        gq_server_destroy(s);
        return gq_fail(ctx, rc, "gq_server_create: stream, event or context creation failed");
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return GQ_OK;
}

gq_status gq_server_submit(gq_server *srv, const gq_query *q, uint64_t *ticket)
{
    if (!srv || !q || !ticket) return GQ_ERR_INVALID_ARG;
    if (q->kind < GQ_QUERY_FILTER_AGG || q->kind > GQ_QUERY_FILTER_TOPK) return GQ_ERR_INVALID_ARG;
    gq_serve_query x{};
    x.kind = q->kind;
    x.k = q->k;
    x.date_hi = q->date_hi;
    x.max_groups = q->max_groups;
    x.out.groups = q->groups;
    x.out.topk_val = q->topk_val;
    x.out.topk_row = q->topk_row;
    x.out.topk_n = q->topk_n;
    if (x.kind == GQ_QUERY_FILTER_TOPK) {
        if (x.k < 1 || x.k > 256) return GQ_ERR_UNSUPPORTED;
        if (!x.out.topk_val || !x.out.topk_row || !x.out.topk_n) return GQ_ERR_INVALID_ARG;
    } else {
        const gq_groups &g = x.out.groups;
        if (x.max_groups < 1 || x.max_groups > g.capacity || !g.count || !g.sum_qty || !g.sum_rev_lo ||
            !g.sum_rev_hi || !g.avg_qty || !g.avg_rev || !g.n_groups)
            return GQ_ERR_INVALID_ARG;
        if (x.kind == GQ_QUERY_FILTER_AGG && !g.key64) return GQ_ERR_INVALID_ARG;
        if (x.kind != GQ_QUERY_FILTER_AGG && !g.key32) return GQ_ERR_INVALID_ARG;
        if (!srv->serial && x.kind != GQ_QUERY_JOIN_AGG && x.max_groups > SV_MAX_AGG_GROUPS)
            return GQ_ERR_UNSUPPORTED;
    }
    // a query that could never be admitted, even into an idle pool, is refused
    if (((srv->bytes_of(&x, 1) + 255) & ~size_t(255)) > (srv->pool_bytes & ~size_t(255))) return GQ_ERR_CAPACITY;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        *ticket = srv->next_ticket++;
        done_state d;
        d.submitted = clk::now();
        srv->states[*ticket] = d;
        srv->queue.push_back({*ticket, x, d.submitted});
    }
    srv->cv_work.notify_one();
    return GQ_OK;
}

gq_status gq_server_wait(gq_server *srv, uint64_t ticket, gq_status *query_status, double *latency_s)
{
    if (!srv) return GQ_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->states.find(ticket);
    if (it == srv->states.end()) return GQ_ERR_INVALID_ARG;
    srv->cv_done.wait(lk, [&] { return srv->states[ticket].done; });
    const done_state d = srv->states[ticket];
    srv->states.erase(ticket);
    if (query_status) *query_status = d.status;
    if (latency_s) *latency_s = d.latency;
    return GQ_OK;
}

gq_status gq_server_stats(gq_server *srv, int64_t *done, int64_t *batches, int64_t *max_batch_seen,
                          int64_t *reruns)
{
    if (!srv) return GQ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (done) *done = srv->n_done;
    if (batches) *batches = srv->n_batches;
    if (max_batch_seen) *max_batch_seen = srv->max_seen;
    if (reruns) *reruns = srv->n_reruns;
    return GQ_OK;
}

void gq_server_destroy(gq_server *srv)
{
    if (!srv) return;
    if (srv->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv_work.notify_all();
        srv->th.join();
    }
    for (auto &sl : srv->slots) {
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.status_host) (void)hipHostFree(sl.status_host);
        if (sl.ctx) gq_ctx_destroy(sl.ctx);
    }
    delete srv;
}

}  // extern "C"
