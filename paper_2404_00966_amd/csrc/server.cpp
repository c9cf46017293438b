// Serving: continuous batching of range / kNN requests and streamed updates
// over resident indexes (gts_server_* in include/gts.h).
//
// Per index: one scheduler thread and L lane threads.  The scheduler takes
// the index's FIFO in order.  Every update gets the next epoch of the index
// and applies at once, while batches run: a deletion only stamps epochs
// (tombstones and cache slots) and an insertion fills cache slots above
// those the running batches read.  A query request is admitted at the
// index's current epoch and sees exactly the updates submitted before it
// (Sec. 4.4: the index and the cache list, less the marked objects, as of
// its admission).  Queries at the head are admitted together, with the
// updates between them applied in order, up to the batch limit, into one
// mixed gts_search batch handed to a free lane; each lane owns a HIP stream
// and a query workspace (QueryCtx), so batches overlap on the device.  Only
// an update that moves memory the batches read -- a cache list that must
// grow, a rebuild, new bytes in an edit index's alphabet -- waits until no
// batch of the index is in flight.  Answers of a batch are split back into
// per-request host CSR completions.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

#include "gts_internal.h"

namespace gts {
namespace {

// Angular indexes: a query request with a zero vector is refused at submission
// (in a batch it would fail every request admitted with it).  The search scales
// queries to unit length itself.
void check_directions(const gts_index *idx, const HostObjects &h)
{
    if (!idx->angular) return;
    for (int64_t i = 0; i < h.count(); i++) {
        double s = 0.0;
        for (int j = 0; j < h.dim; j++) s += (double)h.vecs[(size_t)i * h.dim + j] * h.vecs[(size_t)i * h.dim + j];
        GTS_CHECK(s > 0.0, GTS_EINVAL, "a zero vector has no direction (angular metric)");
    }
}


double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    gts_request req{};          // scalars (pointers cleared)
    HostObjects objs;           // queries or new objects (host copy)
    std::vector<int64_t> ids;   // DELETE
    double t_submit = 0.0;
};

struct Completion {
    gts_completion pub{};
    std::string error;
    std::vector<int64_t> offsets, ids, new_ids;
    std::vector<float> df;
    std::vector<int32_t> di;
};

struct Lane;

struct IndexQueue {
    gts_index *idx = nullptr;
    std::deque<std::unique_ptr<Request>> fifo;
    std::vector<std::unique_ptr<Lane>> lanes;
    std::thread scheduler;
    int inflight = 0;
};

struct Lane {
    QueryCtx ctx;
    std::thread th;
    std::vector<std::unique_ptr<Request>> batch;
    std::vector<uint32_t> epoch;   // admission epoch of each request of the batch
    int64_t cache_count = 0;       // cache slots filled when the batch was closed
    int64_t batch_no = -1;
    bool has_work = false;
};

bool is_update(const Request &r)
{
    return r.req.kind == GTS_REQ_INSERT || r.req.kind == GTS_REQ_DELETE;
}

// An update that moves or rewrites memory a running batch reads waits for
// the index's batches to finish: an insertion that grows the cache arrays,
// an insertion or deletion that triggers a rebuild, or an insertion that adds
// bytes to an edit index's alphabet (the match tables of running batches use
// the old codes).
bool update_needs_drain(const gts_index *idx, const Request &r)
{
    if (r.req.kind == GTS_REQ_DELETE) {
        // a delete that leaves the tree mostly deleted rebuilds it (counted
        // generously: a repeated id counts twice)
        int64_t more = 0;
        for (int64_t id : r.ids)
            if (id >= 0 && id < (int64_t)idx->pos_of_id.size() && idx->pos_of_id[id] >= 0 &&
                !idx->h_tomb[idx->pos_of_id[id]])
                more++;
        return tree_mostly_deleted(idx, more);
    }
    if (r.req.kind != GTS_REQ_INSERT) return false;
    const int64_t n = r.objs.count();
    const CacheList &c = idx->cache;
    const int64_t limit = idx->opts.cache_limit > 0 ? idx->opts.cache_limit : 4096;
    if (c.count + n > c.cap || c.n_live + n > limit) return true;
    if (idx->data.metric != GTS_L2_F32)
        for (uint8_t ch : r.objs.chars)
            if (!idx->alpha[ch]) return true;
    return false;
}

}  // namespace
}  // namespace gts

struct gts_server {
    gts_server_opts opts{};
    std::vector<std::unique_ptr<gts::IndexQueue>> ix;
    std::mutex mu;
    std::condition_variable cv;          // any state change
    std::deque<gts::Completion *> done;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t next_batch = 0;
    int64_t pending = 0;                 // submitted, not completed
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, queries = 0, batches = 0, updates = 0, batch_queries = 0;
    std::vector<double> lat;             // query request latencies (ms)
    double t_first = -1.0, t_last = 0.0;
};

namespace gts {
namespace {

void finish(gts_server *s, Completion *c, bool query, int64_t nq)
{
    // caller holds s->mu
    s->completed++;
    s->pending--;
    if (c->pub.status != GTS_OK) s->failed++;
    if (query && c->pub.status == GTS_OK) {
        s->lat.push_back(c->pub.t_done_ms - c->pub.t_submit_ms);
        s->queries += nq;
    }
    s->t_last = std::max(s->t_last, c->pub.t_done_ms);
    if (s->opts.keep_results) s->done.push_back(c);
    else delete c;
}

Completion *make_completion(const Request &r, double t_start)
{
    auto *c = new Completion();
    c->pub.ticket = r.ticket;
    c->pub.tag = r.req.tag;
    c->pub.kind = r.req.kind;
    c->pub.status = GTS_OK;
    c->pub.batch = -1;
    c->pub.t_submit_ms = r.t_submit;
    c->pub.t_start_ms = t_start;
    c->pub.priv = c;
    return c;
}

void set_error(Completion *c, gts_status st, const std::string &msg)
{
    c->pub.status = st;
    c->error = msg;
}

void publish(Completion *c)
{
    c->pub.error = c->error.c_str();
    c->pub.result.offsets = c->offsets.empty() ? nullptr : c->offsets.data();
    c->pub.result.ids = c->ids.empty() ? nullptr : c->ids.data();
    c->pub.result.dist_f32 = c->df.empty() ? nullptr : c->df.data();
    c->pub.result.dist_i32 = c->di.empty() ? nullptr : c->di.data();
    c->pub.new_ids = c->new_ids.empty() ? nullptr : c->new_ids.data();
}

// One update, on the scheduler's thread.
void run_update(gts_server *s, IndexQueue &q, std::unique_ptr<Request> r)
{
    const double t0 = now_ms();
    Completion *c = make_completion(*r, t0);
    gts_status st;
    if (r->req.kind == GTS_REQ_INSERT) {
        c->new_ids.resize(r->objs.count());
        st = run_guarded([&] {
            insert_objects(q.idx, r->objs, c->new_ids.data());
            c->pub.count = r->objs.count();
        });
    } else {
        st = run_guarded([&] { c->pub.count = delete_ids(q.idx, r->ids.data(), (int64_t)r->ids.size()); });
    }
    if (st != GTS_OK) set_error(c, st, gts_last_error());
    c->pub.t_done_ms = now_ms();
    publish(c);
    std::lock_guard<std::mutex> g(s->mu);
    s->updates++;
    finish(s, c, false, 0);
    s->cv.notify_all();
}

// One batch of queries on a lane: one mixed search, answers split back.
void run_batch(gts_server *s, IndexQueue &q, Lane &lane)
{
    const double t0 = now_ms();
    const IndexData &d = q.idx->data;
    const bool l2 = d.metric == GTS_L2_F32;
    int64_t nq = 0;
    for (auto &r : lane.batch) nq += r->objs.count();
    std::vector<float> vecs, radius(nq, 0.f);
    std::vector<uint8_t> chars;
    std::vector<int64_t> offs{0};
    std::vector<int32_t> kk(nq, 0);
    if (l2) vecs.reserve((size_t)nq * d.dim);
    int64_t at = 0;
    for (auto &r : lane.batch) {
        const HostObjects &o = r->objs;
        if (l2) {
            vecs.insert(vecs.end(), o.vecs.begin(), o.vecs.end());
        } else {
            chars.insert(chars.end(), o.chars.begin(), o.chars.end());
            for (int64_t i = 0; i < o.count(); i++) offs.push_back(offs.back() + (o.offsets[i + 1] - o.offsets[i]));
        }
        for (int64_t i = 0; i < o.count(); i++, at++) {
            if (r->req.kind == GTS_REQ_KNN) kk[at] = r->req.k;
            else radius[at] = r->req.radius;
        }
    }
    gts_objects Q{};
    Q.n = nq;
    Q.dim = l2 ? d.dim : 0;
    Q.location = GTS_HOST;
    Q.vecs = l2 ? vecs.data() : nullptr;
    Q.chars = l2 ? nullptr : (chars.empty() ? reinterpret_cast<const uint8_t *>("") : chars.data());
    Q.offsets = l2 ? nullptr : offs.data();
    gts_query_opts qo{};
    qo.mode = GTS_MODE_BATCHED;
    qo.result_location = GTS_HOST;
    qo.mem_budget_bytes = s->opts.mem_budget_bytes > 0
                              ? s->opts.mem_budget_bytes
                              : std::max<int64_t>(q.idx->opts.mem_budget_bytes / s->opts.lanes_per_index, 1 << 20);
    // admission epochs per query
    SnapView &v = lane.ctx.view;
    v.on = true;
    v.qep.clear();
    v.qep.reserve(nq);
    v.e_min = 0xffffffffu;
    v.e_max = 0;
    for (size_t i = 0; i < lane.batch.size(); i++) {
        const uint32_t e = lane.epoch[i];
        v.qep.insert(v.qep.end(), (size_t)lane.batch[i]->objs.count(), e);
        v.e_min = std::min(v.e_min, e);
        v.e_max = std::max(v.e_max, e);
    }
    v.cache_count = lane.cache_count;
    gts_result res{};
    const gts_status st = run_guarded([&] { search(q.idx, &lane.ctx, &Q, radius.data(), kk.data(), &qo, &res); });
    const std::string err = st == GTS_OK ? std::string() : std::string(gts_last_error());
    const double t1 = now_ms();
    std::vector<Completion *> out;
    at = 0;
    for (auto &r : lane.batch) {
        Completion *c = make_completion(*r, t0);
        c->pub.batch = lane.batch_no;
        const int64_t n = r->objs.count();
        if (st != GTS_OK) {
            set_error(c, st, err);
        } else {
            const int64_t a = res.offsets[at], b = res.offsets[at + n];
            c->offsets.resize(n + 1);
            for (int64_t i = 0; i <= n; i++) c->offsets[i] = res.offsets[at + i] - a;
            c->ids.assign(res.ids + a, res.ids + b);
            if (l2) c->df.assign(res.dist_f32 + a, res.dist_f32 + b);
            else c->di.assign(res.dist_i32 + a, res.dist_i32 + b);
            c->pub.result.nq = n;
            c->pub.result.total = b - a;
            c->pub.result.location = GTS_HOST;
            c->pub.result.metric = q.idx->angular ? GTS_COSINE_F32 : q.idx->l1 ? GTS_L1_F32 : d.metric;
        }
        c->pub.t_done_ms = t1;
        publish(c);
        out.push_back(c);
        at += n;
    }
    if (st == GTS_OK) free_result(&res);
    std::lock_guard<std::mutex> g(s->mu);
    s->batches++;
    s->batch_queries += nq;
    for (size_t i = 0; i < out.size(); i++) finish(s, out[i], true, lane.batch[i]->objs.count());
    lane.batch.clear();
    lane.epoch.clear();
    lane.has_work = false;
    q.inflight--;
    s->cv.notify_all();
}

void lane_loop(gts_server *s, IndexQueue *q, Lane *lane)
{
    for (;;) {
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv.wait(g, [&] { return lane->has_work || s->stop; });
            if (!lane->has_work) return;
        }
        run_batch(s, *q, *lane);
    }
}

void scheduler_loop(gts_server *s, IndexQueue *q)
{
    const int64_t max_q = s->opts.max_batch_queries;
    for (;;) {
        std::unique_lock<std::mutex> g(s->mu);
        Lane *free_lane = nullptr;
        s->cv.wait(g, [&] {
            if (q->fifo.empty()) return s->stop;
            const Request &h = *q->fifo.front();
            if (is_update(h)) return q->inflight == 0 || !update_needs_drain(q->idx, h);
            free_lane = nullptr;
            for (auto &l : q->lanes)
                if (!l->has_work) {
                    free_lane = l.get();
                    break;
                }
            return free_lane != nullptr;
        });
        if (q->fifo.empty()) return;   // stopping, nothing left
        if (is_update(*q->fifo.front())) {
            std::unique_ptr<Request> r = std::move(q->fifo.front());
            q->fifo.pop_front();
            g.unlock();
            run_update(s, *q, std::move(r));
            continue;
        }
        // queries at the head, each at the epoch of the updates before it;
        // updates between them apply in order unless one must wait for the
        // running batches (then the batch closes before it)
        int64_t nq = 0;
        while (!q->fifo.empty()) {
            Request *r = q->fifo.front().get();
            if (is_update(*r)) {
                if (update_needs_drain(q->idx, *r)) break;
                std::unique_ptr<Request> u = std::move(q->fifo.front());
                q->fifo.pop_front();
                g.unlock();
                run_update(s, *q, std::move(u));
                g.lock();
                continue;
            }
            if (nq > 0 && nq + r->objs.count() > max_q) break;
            nq += r->objs.count();
            free_lane->epoch.push_back(q->idx->epoch);
            free_lane->batch.push_back(std::move(q->fifo.front()));
            q->fifo.pop_front();
        }
        free_lane->cache_count = q->idx->cache.count;
        free_lane->batch_no = s->next_batch++;
        free_lane->has_work = true;
        q->inflight++;
        s->cv.notify_all();
    }
}

}  // namespace
}  // namespace gts

using namespace gts;

extern "C" {

gts_status gts_server_create(gts_index *const *indexes, int32_t n_indexes, const gts_server_opts *opts,
                             gts_server **out)
{
    return run_guarded([&] {
        GTS_CHECK(out != nullptr, GTS_EINVAL, "null output handle");
        GTS_CHECK(indexes != nullptr && n_indexes >= 1, GTS_EINVAL, "a server needs at least one index");
        auto s = std::make_unique<gts_server>();
        if (opts) s->opts = *opts;
        else s->opts.keep_results = 1;
        if (s->opts.lanes_per_index <= 0) s->opts.lanes_per_index = 2;
        GTS_CHECK(s->opts.lanes_per_index <= 8, GTS_EINVAL, "at most 8 lanes per index");
        if (s->opts.max_batch_queries <= 0) s->opts.max_batch_queries = 16384;
        for (int32_t i = 0; i < n_indexes; i++) {
            GTS_CHECK(indexes[i] != nullptr, GTS_EINVAL, "null index in the server's list");
            auto q = std::make_unique<IndexQueue>();
            q->idx = indexes[i];
            for (int l = 0; l < s->opts.lanes_per_index; l++) {
                auto lane = std::make_unique<Lane>();
                GTS_HIP(hipStreamCreateWithFlags(&lane->ctx.stream, hipStreamNonBlocking));
                q->lanes.push_back(std::move(lane));
            }
            s->ix.push_back(std::move(q));
        }
        gts_server *sp = s.get();
        for (auto &q : s->ix) {
            for (auto &l : q->lanes) l->th = std::thread(lane_loop, sp, q.get(), l.get());
            q->scheduler = std::thread(scheduler_loop, sp, q.get());
        }
        *out = s.release();
    });
}

gts_status gts_server_submit(gts_server *s, const gts_request *req, uint64_t *ticket)
{
    return run_guarded([&] {
        GTS_CHECK(s != nullptr && req != nullptr, GTS_EINVAL, "null server or request");
        GTS_CHECK(req->index >= 0 && req->index < (int32_t)s->ix.size(), GTS_EINVAL, "index out of range");
        IndexQueue &q = *s->ix[req->index];
        const IndexData &d = q.idx->data;
        auto r = std::make_unique<Request>();
        r->req = *req;
        r->req.objects = gts_objects{};
        r->req.ids = nullptr;
        switch (req->kind) {
        case GTS_REQ_RANGE:
            GTS_CHECK(std::isfinite(req->radius) && req->radius >= 0.f, GTS_EINVAL, "radius must be finite and >= 0");
            read_objects(&req->objects, d.metric, d.dim, q.idx->opts.max_strlen, &r->objs);
            check_directions(q.idx, r->objs);
            break;
        case GTS_REQ_KNN:
            GTS_CHECK(req->k >= 1, GTS_EINVAL, "k must be >= 1");
            read_objects(&req->objects, d.metric, d.dim, q.idx->opts.max_strlen, &r->objs);
            check_directions(q.idx, r->objs);
            break;
        case GTS_REQ_INSERT:
            read_objects(&req->objects, d.metric, d.dim, q.idx->opts.max_strlen, &r->objs, q.idx->angular);
            break;
        case GTS_REQ_DELETE:
            GTS_CHECK(req->n_ids >= 0 && (req->ids != nullptr || req->n_ids == 0), GTS_EINVAL, "bad delete ids");
            r->ids.assign(req->ids, req->ids + req->n_ids);
            break;
        default:
            fail(GTS_EINVAL, "unknown request kind");
        }
        r->t_submit = now_ms();
        std::lock_guard<std::mutex> g(s->mu);
        GTS_CHECK(!s->stop, GTS_EINVAL, "server is stopping");
        r->ticket = s->next_ticket++;
        if (ticket) *ticket = r->ticket;
        if (s->t_first < 0) s->t_first = r->t_submit;
        s->submitted++;
        s->pending++;
        q.fifo.push_back(std::move(r));
        s->cv.notify_all();
    });
}

gts_status gts_server_replay(gts_server *s, const gts_request *reqs, const double *arrival_ms, int64_t n,
                             uint64_t *tickets)
{
    return run_guarded([&] {
        GTS_CHECK(s != nullptr && (n == 0 || (reqs != nullptr && arrival_ms != nullptr)), GTS_EINVAL,
                  "null replay arrays");
        const auto t0 = std::chrono::steady_clock::now();
        for (int64_t i = 0; i < n; i++) {
            const auto due = t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                      std::chrono::duration<double, std::milli>(arrival_ms[i]));
            std::this_thread::sleep_until(due);
            const gts_status st = gts_server_submit(s, &reqs[i], tickets ? &tickets[i] : nullptr);
            if (st != GTS_OK) fail(st, std::string("request ") + std::to_string(i) + ": " + gts_last_error());
        }
    });
}

gts_status gts_server_poll(gts_server *s, gts_completion *out, int32_t max, int32_t wait_ms, int32_t *n_out)
{
    return run_guarded([&] {
        GTS_CHECK(s != nullptr && n_out != nullptr && (out != nullptr || max == 0), GTS_EINVAL, "null poll argument");
        std::unique_lock<std::mutex> g(s->mu);
        auto ready = [&] { return !s->done.empty() || s->pending == 0; };
        if (wait_ms < 0) s->cv.wait(g, ready);
        else if (wait_ms > 0) s->cv.wait_for(g, std::chrono::milliseconds(wait_ms), ready);
        int32_t n = 0;
        while (n < max && !s->done.empty()) {
            out[n++] = s->done.front()->pub;
            s->done.pop_front();
        }
        *n_out = n;
    });
}

gts_status gts_server_release(gts_completion *c)
{
    return run_guarded([&] {
        if (c && c->priv) {
            delete static_cast<Completion *>(c->priv);
            c->priv = nullptr;
        }
    });
}

gts_status gts_server_flush(gts_server *s)
{
    return run_guarded([&] {
        GTS_CHECK(s != nullptr, GTS_EINVAL, "null server");
        std::unique_lock<std::mutex> g(s->mu);
        s->cv.wait(g, [&] { return s->pending == 0; });
    });
}

gts_status gts_server_get_stats(gts_server *s, gts_server_stats *out)
{
    return run_guarded([&] {
        GTS_CHECK(s != nullptr && out != nullptr, GTS_EINVAL, "null argument");
        std::lock_guard<std::mutex> g(s->mu);
        gts_server_stats r{};
        r.submitted = s->submitted;
        r.completed = s->completed;
        r.failed = s->failed;
        r.queries = s->queries;
        r.batches = s->batches;
        r.updates = s->updates;
        r.mean_batch_queries = s->batches ? (double)s->batch_queries / (double)s->batches : 0.0;
        if (!s->lat.empty()) {
            std::vector<double> v = s->lat;
            auto pct = [&](double p) {
                const size_t i = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
                std::nth_element(v.begin(), v.begin() + i, v.end());
                return v[i];
            };
            r.p50_ms = pct(0.50);
            r.p99_ms = pct(0.99);
            r.max_ms = *std::max_element(v.begin(), v.end());
        }
        r.span_ms = s->t_first >= 0 ? s->t_last - s->t_first : 0.0;
        *out = r;
    });
}

gts_status gts_server_destroy(gts_server *s)
{
    return run_guarded([&] {
        if (!s) return;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv.wait(g, [&] { return s->pending == 0; });
            s->stop = true;
            s->cv.notify_all();
        }
        for (auto &q : s->ix) {
            if (q->scheduler.joinable()) q->scheduler.join();
            for (auto &l : q->lanes)
                if (l->th.joinable()) l->th.join();
        }
        for (auto &q : s->ix)
            for (auto &l : q->lanes)
                if (l->ctx.stream) (void)hipStreamDestroy(l->ctx.stream);
        for (Completion *c : s->done) delete c;
        delete s;
    });
}

}  // extern "C"
