// serve.hip - continuous batching of count requests (gs_submit, gs_poll,
// gs_cancel): triangle counts, exact weighted triangle sums and
// parity-decomposed 4-clique counts.
//
// Per context, a pool of builder threads and one count thread. A submitted
// catalogue waits in a FIFO queue. A free builder (each has its own stream
// and scratch, so builds run concurrently) takes the queue head while a
// batch slot is free, runs the first build phase (cells, relabelling, degree
// pass: O(n) memory, after which the exact CSR size is known), waits until
// that footprint fits the context budget next to the graphs already held
// (or nothing else is held), and finishes the build. The count thread takes
// every graph built so far: the plain triangle counts of one bin count go
// into one batched launch, and each weighted triangle count and each parity
// count runs as a count of its own (one such count already fills the
// device); it hands each request its results, frees its graph, and starts
// the next step over whatever was built meanwhile.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "common.h"

namespace gsn {

using Clock = std::chrono::steady_clock;

namespace {

enum ReqState { kQueued, kBuilding, kBuilt, kCounting, kDone, kFailed, kCancelled };

struct Request {
    uint64_t ticket = 0;
    std::vector<double> xyz;
    std::vector<double> w;        // weights (weighted triangle counts)
    int64_t n = 0;
    gs_graph_params p{};
    int kind = GS_3PCF;
    ReqState state = kQueued;
    bool cancel = false;
    int error = 0;
    std::vector<uint64_t> hist;   // triangle counts, or the even channel
    std::vector<uint64_t> pos, neg, wsum;
    int wscale = 0;
    uint64_t ntri = 0;            // triangles or 4-cliques
    uint32_t step_size = 0;
    Clock::time_point t_submit, t_build0, t_build1, t_count0, t_done;
    std::unique_ptr<gs_graph> g;
    std::unique_ptr<BuildJob> job;
    uint64_t footprint = 0;
};

double secs(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
}

}  // namespace

struct Server {
    std::vector<std::unique_ptr<Ctx>> bctx;   // one per builder: own stream, scratch and events
    Ctx cctx;                                  // count step planning (tuned schedules)
    hipStream_t cstream = nullptr;
    std::vector<std::thread> builders;
    std::thread counter;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Request *> queue;                        // submitted, not yet taken by a builder
    std::vector<Request *> ready;                       // built, waiting for a count step
    int building = 0, counting = 0;                     // requests in those states
    std::map<uint64_t, std::unique_ptr<Request>> all;   // live tickets
    uint64_t budget = 0, used = 0;
    int max_slots = 64;
    size_t max_queue = 1 << 16;
};

namespace {

void fail_request(Server &S, Request *r, int code) {
    std::lock_guard<std::mutex> lk(S.mu);
    r->state = kFailed;
    r->error = code;
    r->t_done = Clock::now();
    r->g.reset();
    r->job.reset();
}

void builder(Server *Sp, int k) {
    Server &S = *Sp;
    Ctx &B = *S.bctx[k];
    (void)hipSetDevice(B.device);
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] {
                return S.stop || (!S.queue.empty() &&
                                  (int)S.ready.size() + S.building + S.counting < S.max_slots);
            });
            if (S.stop) return;
            r = S.queue.front();
            S.queue.pop_front();
            if (r->cancel) {
                r->state = kCancelled;
                r->t_done = Clock::now();
                continue;
            }
            r->state = kBuilding;
            r->t_build0 = Clock::now();
            ++S.building;
        }
        bool reserved = false;
        try {
            r->g.reset(new gs_graph());
            Graph &g = *r->g;
            g.device = B.device;
            g.n = r->n;
            g.box = r->p.box;
            g.rmin = r->p.rmin;
            g.rmax = r->p.rmax;
            g.nbins = r->p.nbins;
            g.flags = (r->w.empty() ? 0u : GS_WEIGHTED) | (r->kind == GS_4PCF_PARITY ? GS_KEEP_COORDS : 0u) |
                      (r->p.flags & GS_NONPERIODIC);
            g.periodic = !(r->p.flags & GS_NONPERIODIC);
            g.bins = make_bins(r->p.rmin, r->p.rmax, r->p.nbins);
            r->job.reset(new BuildJob());
            build_begin(B, g, r->xyz.data(), r->w.empty() ? nullptr : r->w.data(), *r->job);
            const uint64_t fp = build_footprint(g, *r->job);
            {
                // admission: the exact footprint fits next to the held graphs,
                // or nothing else is held
                std::unique_lock<std::mutex> lk(S.mu);
                S.cv.wait(lk, [&] { return S.stop || S.used + fp <= S.budget || S.used == 0; });
                if (S.stop) {
                    --S.building;
                    return;
                }
                S.used += fp;
                r->footprint = fp;
                reserved = true;
            }
            build_end(B, g, *r->job, false);
            r->job.reset();
            {
                std::lock_guard<std::mutex> lk(S.mu);
                --S.building;
                r->t_build1 = Clock::now();
                r->xyz.clear();
                r->xyz.shrink_to_fit();
                r->w.clear();
                r->w.shrink_to_fit();
                if (r->cancel) {
                    r->state = kCancelled;
                    r->t_done = r->t_build1;
                    S.used -= r->footprint;
                    r->g.reset();
                } else {
                    r->state = kBuilt;
                    S.ready.push_back(r);
                }
            }
        } catch (const Error &e) {
            {
                std::lock_guard<std::mutex> lk(S.mu);
                --S.building;
                if (reserved) S.used -= r->footprint;
            }
            fail_request(S, r, e.code);
        } catch (...) {
            {
                std::lock_guard<std::mutex> lk(S.mu);
                --S.building;
                if (reserved) S.used -= r->footprint;
            }
            fail_request(S, r, GS_ENOMEM);
        }
        S.cv.notify_all();
    }
}

// A plain (unweighted) triangle count: the kind that batched launches take.
bool batchable(const Request *q) { return q->kind == GS_3PCF && !(q->g->flags & GS_WEIGHTED); }

void count_loop(Server *Sp) {
    Server &S = *Sp;
    (void)hipSetDevice(S.cctx.device);
    // one batch object for every step: its device and pinned buffers are
    // reused (a step starts after the previous one has completed), so no
    // step pays for a free that would wait for the builders' kernels
    std::unique_ptr<Batch3> b(new Batch3());
    while (true) {
        std::vector<Request *> step;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.stop || !S.ready.empty(); });
            if (S.stop) return;
            // one step takes the plain triangle counts that share the first
            // one's bin count (one histogram layout per launch) and every
            // weighted or parity count; other plain counts wait
            int nb = -1;
            for (Request *q : S.ready)
                if (batchable(q)) { nb = q->p.nbins; break; }
            std::vector<Request *> rest;
            for (Request *q : S.ready) (!batchable(q) || q->p.nbins == nb ? step : rest).push_back(q);
            S.ready.swap(rest);
            S.counting = (int)step.size();
            const Clock::time_point now = Clock::now();
            for (Request *q : step) {
                q->state = kCounting;
                q->t_count0 = now;
                q->step_size = (uint32_t)step.size();
            }
        }
        std::vector<Request *> plain;
        std::vector<const Graph *> gs;
        for (Request *q : step)
            if (batchable(q)) {
                plain.push_back(q);
                gs.push_back(q->g.get());
            }
        int err = GS_OK;
        if (!plain.empty()) {
            try {
                count3_batch_enqueue(S.cctx, S.cstream, gs.data(), (int)gs.size(), *b);
                GS_HIP(hipEventSynchronize(b->done));
                if (b->error()) err = GS_EUNSUPPORTED;
            } catch (const Error &e) {
                (void)hipStreamSynchronize(S.cstream);
                err = e.code;
            }
        }
        // weighted and parity counts, one at a time, results into the request
        std::vector<int> own_err(step.size(), GS_OK);
        for (size_t k = 0; k < step.size(); ++k) {
            Request *r = step[k];
            if (batchable(r) || r->cancel) continue;
            try {
                const int64_t nconf = n_configs(r->p.nbins);
                const Graph &g = *r->g;
                r->hist.assign(nconf, 0);
                if (r->kind == GS_4PCF_PARITY) {
                    r->pos.assign(nconf, 0);
                    r->neg.assign(nconf, 0);
                    Count4Out o;
                    o.kind = kParity4;
                    o.cnt[0] = r->pos.data();
                    o.cnt[1] = r->neg.data();
                    o.cnt[2] = r->hist.data();
                    o.ncl = &r->ntri;
                    count4_run(S.cctx, g, o, nullptr);
                    for (int64_t c = 0; c < nconf; ++c) r->hist[c] += r->pos[c] + r->neg[c];
                } else {
                    r->wsum.assign(2 * nconf, 0);
                    r->wscale = weight_scale(g, 3);
                    count3_run(S.cctx, g, r->hist.data(), r->wsum.data(), &r->ntri, nullptr);
                }
            } catch (const Error &e) {
                (void)hipStreamSynchronize(S.cstream);
                own_err[k] = e.code;
            }
        }
        {
            std::lock_guard<std::mutex> lk(S.mu);
            const unsigned long long *o = err == GS_OK && !plain.empty() ? b->out.as<unsigned long long>() : nullptr;
            const size_t per = (size_t)b->nconf + 1;
            const Clock::time_point now = Clock::now();
            size_t slot = 0;
            for (size_t k = 0; k < step.size(); ++k) {
                Request *r = step[k];
                const bool in_batch = batchable(r);
                const int e = in_batch ? err : own_err[k];
                if (r->cancel) {
                    r->state = kCancelled;
                } else if (e != GS_OK) {
                    r->state = kFailed;
                    r->error = e;
                } else {
                    if (in_batch) {
                        r->hist.assign(o + slot * per, o + slot * per + b->nconf);
                        r->ntri = o[slot * per + b->nconf];
                    }
                    r->state = kDone;
                }
                if (in_batch) ++slot;
                r->t_done = now;
                S.used -= r->footprint;
                r->g.reset();
            }
            S.counting = 0;
        }
        S.cv.notify_all();
    }
}

// A builder's context: device properties and tuned schedules of the parent,
// its own streams and events.
Ctx *builder_ctx(const Ctx &ctx, int n_builders) {
    std::unique_ptr<Ctx> b(new Ctx());
    b->device = ctx.device;
    b->n_cu = ctx.n_cu;
    b->max_lds = ctx.max_lds;
    b->budget = ~0ull;  // serving admits by footprint itself; graphs stay resident
    b->tuned = ctx.tuned;
    // a cache of its own: its build temporaries are handed back before its
    // stream has finished with them, so no other stream may take them
    b->pool = std::make_shared<DevPool>();
    b->pool->device = ctx.device;
    b->pool->cap = (ctx.pool ? ctx.pool->cap : 0) / std::max(1, n_builders);
    GS_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->own_stream = true;
    GS_HIP(hipStreamCreateWithFlags(&b->copy_stream, hipStreamNonBlocking));
    for (auto &e : b->ev) GS_HIP(hipEventCreate(&e));
    return b.release();
}

void release_ctx(Ctx &b) {
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    for (auto &e : b.ev)
        if (e) (void)hipEventDestroy(e);
    if (b.copy_stream) (void)hipStreamDestroy(b.copy_stream);
    if (b.own_stream && b.stream) (void)hipStreamDestroy(b.stream);
    if (b.pinned) (void)hipHostFree(b.pinned);
    b.pinned = nullptr;
}

Server &server_of(Ctx &ctx) {
    if (!ctx.server) {
        std::unique_ptr<Server> S(new Server());
        int nb = 4;
        if (const char *eb = getenv("GS_BUILDERS")) nb = std::max(1, std::min(16, atoi(eb)));
        for (int k = 0; k < nb; ++k) S->bctx.emplace_back(builder_ctx(ctx, nb));
        Ctx &c = S->cctx;
        c.device = ctx.device;
        c.n_cu = ctx.n_cu;
        c.max_lds = ctx.max_lds;
        c.budget = ~0ull;
        c.tuned = ctx.tuned;  // schedules tuned in the context before its first request
        GS_HIP(hipStreamCreateWithFlags(&S->cstream, hipStreamNonBlocking));
        // weighted and parity counts run through the lone-count paths on
        // the count stream, with the count context's events and scratch
        c.stream = S->cstream;
        for (auto &e : c.ev) GS_HIP(hipEventCreate(&e));
        S->budget = ctx.budget;
        if (const char *ms = getenv("GS_MAX_SLOTS")) S->max_slots = std::max(1, atoi(ms));
        for (int k = 0; k < nb; ++k) S->builders.emplace_back(builder, S.get(), k);
        S->counter = std::thread(count_loop, S.get());
        ctx.server = S.release();
    }
    return *ctx.server;
}

}  // namespace

void server_stop(Ctx &ctx) {
    Server *S = ctx.server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto &t : S->builders)
        if (t.joinable()) t.join();
    if (S->counter.joinable()) S->counter.join();
    S->all.clear();
    (void)hipStreamSynchronize(S->cstream);
    for (auto &e : S->cctx.ev)
        if (e) (void)hipEventDestroy(e);
    S->cctx.stream = nullptr;
    S->cctx.scratch.reset();
    (void)hipStreamDestroy(S->cstream);
    for (auto &b : S->bctx) release_ctx(*b);
    delete S;
    ctx.server = nullptr;
}

}  // namespace gsn

using namespace gsn;

extern "C" {

int gs_submit(gs_ctx *ctx, const gs_request *req, uint64_t *ticket) {
    return guarded([&] {
        if (!ctx || !req || !ticket) fail(GS_EINVAL, "null argument");
        const gs_graph_params &p = req->p;
        if (req->n < 0 || (req->n > 0 && !req->xyz)) fail(GS_EINVAL, "bad catalogue");
        if (req->n >= 0xFFFFFFFFll) fail(GS_EOVERFLOW, "n must be below 2^32 - 1");
        if (req->kind != GS_3PCF && req->kind != GS_4PCF_PARITY) fail(GS_EINVAL, "unknown request kind");
        if (p.flags & GS_INPUT_ON_DEVICE) fail(GS_EUNSUPPORTED, "served requests take host input");
        if (p.flags & ~(GS_WEIGHTED | GS_KEEP_COORDS | GS_NONPERIODIC)) fail(GS_EINVAL, "unknown flags");
        const bool weighted = (p.flags & GS_WEIGHTED) != 0;
        if (weighted != (req->weights != nullptr)) fail(GS_EINVAL, "weights given iff GS_WEIGHTED");
        if (weighted && req->kind != GS_3PCF) fail(GS_EINVAL, "weights apply to triangle counts only");
        if (!(p.box > 0) || !std::isfinite(p.box)) fail(GS_EINVAL, "box must be finite and > 0");
        if (p.nbins < 1 || p.nbins > 255) fail(GS_EINVAL, "nbins must be in 1..255");
        const bool periodic = !(p.flags & GS_NONPERIODIC);
        if (!(p.rmin >= 0) || !(p.rmin < p.rmax) || !std::isfinite(p.rmax) || (periodic && !(p.rmax < 0.5 * p.box)))
            fail(GS_EINVAL, periodic ? "need 0 <= rmin < rmax < box/2" : "need 0 <= rmin < rmax, finite");
        ctx->use();
        Server &S = server_of(*ctx);
        std::unique_ptr<Request> r(new Request());
        r->xyz.assign(req->xyz, req->xyz + 3 * req->n);
        if (weighted) r->w.assign(req->weights, req->weights + req->n);
        r->n = req->n;
        r->p = p;
        r->kind = req->kind;
        r->t_submit = Clock::now();
        {
            std::lock_guard<std::mutex> lk(S.mu);
            if (S.queue.size() >= S.max_queue) fail(GS_EAGAIN, "submit queue full");
            r->ticket = S.next_ticket++;
            *ticket = r->ticket;
            S.queue.push_back(r.get());
            S.all[r->ticket] = std::move(r);
        }
        S.cv.notify_all();
    });
}

int gs_poll(gs_ctx *ctx, uint64_t ticket, gs_result *out) {
    return guarded([&] {
        if (!ctx || !out) fail(GS_EINVAL, "null argument");
        if (!ctx->server) fail(GS_ENOTFOUND, "no such ticket");
        Server &S = *ctx->server;
        std::lock_guard<std::mutex> lk(S.mu);
        auto it = S.all.find(ticket);
        if (it == S.all.end()) fail(GS_ENOTFOUND, "no such ticket");
        Request &r = *it->second;
        if (r.state == kQueued || r.state == kBuilding || r.state == kBuilt || r.state == kCounting) {
            out->status = GS_PENDING;
            return;
        }
        out->status = r.state == kDone ? GS_DONE : (r.state == kFailed ? GS_FAILED : GS_CANCELLED);
        out->error = r.error;
        out->n_tuples = r.ntri;
        out->wscale = r.wscale;
        if (r.state == kDone) {
            if (out->hist) memcpy(out->hist, r.hist.data(), sizeof(uint64_t) * r.hist.size());
            if (out->pos && !r.pos.empty()) memcpy(out->pos, r.pos.data(), sizeof(uint64_t) * r.pos.size());
            if (out->neg && !r.neg.empty()) memcpy(out->neg, r.neg.data(), sizeof(uint64_t) * r.neg.size());
            if (out->wsum128 && !r.wsum.empty())
                memcpy(out->wsum128, r.wsum.data(), sizeof(uint64_t) * r.wsum.size());
            if (out->whist && !r.wsum.empty())
                for (size_t c = 0; c < r.wsum.size() / 2; ++c) out->whist[c] = sum128_to_double(&r.wsum[2 * c], r.wscale);
        }
        const bool built = r.t_build1 != Clock::time_point{};
        out->t_queue_s = r.t_build0 != Clock::time_point{} ? secs(r.t_submit, r.t_build0) : secs(r.t_submit, r.t_done);
        out->t_build_s = built ? secs(r.t_build0, r.t_build1) : 0.0;
        out->t_count_s = r.t_count0 != Clock::time_point{} ? secs(r.t_count0, r.t_done) : 0.0;
        out->t_total_s = secs(r.t_submit, r.t_done);
        out->step_size = r.step_size;
        S.all.erase(it);
    });
}

int gs_cancel(gs_ctx *ctx, uint64_t ticket) {
    return guarded([&] {
        if (!ctx) fail(GS_EINVAL, "null argument");
        if (!ctx->server) fail(GS_ENOTFOUND, "no such ticket");
        Server &S = *ctx->server;
        std::lock_guard<std::mutex> lk(S.mu);
        auto it = S.all.find(ticket);
        if (it == S.all.end()) fail(GS_ENOTFOUND, "no such ticket");
        it->second->cancel = true;
    });
}

}  // extern "C"
