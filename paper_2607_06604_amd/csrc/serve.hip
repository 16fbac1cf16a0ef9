// serve.hip - continuous batching of triangle-count requests (gs_submit,
// gs_poll, gs_cancel).
//
// One scheduler thread per context. A submitted catalogue waits in a FIFO
// queue; the scheduler runs the first build phase of the queue head (cells,
// relabelling, degree pass: O(n) memory, after which the exact CSR size is
// known), admits it when that footprint fits the context budget next to the
// graphs already held and a batch slot is free, and finishes its build. Built
// graphs wait for the next count step: one batched launch over every built
// graph. Builds run on the build stream while a step runs on the count
// stream, so requests arriving during a step are built in the meantime and
// join the next one. A finished step hands each request its histogram and
// frees its graph.
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

enum ReqState { kQueued, kBuilt, kCounting, kDone, kFailed, kCancelled };

struct Request {
    uint64_t ticket = 0;
    std::vector<double> xyz;
    int64_t n = 0;
    gs_graph_params p{};
    ReqState state = kQueued;
    bool cancel = false;
    int error = 0;
    std::vector<uint64_t> hist;
    uint64_t ntri = 0;
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
    Ctx bctx;                  // build context: own stream, scratch and events
    hipStream_t cstream = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Request *> queue;                        // submitted, not yet built
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

void run(Server *Sp) {
    Server &S = *Sp;
    (void)hipSetDevice(S.bctx.device);
    std::vector<Request *> ready, step;
    std::unique_ptr<Batch3> inflight;
    while (true) {
        bool progress = false;
        // 1. a finished step hands out its results
        if (inflight && hipEventQuery(inflight->done) == hipSuccess) {
            const unsigned long long *o = inflight->out.as<unsigned long long>();
            const size_t per = (size_t)inflight->nconf + 1;
            const bool bad = inflight->error() != 0;
            std::lock_guard<std::mutex> lk(S.mu);
            const Clock::time_point now = Clock::now();
            for (size_t k = 0; k < step.size(); ++k) {
                Request *r = step[k];
                if (r->cancel) {
                    r->state = kCancelled;
                } else if (bad) {
                    r->state = kFailed;
                    r->error = GS_EUNSUPPORTED;
                } else {
                    r->hist.assign(o + k * per, o + k * per + inflight->nconf);
                    r->ntri = o[k * per + inflight->nconf];
                    r->state = kDone;
                }
                r->t_done = now;
                S.used -= r->footprint;
                r->g.reset();
            }
            step.clear();
            inflight.reset();
            progress = true;
        }
        // 2. build the queue head if a slot is free and its graph fits
        Request *r = nullptr;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            if (S.stop) break;
            while (!S.queue.empty() && S.queue.front()->cancel) {
                S.queue.front()->state = kCancelled;
                S.queue.front()->t_done = Clock::now();
                S.queue.front()->job.reset();
                S.queue.pop_front();
            }
            if (!S.queue.empty() && (int)(ready.size() + step.size()) < S.max_slots) r = S.queue.front();
        }
        if (r) {
            bool admitted = false;
            try {
                if (!r->job) {
                    r->t_build0 = Clock::now();
                    r->g.reset(new gs_graph());
                    Graph &g = *r->g;
                    g.device = S.bctx.device;
                    g.n = r->n;
                    g.box = r->p.box;
                    g.rmin = r->p.rmin;
                    g.rmax = r->p.rmax;
                    g.nbins = r->p.nbins;
                    g.flags = 0;
                    g.bins = make_bins(r->p.rmin, r->p.rmax, r->p.nbins);
                    r->job.reset(new BuildJob());
                    build_begin(S.bctx, g, r->xyz.data(), nullptr, *r->job);
                    r->footprint = build_footprint(g, *r->job);
                }
                const bool idle = ready.empty() && step.empty();
                if (S.used + r->footprint <= S.budget || idle) {
                    build_end(S.bctx, *r->g, *r->job, false);
                    r->job.reset();
                    r->t_build1 = Clock::now();
                    admitted = true;
                }
            } catch (const Error &e) {
                {
                    std::lock_guard<std::mutex> lk(S.mu);
                    S.queue.pop_front();
                }
                fail_request(S, r, e.code);
                progress = true;
                r = nullptr;
            } catch (...) {
                {
                    std::lock_guard<std::mutex> lk(S.mu);
                    S.queue.pop_front();
                }
                fail_request(S, r, GS_ENOMEM);
                progress = true;
                r = nullptr;
            }
            if (r && admitted) {
                std::lock_guard<std::mutex> lk(S.mu);
                S.queue.pop_front();
                r->state = kBuilt;
                r->xyz.clear();
                r->xyz.shrink_to_fit();
                S.used += r->footprint;
                ready.push_back(r);
                progress = true;
            }
        }
        // 3. no step in flight: count everything built, in one launch
        if (!inflight && !ready.empty()) {
            step.swap(ready);
            std::vector<const Graph *> gs;
            for (Request *q : step) gs.push_back(q->g.get());
            const Clock::time_point now = Clock::now();
            try {
                inflight.reset(new Batch3());
                count3_batch_enqueue(S.bctx, S.cstream, gs.data(), (int)gs.size(), *inflight);
                std::lock_guard<std::mutex> lk(S.mu);
                for (Request *q : step) {
                    q->state = kCounting;
                    q->t_count0 = now;
                    q->step_size = (uint32_t)step.size();
                }
            } catch (const Error &e) {
                (void)hipStreamSynchronize(S.cstream);
                std::lock_guard<std::mutex> lk(S.mu);
                for (Request *q : step) {
                    q->state = kFailed;
                    q->error = e.code;
                    q->t_done = Clock::now();
                    S.used -= q->footprint;
                    q->g.reset();
                }
                step.clear();
                inflight.reset();
            }
            progress = true;
        }
        if (!progress) {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait_for(lk, std::chrono::microseconds(inflight ? 100 : 2000),
                          [&] { return S.stop || (!S.queue.empty() && !inflight); });
        }
    }
    if (inflight) (void)hipEventSynchronize(inflight->done);
    (void)hipStreamSynchronize(S.cstream);
    (void)hipStreamSynchronize(S.bctx.stream);
}

Server &server_of(Ctx &ctx) {
    if (!ctx.server) {
        std::unique_ptr<Server> S(new Server());
        Ctx &b = S->bctx;
        b.device = ctx.device;
        b.n_cu = ctx.n_cu;
        b.max_lds = ctx.max_lds;
        b.budget = ~0ull;  // serving admits by footprint itself; graphs stay resident
        b.tuned = ctx.tuned;  // schedules tuned in the context before its first request
        GS_HIP(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
        b.own_stream = true;
        GS_HIP(hipStreamCreateWithFlags(&b.copy_stream, hipStreamNonBlocking));
        for (auto &e : b.ev) GS_HIP(hipEventCreate(&e));
        GS_HIP(hipStreamCreateWithFlags(&S->cstream, hipStreamNonBlocking));
        S->budget = ctx.budget;
        if (const char *ms = getenv("GS_MAX_SLOTS")) S->max_slots = std::max(1, atoi(ms));
        S->th = std::thread(run, S.get());
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
    if (S->th.joinable()) S->th.join();
    S->all.clear();
    (void)hipStreamDestroy(S->cstream);
    for (auto &e : S->bctx.ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(S->bctx.copy_stream);
    (void)hipStreamDestroy(S->bctx.stream);
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
        if (p.flags != 0) fail(GS_EUNSUPPORTED, "served requests take host, unweighted input");
        if (!(p.box > 0) || !std::isfinite(p.box)) fail(GS_EINVAL, "box must be finite and > 0");
        if (p.nbins < 1 || p.nbins > 255) fail(GS_EINVAL, "nbins must be in 1..255");
        if (!(p.rmin >= 0) || !(p.rmin < p.rmax) || !(p.rmax < 0.5 * p.box))
            fail(GS_EINVAL, "need 0 <= rmin < rmax < box/2");
        ctx->use();
        Server &S = server_of(*ctx);
        std::unique_ptr<Request> r(new Request());
        r->xyz.assign(req->xyz, req->xyz + 3 * req->n);
        r->n = req->n;
        r->p = p;
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
        if (r.state == kQueued || r.state == kBuilt || r.state == kCounting) {
            out->status = GS_PENDING;
            return;
        }
        out->status = r.state == kDone ? GS_DONE : (r.state == kFailed ? GS_FAILED : GS_CANCELLED);
        out->error = r.error;
        out->n_triangles = r.ntri;
        if (r.state == kDone && out->hist) memcpy(out->hist, r.hist.data(), sizeof(uint64_t) * r.hist.size());
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
