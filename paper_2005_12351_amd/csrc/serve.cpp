// Continuous-batching request server of libfmm.so.
//
// Requests (positions, moments, order, p, theta, ncrit, method, precision)
// queue in arrival order.  A request is admitted when a worker slot is free
// and its estimated device footprint fits in the context budget next to the
// requests already running; a request that can never fit is rejected at
// submission.  Every slot owns a sub-context (own HIP streams) on the same
// device and runs tree build, upward pass and evaluation of one request at a
// time, so the host work of several requests proceeds in parallel threads and
// their kernels overlap on the GPU.  A request's memory is released as soon as
// it completes.  A context created without a device (fmm_ctx_create_fake)
// runs the same scheduler with an executor that only waits a simulated time,
// for tests of the admission logic.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "fmm_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    fmm_request r{};
    size_t footprint = 0;
    int state = FMM_REQ_QUEUED;
    int status = FMM_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double t_built = 0, t_computed = 0;   // tree and lists ready; results ready
    int64_t bytes_used = 0;
};

}  // namespace

struct Server {
    fmm_ctx *ctx = nullptr;
    bool fake = false;
    double fake_ns_per_particle = 0.0;
    size_t budget = 0, in_use = 0, peak_in_use = 0;
    int nslots = 0, running = 0, peak_running = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<std::thread> workers;
    std::vector<fmm_ctx *> sub;
    bool stopping = false;
    uint64_t next_id = 1;
    Clock::time_point origin;

    double now() const { return std::chrono::duration<double>(Clock::now() - origin).count(); }
};

// Estimated device bytes of one request (tree, expansions, lists, near-field
// buffers): particles cost ~112 B plus the sorted moments, cells (about
// 2.3 n / ncrit) cost their multipole and local rows, the interaction-list
// tiles and partial results (~2 kB) and their M2L list (~1 kB), plus a fixed
// 4 MB for derivative tables.
static size_t footprint_estimate(const fmm_request &r)
{
    const int mask = code_mask(r.order), s = mask_min_order(mask);
    const double w = mask_width(mask);
    const double cells = std::max(1.0, 2.3 * (double)r.n / std::max(1, r.ncrit));
    const double nm = nterms(r.p) - nterms(s - 1), nl = nterms(std::max(0, r.p - s));
    const double per_part = 112.0 + 8.0 * w;
    const double per_cell = 48.0 + nm * 12.0 + nl * 24.0 + 3072.0;
    return (size_t)(per_part * (double)r.n + per_cell * cells + 4.0 * (1 << 20));
}

static int run_real(Server *S, fmm_ctx *c, Req &q)
{
    const fmm_request &r = q.r;
    fmm_tree *t = nullptr;
    int rc = fmm_build_tree(c, r.pos, r.n, r.ncrit, r.theta, r.method, &t);
    q.t_built = S->now();
    if (rc == FMM_OK) rc = fmm_upward(c, t, r.order, r.moments, r.p, r.precision);
    if (rc == FMM_OK) rc = fmm_evaluate(c, t, r.outputs, r.phi, r.field);
    if (rc == FMM_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = FMM_EDEVICE;
    q.t_computed = S->now();
    if (t) {
        q.bytes_used = (int64_t)t->dev_bytes;
        fmm_tree_destroy(t);
    }
    return rc;
}

static void worker_main(Server *S, int slot)
{
    for (;;) {
        uint64_t id = 0;
        Req *q = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                if (S->stopping && S->queue.empty()) return true;
                if (S->queue.empty()) return false;
                const Req &f = S->reqs[S->queue.front()];
                return S->in_use + f.footprint <= S->budget;   // strict arrival order
            });
            if (S->queue.empty()) return;   // stopping
            id = S->queue.front();
            S->queue.pop_front();
            q = &S->reqs[id];
            q->state = FMM_REQ_RUNNING;
            q->t_admit = S->now();
            S->in_use += q->footprint;
            S->peak_in_use = std::max(S->peak_in_use, S->in_use);
            S->running += 1;
            S->peak_running = std::max(S->peak_running, S->running);
        }
        int rc;
        if (S->fake) {
            const double ns = S->fake_ns_per_particle * (double)q->r.n;
            std::this_thread::sleep_for(std::chrono::nanoseconds((int64_t)ns));
            q->bytes_used = (int64_t)q->footprint;
            rc = FMM_OK;
        } else {
            rc = run_real(S, S->sub[slot], *q);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            q->status = rc;
            q->state = rc == FMM_OK ? FMM_REQ_DONE : FMM_REQ_FAILED;
            q->t_done = S->now();
            S->in_use -= q->footprint;
            S->running -= 1;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

int serve_destroy(fmm_ctx *ctx)
{
    Server *S = ctx ? ctx->server : nullptr;
    if (!S) return FMM_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto &th : S->workers) th.join();
    for (fmm_ctx *c : S->sub) fmm_ctx_destroy(c);
    delete S;
    ctx->server = nullptr;
    return FMM_OK;
}

extern "C" int fmm_ctx_create_fake(size_t budget_bytes, double ns_per_particle, fmm_ctx **out)
{
    if (!out || budget_bytes == 0 || !(ns_per_particle >= 0.0)) {
        set_error("fake context needs a budget and a non-negative simulated cost");
        return FMM_EINVAL;
    }
    fmm_ctx *c = new fmm_ctx();
    c->device = -1;
    c->fake = true;
    c->budget = budget_bytes;
    c->fake_ns = ns_per_particle;
    *out = c;
    return FMM_OK;
}

extern "C" int fmm_serve_start(fmm_ctx *ctx, int max_concurrent)
{
    if (!ctx) {
        set_error("null context");
        return FMM_EINVAL;
    }
    if (ctx->server) {
        set_error("server already running");
        return FMM_ESTATE;
    }
    if (max_concurrent < 1 || max_concurrent > 64) {
        set_error("max_concurrent = %d must lie in [1, 64]", max_concurrent);
        return FMM_EINVAL;
    }
    Server *S = new Server();
    S->ctx = ctx;
    S->fake = ctx->fake;
    S->fake_ns_per_particle = ctx->fake_ns;
    S->budget = ctx->budget;
    S->nslots = max_concurrent;
    S->origin = Clock::now();
    if (!S->fake) {
        for (int k = 0; k < max_concurrent; ++k) {
            fmm_ctx *c = nullptr;
            int rc = fmm_ctx_create(ctx->device, nullptr, ctx->budget, &c);
            if (rc != FMM_OK) {
                for (fmm_ctx *d : S->sub) fmm_ctx_destroy(d);
                delete S;
                return rc;
            }
            c->graphs = false;   // one-shot trees: capturing would not pay off
            // the slot's build arena sized before the first request (a build
            // of 2·10^5 particles needs about 40-60 MB); a larger one grows it
            (void)ctx_arena_reserve(c, (size_t)64 << 20);
            S->sub.push_back(c);
        }
    }
    ctx->server = S;
    for (int k = 0; k < max_concurrent; ++k) S->workers.emplace_back(worker_main, S, k);
    return FMM_OK;
}

extern "C" int fmm_serve_stop(fmm_ctx *ctx)
{
    if (!ctx) {
        set_error("null context");
        return FMM_EINVAL;
    }
    return serve_destroy(ctx);
}

extern "C" int fmm_submit(fmm_ctx *ctx, const fmm_request *req, uint64_t *ticket)
{
    if (!ctx || !req || !ticket) {
        set_error("null argument");
        return FMM_EINVAL;
    }
    Server *S = ctx->server;
    if (!S) {
        set_error("server not started");
        return FMM_ESTATE;
    }
    const fmm_request &r = *req;
    const bool code_ok = (r.order >= 0 && r.order <= 3) || (r.order > FMM_MIXED && r.order < FMM_MIXED + 16);
    const int s = code_ok ? mask_min_order(code_mask(r.order)) : 0;
    const int pmin = r.method == FMM_METHOD_BH ? std::max(s, 1) : s + 1;
    if (r.n < 1 || !code_ok || r.p < pmin || r.p > FMM_P_MAX || r.ncrit < 1 ||
        !(r.theta > 0.0 && r.theta < 1.0) || (r.method != FMM_METHOD_FMM && r.method != FMM_METHOD_BH) ||
        (r.precision != FMM_PREC_FP64 && r.precision != FMM_PREC_MIXED) || r.outputs <= 0 ||
        (r.outputs & ~(FMM_POT | FMM_FIELD))) {
        set_error("invalid request parameters");
        return FMM_EINVAL;
    }
    if (!S->fake && (!r.pos || !r.moments || ((r.outputs & FMM_POT) && !r.phi) || ((r.outputs & FMM_FIELD) && !r.field))) {
        set_error("request buffers missing");
        return FMM_EINVAL;
    }
    Req q;
    q.r = r;
    q.footprint = footprint_estimate(r);
    if (q.footprint > S->budget) {
        set_error("request needs about %zu bytes, more than the whole budget of %zu", q.footprint, S->budget);
        return FMM_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) {
            set_error("server stopping");
            return FMM_ESTATE;
        }
        q.t_submit = S->now();
        const uint64_t id = S->next_id++;
        S->reqs.emplace(id, q);
        S->queue.push_back(id);
        *ticket = id;
    }
    S->cv_work.notify_all();
    return FMM_OK;
}

extern "C" int fmm_poll(fmm_ctx *ctx, uint64_t ticket, int *state)
{
    if (!ctx || !ctx->server || !state) {
        set_error("server not started or null argument");
        return FMM_ESTATE;
    }
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket");
        return FMM_EINVAL;
    }
    *state = it->second.state;
    return FMM_OK;
}

extern "C" int fmm_wait(fmm_ctx *ctx, uint64_t ticket, double timeout_s)
{
    if (!ctx || !ctx->server) {
        set_error("server not started");
        return FMM_ESTATE;
    }
    Server *S = ctx->server;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket");
        return FMM_EINVAL;
    }
    auto done = [&] { return it->second.state == FMM_REQ_DONE || it->second.state == FMM_REQ_FAILED; };
    if (timeout_s < 0) {
        S->cv_done.wait(lk, done);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        set_error("request %llu not finished after %g s", (unsigned long long)ticket, timeout_s);
        return FMM_ETIMEOUT;
    }
    if (it->second.state == FMM_REQ_FAILED) {
        set_error("request %llu failed with code %d", (unsigned long long)ticket, it->second.status);
        return it->second.status;
    }
    return FMM_OK;
}

extern "C" int fmm_request_times(fmm_ctx *ctx, uint64_t ticket, double *t, int64_t *bytes)
{
    if (!ctx || !ctx->server) {
        set_error("server not started");
        return FMM_ESTATE;
    }
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket");
        return FMM_EINVAL;
    }
    if (t) {
        t[0] = it->second.t_submit;
        t[1] = it->second.t_admit;
        t[2] = it->second.t_done;
    }
    if (bytes) {
        bytes[0] = (int64_t)it->second.footprint;
        bytes[1] = it->second.bytes_used;
    }
    return FMM_OK;
}

extern "C" int fmm_request_phases(fmm_ctx *ctx, uint64_t ticket, double *t)
{
    if (!ctx || !ctx->server) {
        set_error("server not started");
        return FMM_ESTATE;
    }
    if (!t) {
        set_error("null output");
        return FMM_EINVAL;
    }
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("unknown ticket");
        return FMM_EINVAL;
    }
    t[0] = it->second.t_built;
    t[1] = it->second.t_computed;
    return FMM_OK;
}

extern "C" int fmm_serve_stats(fmm_ctx *ctx, int64_t *stats)
{
    if (!ctx || !ctx->server || !stats) {
        set_error("server not started or null argument");
        return FMM_ESTATE;
    }
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    stats[0] = (int64_t)S->budget;
    stats[1] = (int64_t)S->in_use;
    stats[2] = (int64_t)S->peak_in_use;
    stats[3] = S->running;
    stats[4] = S->peak_running;
    stats[5] = (int64_t)S->queue.size();
    stats[6] = S->nslots;
    return FMM_OK;
}
