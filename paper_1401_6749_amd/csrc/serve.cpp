// Serving loop: continuous batching of loop requests.
//
// The scheduling state machine (admission by footprint, packing of sources
// that share a gauge field into multi-RHS batches, refill of finished slots
// between chunks, per-request finalization) is in serve_sched.h.  This file
// gives it its HIP device: batches on their own non-blocking streams (so
// batches on different gauge fields overlap on the device), chunk completion
// by event queries, finalization (projection, TSM combination, copy of the
// results into pinned host memory) on a separate stream.  A worker thread
// runs the loop and makes every device call of the serving engine between
// tm_serve_create and tm_serve_destroy; submit, poll, status and drain only
// exchange host data with it under its lock.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "serve_sched.h"
#include "tm_internal.h"

using namespace tmk;
using namespace tmi;

int tsm_check(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P);

namespace {

void *arena_alloc(void *self, size_t n) { return ((tmi::Arena *)self)->alloc(n); }
void arena_free(void *self, void *p) { ((tmi::Arena *)self)->release(p); }

struct HipDev {
    tm_context *ctx = nullptr;
    int slots = 12;
    Mem mem;  // batches are carved from the scheduler's arena
    hipStream_t fin_stream = nullptr;
    std::vector<std::pair<size_t, double *>> pinned;  // free pinned result buffers

    struct Batch {
        tmi::Batch *b = nullptr;
        hipStream_t stream = nullptr;
    };
    struct ReqDev {
        // recorded on a batch stream after each harvest of one of the
        // request's HP / LP sources; the finalization stream waits on both
        hipEvent_t ev_hp = nullptr, ev_lp = nullptr, fin_ev = nullptr;
        double *h_out = nullptr;  // pinned: est, var_re, var_im
        size_t h_bytes = 0;
    };
    using Req = SchedReq<ReqDev>;

    int lt(const tm_gauge *G) const { return G->dims[3]; }
    size_t batch_bytes(const tm_gauge *G, Kind k) const { return batch_footprint(G, k, slots) + 32 * 256; }

    Batch *batch_create(const tm_gauge *G, Kind k, int chunk, int &rc)
    {
        Batch *B = new Batch();
        if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
            delete B;
            rc = set_err(ctx, TM_ERR_HIP, "serving: stream creation failed");
            return nullptr;
        }
        rc = tmi::batch_create(ctx, G, k, slots, chunk, B->stream, &B->b, &mem);
        if (rc != TM_OK) {
            (void)hipStreamDestroy(B->stream);
            delete B;
            return nullptr;
        }
        return B;
    }
    void batch_destroy(Batch *B)
    {
        tmi::batch_destroy(B->b);
        (void)hipStreamDestroy(B->stream);
        delete B;
    }
    bool in_flight(Batch *B) const { return B->b->in_flight; }
    int poll(Batch *B)
    {
        const hipError_t q = hipEventQuery(B->b->ev);
        if (q == hipErrorNotReady) return 0;
        if (q == hipSuccess) return 1;
        return set_err(ctx, TM_ERR_HIP, "serving: chunk event: %s", hipGetErrorString(q));
    }
    int process(Batch *B, std::vector<Job *> &fin) { return batch_process(B->b, fin); }
    int free_slot(Batch *B) const { return batch_free_slot(B->b); }
    int active(Batch *B) const { return batch_active(B->b); }
    int fill(Batch *B, Job *const *js, int n) { return batch_fill_many(B->b, js, n); }
    int launch(Batch *B) { return batch_launch_chunk(B->b); }
    void abort(Batch *B, std::vector<Job *> &js)
    {
        for (Job *&j : B->b->slot_job)
            if (j) {
                js.push_back(j);
                j = nullptr;
            }
        B->b->in_flight = false;
    }

    int req_begin(Req &R)
    {
        ReqDev &d = R.dev;
        const size_t need = (size_t)TM_N_OPS * R.lt * 4 * sizeof(double);
        // smallest free pinned buffer that holds the results, else a new one
        size_t best = pinned.size();
        for (size_t i = 0; i < pinned.size(); i++)
            if (pinned[i].first >= need && (best == pinned.size() || pinned[i].first < pinned[best].first)) best = i;
        if (best < pinned.size()) {
            d.h_bytes = pinned[best].first;
            d.h_out = pinned[best].second;
            pinned.erase(pinned.begin() + best);
        } else if (hipHostMalloc((void **)&d.h_out, need, hipHostMallocDefault) == hipSuccess) {
            d.h_bytes = need;
        } else {
            d.h_out = nullptr;
            return set_err(ctx, TM_ERR_HIP, "serving: pinned result buffer");
        }
        if (hipEventCreateWithFlags(&d.ev_hp, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&d.ev_lp, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&d.fin_ev, hipEventDisableTiming) != hipSuccess) {
            release(R);
            return set_err(ctx, TM_ERR_HIP, "serving: event creation failed");
        }
        return TM_OK;
    }
    void job_done(Req &R, Batch *B, bool hp) { (void)hipEventRecord(hp ? R.dev.ev_hp : R.dev.ev_lp, B->stream); }
    int finalize(Req &R)
    {
        const int lt = R.lt, n_hp = R.P.n_hp, n_lpt = R.P.n_hp + R.P.n_lp;
        const size_t ops_per = (size_t)TM_N_OPS * lt * 2;
        if (n_hp > 0) TM_HIP(ctx, hipStreamWaitEvent(fin_stream, R.dev.ev_hp, 0));
        TM_HIP(ctx, hipStreamWaitEvent(fin_stream, R.dev.ev_lp, 0));
        const int *gt = gamma_table();
        launch_project(n_hp, lt, R.raw_hp, R.ops_hp, gt, fin_stream);
        launch_project(n_lpt, lt, R.raw_lp, R.ops_lp, gt, fin_stream);
        launch_tsm_combine(n_hp, R.P.n_lp, lt, R.ops_hp, R.ops_lp, R.ops_lp + (size_t)n_hp * ops_per, R.d_est, R.d_vre,
                           R.d_vim, fin_stream);
        TM_HIP(ctx, hipGetLastError());
        TM_HIP(ctx, hipMemcpyAsync(R.dev.h_out, R.d_est, 2 * ops_per * sizeof(double), hipMemcpyDeviceToHost,
                                   fin_stream));
        TM_HIP(ctx, hipEventRecord(R.dev.fin_ev, fin_stream));
        return TM_OK;
    }
    int fin_poll(Req &R)
    {
        const hipError_t q = hipEventQuery(R.dev.fin_ev);
        if (q == hipErrorNotReady) return 0;
        if (q == hipSuccess) return 1;
        return set_err(ctx, TM_ERR_HIP, "serving: finalization event: %s", hipGetErrorString(q));
    }
    void fin_collect(Req &R, bool ok)
    {
        if (ok) R.res.assign(R.dev.h_out, R.dev.h_out + (size_t)TM_N_OPS * R.lt * 4);
        // after a failed finalization its copy may still be queued: the
        // buffer goes back to the pool only once the stream is past it
        else (void)hipStreamSynchronize(fin_stream);
        release(R);
    }
    void release(Req &R)
    {
        ReqDev &d = R.dev;
        for (hipEvent_t *e : {&d.ev_hp, &d.ev_lp, &d.fin_ev})
            if (*e) {
                (void)hipEventDestroy(*e);
                *e = nullptr;
            }
        if (d.h_out) pinned.emplace_back(d.h_bytes, d.h_out);
        d.h_out = nullptr;
    }
    void free_pinned()
    {
        for (auto &p : pinned) (void)hipHostFree(p.second);
        pinned.clear();
    }
};

using Sched_ = Sched<HipDev>;
using Request = Sched_::Req;

}  // namespace

struct tm_server {
    tm_context *ctx = nullptr;
    HipDev dev;
    Sched_ *sched = nullptr;
    char *arena_base = nullptr;
    std::thread worker;
    double t0 = 0;
};

static double sclock(const tm_server *s) { return now_s() - s->t0; }

static void worker_main(tm_server *S)
{
    (void)hipSetDevice(S->ctx->device);
    Sched_ &Q = *S->sched;
    for (;;) {
        const SchedStep r = Q.step(sclock(S));
        if (r.done) break;
        if (r.progressed) continue;
        if (r.busy) {
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        } else {
            std::unique_lock<std::mutex> lk(Q.mu);
            Q.cv.wait_for(lk, std::chrono::milliseconds(20), [&] { return Q.stop || !Q.queue.empty(); });
        }
    }
    Q.shutdown();
    (void)hipStreamSynchronize(S->dev.fin_stream);
    S->dev.free_pinned();
}

extern "C" int tm_serve_create(tm_context *ctx, int slots, size_t workspace_budget, tm_server **out)
{
    if (!ctx) return TM_ERR_ARG;
    if (!out || slots < 1 || slots > MAX_SLOTS || workspace_budget < (1u << 20))
        return set_err(ctx, TM_ERR_ARG, "tm_serve_create: slots must be 1..%d and the budget >= 1 MiB", MAX_SLOTS);
    *out = nullptr;
    TM_HIP(ctx, hipSetDevice(ctx->device));
    char *base = (char *)dalloc(ctx, workspace_budget);
    if (!base) return set_err(ctx, TM_ERR_NOMEM, "tm_serve_create: cannot allocate the %zu-byte workspace", workspace_budget);
    tm_server *S = new tm_server();
    S->ctx = ctx;
    S->arena_base = base;
    S->dev.ctx = ctx;
    S->dev.slots = slots;
    if (hipStreamCreateWithFlags(&S->dev.fin_stream, hipStreamNonBlocking) != hipSuccess) {
        dfree(ctx, base);
        delete S;
        return set_err(ctx, TM_ERR_HIP, "tm_serve_create: stream creation failed");
    }
    S->sched = new Sched_(S->dev, base, workspace_budget);
    S->dev.mem.alloc = arena_alloc;
    S->dev.mem.free = arena_free;
    S->dev.mem.self = &S->sched->arena;
    S->t0 = now_s();
    S->worker = std::thread(worker_main, S);
    *out = S;
    return TM_OK;
}

extern "C" int tm_serve_footprint(const tm_server *S, const tm_request *req, size_t *bytes)
{
    if (!S || !req || !req->gauge || !bytes) return TM_ERR_ARG;
    int rc = tsm_check(S->ctx, req->gauge, &req->params);
    if (rc) return rc;
    *bytes = S->sched->standalone_bytes(req->gauge, req->params);
    return TM_OK;
}

extern "C" int tm_serve_submit(tm_server *S, const tm_request *req)
{
    if (!S || !req || !req->gauge) return TM_ERR_ARG;
    int rc = tsm_check(S->ctx, req->gauge, &req->params);
    if (rc) return rc;
    if (req->params.ops != 0)
        return set_err(S->ctx, TM_ERR_ARG, "tm_serve_submit: requests compute all operators (ops 0)");
    // never admissible: its own buffers plus fresh batches exceed the arena
    const size_t need = S->sched->standalone_bytes(req->gauge, req->params);
    if (need > S->sched->arena.size)
        return set_err(S->ctx, TM_ERR_NOMEM, "tm_serve_submit: request needs %zu bytes, workspace is %zu", need,
                       S->sched->arena.size);
    Request *R = new Request();
    R->tag = req->tag;
    R->G = req->gauge;
    R->P = req->params;
    S->sched->submit(R, sclock(S));
    return TM_OK;
}

extern "C" int tm_serve_poll(tm_server *S, tm_result *out, int max)
{
    if (!S || (max > 0 && !out)) return TM_ERR_ARG;
    std::vector<Request *> done;
    const int n = S->sched->take_finished(done, max);
    for (int i = 0; i < n; i++) {
        Request *R = done[i];
        tm_result &r = out[i];
        std::memset(&r, 0, sizeof(r));
        r.tag = R->tag;
        r.status = R->status;
        r.lt = R->lt;
        const size_t nops = (size_t)TM_N_OPS * r.lt;
        if (R->res.size() == 4 * nops) {
            r.est = (double *)malloc(2 * nops * sizeof(double));
            r.var_re = (double *)malloc(nops * sizeof(double));
            r.var_im = (double *)malloc(nops * sizeof(double));
            if (r.est && r.var_re && r.var_im) {
                std::memcpy(r.est, R->res.data(), 2 * nops * sizeof(double));
                std::memcpy(r.var_re, R->res.data() + 2 * nops, nops * sizeof(double));
                std::memcpy(r.var_im, R->res.data() + 3 * nops, nops * sizeof(double));
            } else {
                tm_result_free(&r);
                r.status = TM_ERR_NOMEM;
            }
        }
        for (Job &j : R->hp) {
            r.stats.hp_solves++;
            r.stats.hp_iters += j.iters;
            r.stats.hp_max_iters = std::max(r.stats.hp_max_iters, j.iters);
            r.stats.reliable_updates += j.updates;
            r.stats.max_hp_true_resid = std::max(r.stats.max_hp_true_resid, j.true_rel);
        }
        for (Job &j : R->lp) {
            r.stats.lp_solves++;
            r.stats.lp_iters += j.iters;
            r.stats.lp_max_iters = std::max(r.stats.lp_max_iters, j.iters);
            r.stats.max_lp_true_resid = std::max(r.stats.max_lp_true_resid, j.true_rel);
        }
        r.stats.seconds = R->t_done - R->t_admit;
        r.t_submit = R->t_submit;
        r.t_admit = R->t_admit;
        r.t_done = R->t_done;
        delete R;
    }
    return n;
}

extern "C" int tm_serve_drain(tm_server *S)
{
    if (!S) return TM_ERR_ARG;
    S->sched->drain();
    std::lock_guard<std::mutex> lk(S->sched->mu);
    return S->sched->snap.worker_error;
}

extern "C" void tm_result_free(tm_result *r)
{
    if (!r) return;
    free(r->est);
    free(r->var_re);
    free(r->var_im);
    r->est = r->var_re = r->var_im = nullptr;
}

extern "C" double tm_serve_clock(tm_server *S) { return S ? sclock(S) : 0.0; }

extern "C" int tm_serve_status_get(tm_server *S, tm_serve_status *out)
{
    if (!S || !out) return TM_ERR_ARG;
    std::lock_guard<std::mutex> lk(S->sched->mu);
    *out = S->sched->snap;
    return TM_OK;
}

extern "C" int tm_serve_destroy(tm_server *S)
{
    if (!S) return TM_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(S->sched->mu);
        S->sched->stop = true;
    }
    S->sched->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (Request *R : S->sched->finished) delete R;
    S->sched->finished.clear();
    (void)hipStreamDestroy(S->dev.fin_stream);
    delete S->sched;
    dfree(S->ctx, S->arena_base);
    delete S;
    return TM_OK;
}
