// Serving loop: continuous batching of loop requests.
//
// A worker thread owns every device operation.  Requests wait in a FIFO
// queue until their device footprint fits the workspace arena (admission by
// footprint); their sources become jobs on the batch of their (gauge field,
// solver kind), so sources of different requests that share a gauge field
// run in the same multi-RHS launches.  Between chunks of CG iterations the
// worker harvests finished slots and refills them from any request (a slot
// freed by one request is taken by the next job in line), batches on
// different gauge fields run on their own streams and overlap on the
// device, and a request's projection and TSM combination run on a separate
// stream once its last source is contracted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "tm_arena.h"
#include "tm_internal.h"

using namespace tmk;
using namespace tmi;

int tsm_check(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P);

namespace {

void *arena_alloc(void *self, size_t n) { return ((tmi::Arena *)self)->alloc(n); }
void arena_free(void *self, void *p) { ((tmi::Arena *)self)->release(p); }

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_FINALIZING, RQ_DONE };

struct Request {
    uint64_t tag = 0;
    const tm_gauge *G = nullptr;
    tm_tsm_params P;
    ReqState state = RQ_QUEUED;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<Job> hp, lp;
    int remaining = 0;
    int status = TM_OK;
    char *dbuf = nullptr;  // raw, ops, est, var (arena)
    double *raw_hp = nullptr, *raw_lp = nullptr, *ops_hp = nullptr, *ops_lp = nullptr;
    double *d_est = nullptr, *d_vre = nullptr, *d_vim = nullptr;
    double *h_out = nullptr;  // pinned: est, vre, vim
    hipEvent_t fin_ev = nullptr;
    // recorded on a batch stream after each harvest of this request's HP /
    // LP sources; the finalization stream waits on both (no batch pointers
    // are kept: an idle batch may be released before the request finishes)
    hipEvent_t ev_hp = nullptr, ev_lp = nullptr;
};

struct BatchRec {
    Batch *b = nullptr;
    hipStream_t stream = nullptr;
    std::deque<Job *> pending;
    const tm_gauge *G = nullptr;
    Kind kind = K_F64;
};

size_t req_bytes(const tm_gauge *G, const tm_tsm_params &P)
{
    const int lt = G->dims[3];
    const size_t raw_per = (size_t)9 * lt * 32, ops_per = (size_t)TM_N_OPS * lt * 2;
    const int n_hp = P.n_hp, n_lpt = P.n_hp + P.n_lp;
    return ((size_t)(n_hp + n_lpt) * (raw_per + ops_per) + 2 * ops_per) * sizeof(double) + 4096;
}

}  // namespace

struct tm_server {
    tm_context *ctx = nullptr;
    int slots = 12;
    tmi::Arena arena;
    char *arena_base = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request *> queue;        // submitted, not admitted (guarded by mu)
    std::vector<Request *> active;      // worker only
    std::deque<Request *> finished;     // guarded by mu
    int outstanding = 0;                // guarded by mu
    bool stop = false;
    std::map<std::pair<const tm_gauge *, int>, BatchRec *> batches;  // worker only
    hipStream_t fin_stream = nullptr;
    double t0 = 0;
    Mem mem;
    int worker_error = TM_OK;
    tm_serve_status snap{};  // guarded by mu
};

static double sclock(tm_server *s) { return now_s() - s->t0; }

static BatchRec *get_batch(tm_server *S, const tm_gauge *G, Kind k, int chunk, int &rc)
{
    auto key = std::make_pair(G, (int)k);
    auto it = S->batches.find(key);
    if (it != S->batches.end()) return it->second;
    BatchRec *br = new BatchRec();
    br->G = G;
    br->kind = k;
    if (hipStreamCreateWithFlags(&br->stream, hipStreamNonBlocking) != hipSuccess) {
        delete br;
        rc = TM_ERR_HIP;
        return nullptr;
    }
    rc = batch_create(S->ctx, G, k, S->slots, chunk, br->stream, &br->b, &S->mem);
    if (rc != TM_OK) {
        (void)hipStreamDestroy(br->stream);
        delete br;
        return nullptr;
    }
    S->batches[key] = br;
    return br;
}

static void drop_batch(tm_server *S, BatchRec *br)
{
    batch_destroy(br->b);
    (void)hipStreamDestroy(br->stream);
    for (auto it = S->batches.begin(); it != S->batches.end(); ++it)
        if (it->second == br) {
            S->batches.erase(it);
            break;
        }
    delete br;
}

static bool batch_idle(BatchRec *br) { return !br->b->in_flight && batch_active(br->b) == 0 && br->pending.empty(); }

// footprint of a request given the batches already resident
static size_t footprint(tm_server *S, Request *R)
{
    size_t f = req_bytes(R->G, R->P);
    Kind kh = kind_of(R->P.hp), kl = kind_of(R->P.lp);
    if (R->P.n_hp > 0 && !S->batches.count({R->G, (int)kh})) f += batch_footprint(R->G, kh, S->slots) + 32 * 256;
    if (!(kl == kh && R->P.n_hp > 0) && !S->batches.count({R->G, (int)kl}))
        f += batch_footprint(R->G, kl, S->slots) + 32 * 256;
    return f;
}

// workspace a request needs when none of its batches is resident
static size_t standalone_bytes(const tm_server *S, const tm_gauge *G, const tm_tsm_params &P)
{
    const Kind kh = kind_of(P.hp), kl = kind_of(P.lp);
    size_t f = req_bytes(G, P);
    if (P.n_hp > 0) f += batch_footprint(G, kh, S->slots) + 32 * 256;
    if (!(kl == kh && P.n_hp > 0)) f += batch_footprint(G, kl, S->slots) + 32 * 256;
    return f;
}

static int admit(tm_server *S, Request *R)
{
    const int lt = R->G->dims[3];
    const size_t raw_per = (size_t)9 * lt * 32, ops_per = (size_t)TM_N_OPS * lt * 2;
    const int n_hp = R->P.n_hp, n_lpt = R->P.n_hp + R->P.n_lp;
    R->dbuf = (char *)S->arena.alloc(req_bytes(R->G, R->P));
    if (!R->dbuf) return TM_ERR_NOMEM;
    double *d = (double *)R->dbuf;
    R->raw_hp = d;
    R->raw_lp = R->raw_hp + n_hp * raw_per;
    R->ops_hp = R->raw_lp + n_lpt * raw_per;
    R->ops_lp = R->ops_hp + n_hp * ops_per;
    R->d_est = R->ops_lp + n_lpt * ops_per;
    R->d_vre = R->d_est + ops_per;
    R->d_vim = R->d_vre + ops_per / 2;
    int rc = TM_OK;
    BatchRec *bh = nullptr, *bl = nullptr;
    if (n_hp > 0) {
        bh = get_batch(S, R->G, kind_of(R->P.hp), R->P.hp.chunk, rc);
        if (!bh) {
            S->arena.release(R->dbuf);
            R->dbuf = nullptr;
            return rc;
        }
    }
    bl = get_batch(S, R->G, kind_of(R->P.lp), R->P.lp.chunk, rc);
    if (!bl) {
        S->arena.release(R->dbuf);
        R->dbuf = nullptr;
        return rc;
    }
    R->hp.resize(n_hp);
    R->lp.resize(n_lpt);
    auto setup = [&](Job &j, int i, const tm_solver_params &sp, double *raw, bool hp) {
        j.noise = true;
        j.seed = R->P.noise_seed;
        j.src = i;
        j.kappa = R->P.kappa;
        j.a = R->P.two_kappa_mu;
        j.tol = sp.tol;
        j.max_iter = sp.max_iter;
        j.fixed = sp.fixed_iters;
        j.delta = sp.delta > 0 ? sp.delta : TM_DEFAULT_DELTA;
        j.raw_out = raw;
        j.want_true = R->P.want_true_resid;
        j.owner = R;
        j.hp = hp;
    };
    for (int i = 0; i < n_hp; i++) {
        setup(R->hp[i], i, R->P.hp, R->raw_hp + i * raw_per, true);
        bh->pending.push_back(&R->hp[i]);
    }
    for (int i = 0; i < n_lpt; i++) {
        setup(R->lp[i], i, R->P.lp, R->raw_lp + i * raw_per, false);
        bl->pending.push_back(&R->lp[i]);
    }
    R->remaining = n_hp + n_lpt;
    if (!R->ev_hp && hipEventCreateWithFlags(&R->ev_hp, hipEventDisableTiming) != hipSuccess) return TM_ERR_HIP;
    if (!R->ev_lp && hipEventCreateWithFlags(&R->ev_lp, hipEventDisableTiming) != hipSuccess) return TM_ERR_HIP;
    R->state = RQ_RUNNING;
    R->t_admit = sclock(S);
    return TM_OK;
}

static void finalize(tm_server *S, Request *R)
{
    const int lt = R->G->dims[3];
    const size_t ops_per = (size_t)TM_N_OPS * lt * 2;
    if (R->P.n_hp > 0) (void)hipStreamWaitEvent(S->fin_stream, R->ev_hp, 0);
    (void)hipStreamWaitEvent(S->fin_stream, R->ev_lp, 0);
    const int *gt = gamma_table();
    const int n_hp = R->P.n_hp, n_lpt = R->P.n_hp + R->P.n_lp;
    launch_project(n_hp, lt, R->raw_hp, R->ops_hp, gt, S->fin_stream);
    launch_project(n_lpt, lt, R->raw_lp, R->ops_lp, gt, S->fin_stream);
    launch_tsm_combine(n_hp, R->P.n_lp, lt, R->ops_hp, R->ops_lp, R->ops_lp + (size_t)n_hp * ops_per, R->d_est,
                       R->d_vre, R->d_vim, S->fin_stream);
    (void)hipMemcpyAsync(R->h_out, R->d_est, 2 * ops_per * sizeof(double), hipMemcpyDeviceToHost, S->fin_stream);
    (void)hipEventCreateWithFlags(&R->fin_ev, hipEventDisableTiming);
    (void)hipEventRecord(R->fin_ev, S->fin_stream);
    R->state = RQ_FINALIZING;
}

static void worker_main(tm_server *S)
{
    (void)hipSetDevice(S->ctx->device);
    for (;;) {
        bool progressed = false;
        // ---- admission (FIFO, by footprint) ----
        {
            std::unique_lock<std::mutex> lk(S->mu);
            while (!S->queue.empty()) {
                Request *R = S->queue.front();
                if (footprint(S, R) > S->arena.size - S->arena.used || S->arena.largest_free() < req_bytes(R->G, R->P)) {
                    // free workspaces of idle batches, then retry once
                    bool dropped = false;
                    for (auto it = S->batches.begin(); it != S->batches.end();) {
                        BatchRec *br = (it++)->second;
                        if (batch_idle(br)) {
                            lk.unlock();
                            drop_batch(S, br);
                            lk.lock();
                            dropped = true;
                        }
                    }
                    if (!dropped || footprint(S, R) > S->arena.size - S->arena.used) break;
                }
                S->queue.pop_front();
                lk.unlock();
                int rc = admit(S, R);
                if (rc == TM_ERR_NOMEM) {
                    // the free bytes suffice but not in one piece: free the
                    // workspaces of idle batches and try again
                    for (auto it = S->batches.begin(); it != S->batches.end();) {
                        BatchRec *br = (it++)->second;
                        if (batch_idle(br)) drop_batch(S, br);
                    }
                    rc = admit(S, R);
                }
                lk.lock();
                if (rc == TM_ERR_NOMEM && !S->active.empty()) {
                    S->queue.push_front(R);  // wait for memory
                    break;
                }
                if (rc != TM_OK) {
                    R->status = rc;
                    R->state = RQ_DONE;
                    R->t_done = sclock(S);
                    S->finished.push_back(R);
                    S->cv_done.notify_all();
                    continue;
                }
                S->active.push_back(R);
                progressed = true;
            }
            if (S->stop && S->queue.empty() && S->active.empty()) break;
        }
        // ---- batches ----
        std::vector<BatchRec *> brs;
        for (auto &kv : S->batches) brs.push_back(kv.second);
        bool any_flight = false;
        for (BatchRec *br : brs) {
            Batch *b = br->b;
            if (b->in_flight) {
                hipError_t q = hipEventQuery(b->ev);
                if (q == hipErrorNotReady) {
                    any_flight = true;
                    continue;
                }
                std::vector<Job *> fin;
                int e = batch_process(b, fin);
                if (e != TM_OK && S->worker_error == TM_OK) S->worker_error = e;
                for (Job *j : fin) {
                    Request *R = (Request *)j->owner;
                    (void)hipEventRecord(j->hp ? R->ev_hp : R->ev_lp, br->stream);
                    if (j->status != TM_OK && R->status == TM_OK) R->status = j->status;
                    if (--R->remaining == 0) finalize(S, R);
                }
                progressed = true;
            }
            if (!br->pending.empty() && batch_free_slot(b) >= 0) {
                std::vector<Job *> js(br->pending.begin(), br->pending.end());
                const int m = batch_fill_many(b, js.data(), (int)js.size());
                for (int i = 0; i < m; i++) br->pending.pop_front();
                progressed = true;
            }
            if (batch_active(b) > 0) {
                batch_launch_chunk(b);
                any_flight = true;
            }
        }
        // ---- finished requests ----
        for (size_t i = 0; i < S->active.size();) {
            Request *R = S->active[i];
            if (R->state == RQ_FINALIZING && hipEventQuery(R->fin_ev) == hipSuccess) {
                (void)hipEventDestroy(R->fin_ev);
                (void)hipEventDestroy(R->ev_hp);
                (void)hipEventDestroy(R->ev_lp);
                R->fin_ev = R->ev_hp = R->ev_lp = nullptr;
                S->arena.release(R->dbuf);
                R->dbuf = nullptr;
                R->t_done = sclock(S);
                R->state = RQ_DONE;
                S->active.erase(S->active.begin() + i);
                std::lock_guard<std::mutex> lk(S->mu);
                S->finished.push_back(R);
                S->cv_done.notify_all();
                progressed = true;
                continue;
            }
            i++;
        }
        {
            // publish a snapshot for tm_serve_status_get
            tm_serve_status st{};
            st.active = (int)S->active.size();
            st.batches = (int)S->batches.size();
            for (auto &kv : S->batches) {
                st.in_flight += kv.second->b->in_flight ? 1 : 0;
                st.pending_jobs += (int)kv.second->pending.size();
                st.running_slots += batch_active(kv.second->b);
            }
            st.worker_error = S->worker_error;
            st.arena_used = S->arena.used;
            st.arena_size = S->arena.size;
            st.arena_largest_free = S->arena.largest_free();
            st.t_snapshot = sclock(S);
            std::lock_guard<std::mutex> lk(S->mu);
            st.queued = (int)S->queue.size();
            st.finished = (int)S->finished.size();
            S->snap = st;
        }
        if (!progressed) {
            bool finalizing = false;
            for (Request *R : S->active) finalizing |= R->state == RQ_FINALIZING;
            if (any_flight || finalizing) {
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            } else {
                std::unique_lock<std::mutex> lk(S->mu);
                S->cv.wait_for(lk, std::chrono::milliseconds(20), [&] { return S->stop || !S->queue.empty(); });
            }
        }
    }
    for (auto &kv : S->batches) {
        batch_destroy(kv.second->b);
        (void)hipStreamDestroy(kv.second->stream);
        delete kv.second;
    }
    S->batches.clear();
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
    S->slots = slots;
    S->arena_base = base;
    S->arena.init(base, workspace_budget);
    S->mem.alloc = arena_alloc;
    S->mem.free = arena_free;
    S->mem.self = &S->arena;
    S->t0 = now_s();
    if (hipStreamCreateWithFlags(&S->fin_stream, hipStreamNonBlocking) != hipSuccess) {
        dfree(ctx, base);
        delete S;
        return set_err(ctx, TM_ERR_HIP, "tm_serve_create: stream creation failed");
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return TM_OK;
}

extern "C" int tm_serve_footprint(const tm_server *S, const tm_request *req, size_t *bytes)
{
    if (!S || !req || !req->gauge || !bytes) return TM_ERR_ARG;
    int rc = tsm_check(S->ctx, req->gauge, &req->params);
    if (rc) return rc;
    *bytes = standalone_bytes(S, req->gauge, req->params);
    return TM_OK;
}

extern "C" int tm_serve_submit(tm_server *S, const tm_request *req)
{
    if (!S || !req || !req->gauge) return TM_ERR_ARG;
    int rc = tsm_check(S->ctx, req->gauge, &req->params);
    if (rc) return rc;
    if (req->params.ops != 0)
        return set_err(S->ctx, TM_ERR_ARG, "tm_serve_submit: requests compute all operators (ops 0)");
    Request *R = new Request();
    R->tag = req->tag;
    R->G = req->gauge;
    R->P = req->params;
    R->t_submit = sclock(S);
    // never admissible: its own buffers plus fresh batches exceed the arena
    const size_t need = standalone_bytes(S, R->G, R->P);
    if (need > S->arena.size) {
        delete R;
        return set_err(S->ctx, TM_ERR_NOMEM, "tm_serve_submit: request needs %zu bytes, workspace is %zu", need,
                       S->arena.size);
    }
    const int lt = R->G->dims[3];
    if (hipHostMalloc((void **)&R->h_out, (size_t)TM_N_OPS * lt * 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete R;
        return set_err(S->ctx, TM_ERR_HIP, "tm_serve_submit: pinned buffer");
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->queue.push_back(R);
        S->outstanding++;
    }
    S->cv.notify_all();
    return TM_OK;
}

extern "C" int tm_serve_poll(tm_server *S, tm_result *out, int max)
{
    if (!S || (max > 0 && !out)) return TM_ERR_ARG;
    // pinned buffers are released after the lock: hipHostFree may wait for
    // the device, and the worker must not wait for it on the lock
    std::vector<double *> unpin;
    std::unique_lock<std::mutex> lk(S->mu);
    int n = 0;
    while (n < max && !S->finished.empty()) {
        Request *R = S->finished.front();
        S->finished.pop_front();
        S->outstanding--;
        tm_result &r = out[n++];
        std::memset(&r, 0, sizeof(r));
        r.tag = R->tag;
        r.status = R->status;
        r.lt = R->G->dims[3];
        const size_t nops = (size_t)TM_N_OPS * r.lt;
        if (R->status == TM_OK || R->status == TM_ERR_NOCONV) {
            r.est = (double *)malloc(2 * nops * sizeof(double));
            r.var_re = (double *)malloc(nops * sizeof(double));
            r.var_im = (double *)malloc(nops * sizeof(double));
            std::memcpy(r.est, R->h_out, 2 * nops * sizeof(double));
            std::memcpy(r.var_re, R->h_out + 2 * nops, nops * sizeof(double));
            std::memcpy(r.var_im, R->h_out + 3 * nops, nops * sizeof(double));
        }
        std::memset(&r.stats, 0, sizeof(r.stats));
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
        unpin.push_back(R->h_out);
        delete R;
    }
    lk.unlock();
    for (double *h : unpin) (void)hipHostFree(h);
    return n;
}

extern "C" int tm_serve_drain(tm_server *S)
{
    if (!S) return TM_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return (int)S->finished.size() >= S->outstanding; });
    return S->worker_error;
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
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->snap;
    return TM_OK;
}

extern "C" int tm_serve_destroy(tm_server *S)
{
    if (!S) return TM_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (Request *R : S->finished) {
        (void)hipHostFree(R->h_out);
        delete R;
    }
    (void)hipStreamSynchronize(S->fin_stream);
    (void)hipStreamDestroy(S->fin_stream);
    dfree(S->ctx, S->arena_base);
    delete S;
    return TM_OK;
}
