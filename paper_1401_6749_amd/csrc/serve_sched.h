// Scheduling state machine of the serving loop, independent of the device.
//
// Requests wait in a FIFO queue until their footprint (output buffers plus
// the batches of their solver kinds that are not resident yet) fits the
// workspace arena; their sources then become jobs on the batch of their
// (gauge field, solver kind), so sources of different requests that share a
// gauge field run in the same multi-RHS launches.  After each chunk of CG
// iterations a batch's finished slots are harvested and refilled from its
// pending jobs; a request whose last job is harvested is finalized
// (projection and TSM combination) and, once that is done, handed to the
// caller.  Batches that hold no work are released when the queue head needs
// their memory.
//
// Every device operation goes through Dev, and Dev is only ever called from
// the thread that runs step() (the worker), so no other thread makes a
// device call while the loop runs.  The serving engine instantiates this
// with the HIP device; a CPU test instantiates it with a simulated device to
// drive the state machine through random arrivals, budgets and failures.
//
// Dev provides:
//   struct Batch; struct ReqDev;                 per-batch and per-request device state
//   int lt(const tm_gauge *)                     time extent of a gauge field
//   size_t batch_bytes(const tm_gauge *, Kind)   arena bytes of a new batch
//   Batch *batch_create(const tm_gauge *, Kind, int chunk, int &rc)
//   void batch_destroy(Batch *)
//   bool in_flight(Batch *)                      a chunk was launched and not processed
//   int poll(Batch *)                            1 chunk done, 0 running, < 0 error
//   int process(Batch *, std::vector<Job *> &)   harvest finished slots (after poll 1)
//   int free_slot(Batch *), active(Batch *)
//   int fill(Batch *, Job *const *, int)         jobs placed into free slots
//   int launch(Batch *)                          next chunk of iterations (tm_status)
//   void abort(Batch *, std::vector<Job *> &)    hand back the jobs in slots, slots empty
//   int req_begin(Req &)                         per-request device state (tm_status)
//   void job_done(Req &, Batch *, bool hp)       after a harvest of one of its jobs
//   int finalize(Req &)                          enqueue projection, TSM and the copy out
//   int fin_poll(Req &)                          1 done, 0 running, < 0 error
//   void fin_collect(Req &, bool ok)             results into Req::res (if ok), release
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

#include "tm.h"
#include "tm_arena.h"
#include "tm_jobs.h"

namespace tmi {

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_FINALIZING, RQ_DONE };

inline Kind sched_kind_of(const tm_solver_params &p) { return kind_of_mode(p.mode, p.half_prec); }

template <class RD>
struct SchedReq {
    uint64_t tag = 0;
    const tm_gauge *G = nullptr;
    tm_tsm_params P{};
    int lt = 0;
    ReqState state = RQ_QUEUED;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<Job> hp, lp;
    int remaining = 0;
    int status = TM_OK;
    // arena buffer: raw spin matrices, projected ops, estimate and variances
    char *dbuf = nullptr;
    double *raw_hp = nullptr, *raw_lp = nullptr, *ops_hp = nullptr, *ops_lp = nullptr;
    double *d_est = nullptr, *d_vre = nullptr, *d_vim = nullptr;
    std::vector<double> res;  // host: est [ops][lt][2], var_re [ops][lt], var_im [ops][lt]
    RD dev{};
};

struct SchedStep {
    bool progressed = false;  // some request or batch changed state
    bool busy = false;        // device work is in flight (chunks or finalizations)
    bool done = false;        // stopped and nothing left
};

template <class Dev>
struct Sched {
    using Req = SchedReq<typename Dev::ReqDev>;
    using Batch = typename Dev::Batch;
    struct BatchRec {
        Batch *b = nullptr;
        std::deque<Job *> pending;
        const tm_gauge *G = nullptr;
        Kind kind = K_F64;
    };

    Dev &dev;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Req *> queue;     // submitted, not admitted (mu)
    std::deque<Req *> finished;  // done, not polled (mu)
    int outstanding = 0;         // submitted, not polled (mu)
    bool stop = false;           // (mu)
    tm_serve_status snap{};      // (mu)
    std::vector<Req *> active;   // worker only
    std::map<std::pair<const tm_gauge *, int>, BatchRec *> batches;  // worker only
    int worker_error = TM_OK;    // worker only (copied into snap)
    double last_progress = 0;    // worker only
    // utilisation integrals (worker only): the state of the last snapshot
    // holds until the next one
    double t_pub = -1, busy_s = 0, slot_s = 0;
    int pub_in_flight = 0, pub_slots = 0;

    Sched(Dev &d, char *base, size_t bytes) : dev(d) { arena.init(base, bytes); }

    static size_t raw_per(int lt) { return (size_t)9 * lt * 32; }
    static size_t ops_per(int lt) { return (size_t)TM_N_OPS * lt * 2; }

    // arena bytes of a request's own buffers
    static size_t req_bytes(int lt, const tm_tsm_params &P)
    {
        const int n_hp = P.n_hp, n_lpt = P.n_hp + P.n_lp;
        return ((size_t)(n_hp + n_lpt) * (raw_per(lt) + ops_per(lt)) + 2 * ops_per(lt)) * sizeof(double) + 4096;
    }

    // arena bytes a request needs given the batches already resident
    size_t footprint(const Req *R) const
    {
        size_t f = req_bytes(R->lt, R->P);
        const Kind kh = sched_kind_of(R->P.hp), kl = sched_kind_of(R->P.lp);
        if (R->P.n_hp > 0 && !batches.count({R->G, (int)kh})) f += dev.batch_bytes(R->G, kh);
        if (!(kl == kh && R->P.n_hp > 0) && !batches.count({R->G, (int)kl})) f += dev.batch_bytes(R->G, kl);
        return f;
    }

    // arena bytes with none of its batches resident
    size_t standalone_bytes(const tm_gauge *G, const tm_tsm_params &P) const
    {
        const Kind kh = sched_kind_of(P.hp), kl = sched_kind_of(P.lp);
        size_t f = req_bytes(dev.lt(G), P);
        if (P.n_hp > 0) f += dev.batch_bytes(G, kh);
        if (!(kl == kh && P.n_hp > 0)) f += dev.batch_bytes(G, kl);
        return f;
    }

    // ---- any thread ----
    // queue a request (ownership passes to the scheduler until poll)
    void submit(Req *R, double now)
    {
        R->lt = dev.lt(R->G);
        R->t_submit = now;
        R->state = RQ_QUEUED;
        {
            std::lock_guard<std::mutex> lk(mu);
            queue.push_back(R);
            outstanding++;
        }
        cv.notify_all();
    }

    // finished requests, oldest first (ownership passes to the caller)
    int take_finished(std::vector<Req *> &out, int max)
    {
        std::lock_guard<std::mutex> lk(mu);
        int n = 0;
        while (n < max && !finished.empty()) {
            out.push_back(finished.front());
            finished.pop_front();
            outstanding--;
            n++;
        }
        return n;
    }

    void drain()
    {
        std::unique_lock<std::mutex> lk(mu);
        cv_done.wait(lk, [&] { return (int)finished.size() >= outstanding; });
    }

    // ---- worker ----
    bool fits(const Req *R) const
    {
        return footprint(R) <= arena.size - arena.used && arena.largest_free() >= req_bytes(R->lt, R->P);
    }

    bool batch_idle(BatchRec *br) { return !dev.in_flight(br->b) && dev.active(br->b) == 0 && br->pending.empty(); }

    void drop_batch(BatchRec *br)
    {
        dev.batch_destroy(br->b);
        batches.erase({br->G, (int)br->kind});
        delete br;
    }

    // release the workspaces of batches that hold no work; true if any
    bool drop_idle()
    {
        std::vector<BatchRec *> idle;
        for (auto &kv : batches)
            if (batch_idle(kv.second)) idle.push_back(kv.second);
        for (BatchRec *br : idle) drop_batch(br);
        return !idle.empty();
    }

    BatchRec *get_batch(const tm_gauge *G, Kind k, int chunk, int &rc)
    {
        auto it = batches.find({G, (int)k});
        if (it != batches.end()) return it->second;
        Batch *b = dev.batch_create(G, k, chunk, rc);
        if (!b) return nullptr;
        BatchRec *br = new BatchRec();
        br->b = b;
        br->G = G;
        br->kind = k;
        batches[{G, (int)k}] = br;
        return br;
    }

    int admit(Req *R, double now)
    {
        const int lt = R->lt;
        const int n_hp = R->P.n_hp, n_lpt = R->P.n_hp + R->P.n_lp;
        R->dbuf = (char *)arena.alloc(req_bytes(lt, R->P));
        if (!R->dbuf) return TM_ERR_NOMEM;
        double *d = (double *)R->dbuf;
        R->raw_hp = d;
        R->raw_lp = R->raw_hp + n_hp * raw_per(lt);
        R->ops_hp = R->raw_lp + n_lpt * raw_per(lt);
        R->ops_lp = R->ops_hp + n_hp * ops_per(lt);
        R->d_est = R->ops_lp + n_lpt * ops_per(lt);
        R->d_vre = R->d_est + ops_per(lt);
        R->d_vim = R->d_vre + ops_per(lt) / 2;
        int rc = TM_OK;
        BatchRec *bh = nullptr, *bl = nullptr;
        if (n_hp > 0) bh = get_batch(R->G, sched_kind_of(R->P.hp), R->P.hp.chunk, rc);
        if (rc == TM_OK) bl = get_batch(R->G, sched_kind_of(R->P.lp), R->P.lp.chunk, rc);
        if (rc == TM_OK) rc = dev.req_begin(*R);
        if (rc != TM_OK) {
            arena.release(R->dbuf);
            R->dbuf = nullptr;
            return rc;
        }
        R->hp.assign(n_hp, Job());
        R->lp.assign(n_lpt, Job());
        auto setup = [&](Job &j, int i, const tm_solver_params &sp, double *raw, bool hp) {
            j.noise = true;
            j.seed = R->P.noise_seed;
            j.src = (uint64_t)i;
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
            setup(R->hp[i], i, R->P.hp, R->raw_hp + i * raw_per(lt), true);
            bh->pending.push_back(&R->hp[i]);
        }
        for (int i = 0; i < n_lpt; i++) {
            setup(R->lp[i], i, R->P.lp, R->raw_lp + i * raw_per(lt), false);
            bl->pending.push_back(&R->lp[i]);
        }
        R->remaining = n_hp + n_lpt;
        R->state = RQ_RUNNING;
        R->t_admit = now;
        return TM_OK;
    }

    // hand a request to the caller (its arena buffer released)
    void complete(Req *R, double now)
    {
        if (R->dbuf) arena.release(R->dbuf);
        R->dbuf = nullptr;
        R->state = RQ_DONE;
        R->t_done = now;
        auto it = std::find(active.begin(), active.end(), R);
        if (it != active.end()) active.erase(it);
        {
            std::lock_guard<std::mutex> lk(mu);
            finished.push_back(R);
        }
        cv_done.notify_all();
    }

    void finalize(Req *R, double now)
    {
        if (R->status == TM_OK || R->status == TM_ERR_NOCONV) {
            const int e = dev.finalize(*R);
            if (e == TM_OK) {
                R->state = RQ_FINALIZING;
                return;
            }
            R->status = e;
            dev.fin_collect(*R, false);
        } else {
            dev.fin_collect(*R, false);
        }
        complete(R, now);
    }

    void job_done(Job *j, Batch *b, double now)
    {
        Req *R = (Req *)j->owner;
        dev.job_done(*R, b, j->hp);
        if (j->status != TM_OK && R->status == TM_OK) R->status = j->status;
        if (--R->remaining == 0) finalize(R, now);
    }

    // a batch that failed: every job in it or waiting for it ends with err
    void fail_batch(BatchRec *br, int err, double now)
    {
        if (worker_error == TM_OK) worker_error = err;
        std::vector<Job *> js;
        dev.abort(br->b, js);
        js.insert(js.end(), br->pending.begin(), br->pending.end());
        br->pending.clear();
        Batch *b = br->b;
        for (Job *j : js) {
            j->status = err;
            job_done(j, b, now);
        }
        drop_batch(br);
    }

    // One pass of the serving loop.
    SchedStep step(double now)
    {
        SchedStep r;
        // ---- admission: FIFO, by footprint ----
        for (;;) {
            Req *R = nullptr;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (queue.empty()) break;
                R = queue.front();  // only this thread pops: it stays the head
            }
            if (!fits(R) && (!drop_idle() || footprint(R) > arena.size - arena.used)) break;
            {
                std::lock_guard<std::mutex> lk(mu);
                queue.pop_front();
            }
            int rc = admit(R, now);
            if (rc == TM_ERR_NOMEM && drop_idle()) rc = admit(R, now);  // free bytes, but not in one piece
            if (rc == TM_ERR_NOMEM && !active.empty()) {
                std::lock_guard<std::mutex> lk(mu);
                queue.push_front(R);  // wait until running requests release memory
                break;
            }
            r.progressed = true;
            if (rc != TM_OK) {
                R->status = rc;
                complete(R, now);
                continue;
            }
            active.push_back(R);
        }
        // ---- batches: harvest, refill, next chunk ----
        std::vector<BatchRec *> brs;
        for (auto &kv : batches) brs.push_back(kv.second);
        for (BatchRec *br : brs) {
            Batch *b = br->b;
            if (dev.in_flight(b)) {
                const int q = dev.poll(b);
                if (q == 0) {
                    r.busy = true;
                    continue;
                }
                r.progressed = true;
                if (q < 0) {
                    fail_batch(br, q, now);
                    continue;
                }
                std::vector<Job *> fin;
                const int e = dev.process(b, fin);
                if (e != TM_OK && worker_error == TM_OK) worker_error = e;
                for (Job *j : fin) job_done(j, b, now);
            }
            if (!br->pending.empty() && dev.free_slot(b) >= 0) {
                std::vector<Job *> js(br->pending.begin(), br->pending.end());
                const int m = dev.fill(b, js.data(), (int)js.size());
                for (int i = 0; i < m; i++) br->pending.pop_front();
                r.progressed = true;
            }
            if (dev.active(b) > 0) {
                const int e = dev.launch(b);
                if (e != TM_OK) {
                    fail_batch(br, e, now);
                    r.progressed = true;
                    continue;
                }
                r.busy = true;
            }
        }
        // ---- finalized requests ----
        std::vector<Req *> fin;
        for (Req *R : active)
            if (R->state == RQ_FINALIZING) fin.push_back(R);
        for (Req *R : fin) {
            const int q = dev.fin_poll(*R);
            if (q == 0) {
                r.busy = true;
                continue;
            }
            if (q < 0) R->status = q;
            dev.fin_collect(*R, q > 0);
            complete(R, now);
            r.progressed = true;
        }
        if (r.progressed) last_progress = now;
        publish(now);
        {
            std::lock_guard<std::mutex> lk(mu);
            r.done = stop && queue.empty() && active.empty();
        }
        return r;
    }

    // snapshot for the status call
    void publish(double now)
    {
        tm_serve_status st{};
        st.active = (int)active.size();
        st.batches = (int)batches.size();
        for (auto &kv : batches) {
            st.in_flight += dev.in_flight(kv.second->b) ? 1 : 0;
            st.pending_jobs += (int)kv.second->pending.size();
            st.running_slots += dev.active(kv.second->b);
        }
        if (t_pub >= 0 && now > t_pub) {
            if (pub_in_flight > 0) busy_s += now - t_pub;
            slot_s += (now - t_pub) * pub_slots;
        }
        t_pub = now;
        pub_in_flight = st.in_flight;
        pub_slots = st.running_slots;
        st.busy_s = busy_s;
        st.slot_s = slot_s;
        st.worker_error = worker_error;
        st.arena_used = arena.used;
        st.arena_size = arena.size;
        st.arena_largest_free = arena.largest_free();
        st.t_snapshot = now;
        std::lock_guard<std::mutex> lk(mu);
        st.queued = (int)queue.size();
        st.finished = (int)finished.size();
        if (queue.empty() && active.empty()) last_progress = now;  // idle: nothing can stall
        st.stall_s = now - last_progress;
        snap = st;
    }

    // release every batch (worker, at the end)
    void shutdown()
    {
        std::vector<BatchRec *> all;
        for (auto &kv : batches) all.push_back(kv.second);
        for (BatchRec *br : all) drop_batch(br);
    }
};

}  // namespace tmi
