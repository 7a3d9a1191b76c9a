// CPU harness of the serving scheduler (paper_1401_6749_amd/csrc/serve_sched.h).
//
// It drives the scheduler's state machine -- admission by footprint, batches
// per (gauge field, solver kind), slot refill between chunks, harvest,
// per-request finalization -- with a simulated device on a virtual clock:
// every chunk of CG iterations takes a time that grows with the lattice
// volume and the slots in use, every solve needs a random number of
// iterations, and (in some scenarios) batch creation, chunk launches, chunk
// completion, request set-up and finalization fail at random.  Requests
// arrive as a seeded Poisson stream over four lattice sizes under a
// workspace budget small enough that admission has to wait.
//
// After every step it checks the invariants (arena within its size, every
// job in exactly one place, batches keep their jobs, FIFO admission).  When a
// step makes no progress it advances the clock to the next event; if there
// is none while requests are outstanding, the loop is stuck: the harness
// prints that state and exits with status 1.  At the end every request must
// be finished exactly once, with correct results unless a failure was
// injected on its path.
//
// usage: serve_sim SEED SCENARIOS
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "serve_sched.h"

// The harness's stand-in for a gauge field: the scheduler only reads the
// lattice through the device (lt) and uses the pointer as a key.
struct tm_gauge {
    int dims[4];
};

using namespace tmi;

namespace {

int g_fail = 0;
void fail(const char *fmt, const char *a = "", long long b = 0, long long c = 0)
{
    std::fprintf(stderr, "serve_sim: ");
    std::fprintf(stderr, fmt, a, b, c);
    std::fprintf(stderr, "\n");
    g_fail = 1;
}

double volume(const tm_gauge *G) { return (double)G->dims[0] * G->dims[1] * G->dims[2] * G->dims[3]; }

struct SimDev {
    std::mt19937_64 rng;
    double now = 0;
    int slots = 12;
    Mem mem;
    // failure probabilities (per call)
    double p_create = 0, p_launch = 0, p_poll = 0, p_begin = 0, p_fin = 0;
    long long injected = 0;
    std::set<const void *> failed_reqs;  // requests with an injected set-up or finalization failure
    std::multiset<double> create_fail_t;  // times of injected batch-creation failures

    struct Batch {
        const tm_gauge *G = nullptr;
        Kind k = K_F64;
        int chunk = 8;
        std::vector<Job *> slot;
        std::vector<int> left;
        bool in_flight = false;
        bool poisoned = false;  // its next poll fails
        double t_done = 0;
        void *mem = nullptr;
    };
    struct ReqDev {
        bool begun = false;
        double t_fin = -1;
        int jobs_done = 0;
    };
    using Req = SchedReq<ReqDev>;
    std::set<Batch *> live;

    double u() { return std::uniform_real_distribution<double>(0, 1)(rng); }
    bool roll(double p) { return p > 0 && u() < p; }

    int lt(const tm_gauge *G) const { return G->dims[3]; }
    // bytes per site per slot of the kind's workspace (LP smaller than mixed HP)
    size_t batch_bytes(const tm_gauge *G, Kind k) const
    {
        const double per = k == K_MIXED ? 720.0 : k == K_F64 ? 900.0 : 330.0;
        return (size_t)(volume(G) * per * slots) + 8192;
    }
    Batch *batch_create(const tm_gauge *G, Kind k, int chunk, int &rc)
    {
        void *p = mem.alloc(mem.self, batch_bytes(G, k));
        if (!p) {
            rc = TM_ERR_NOMEM;
            return nullptr;
        }
        if (roll(p_create)) {
            mem.free(mem.self, p);
            injected++;
            create_fail_t.insert(now);
            rc = TM_ERR_HIP;
            return nullptr;
        }
        Batch *B = new Batch();
        B->G = G;
        B->k = k;
        B->chunk = chunk > 0 ? chunk : (k == K_LP16 || k == K_LPBF ? 4 : 8);
        B->slot.assign(slots, nullptr);
        B->left.assign(slots, 0);
        B->mem = p;
        live.insert(B);
        rc = TM_OK;
        return B;
    }
    void batch_destroy(Batch *B)
    {
        for (Job *j : B->slot)
            if (j) fail("batch destroyed while a slot holds a job%s", "");
        if (B->in_flight) fail("batch destroyed with a chunk in flight%s", "");
        mem.free(mem.self, B->mem);
        live.erase(B);
        delete B;
    }
    bool in_flight(Batch *B) const { return B->in_flight; }
    int poll(Batch *B)
    {
        if (now < B->t_done) return 0;
        if (B->poisoned || roll(p_poll)) {
            injected++;
            for (Job *j : B->slot)
                if (j) failed_reqs.insert(j->owner);
            return TM_ERR_HIP;
        }
        return 1;
    }
    int process(Batch *B, std::vector<Job *> &fin)
    {
        if (!B->in_flight || now < B->t_done) fail("process before the chunk completed%s", "");
        B->in_flight = false;
        for (int s = 0; s < slots; s++) {
            Job *j = B->slot[s];
            if (!j || B->left[s] > 0) continue;
            j->status = TM_OK;
            fin.push_back(j);
            B->slot[s] = nullptr;
        }
        return TM_OK;
    }
    int free_slot(Batch *B) const
    {
        for (int s = 0; s < slots; s++)
            if (!B->slot[s]) return s;
        return -1;
    }
    int active(Batch *B) const
    {
        int n = 0;
        for (Job *j : B->slot) n += j != nullptr;
        return n;
    }
    int fill(Batch *B, Job *const *js, int n)
    {
        if (B->in_flight) fail("fill while a chunk is in flight%s", "");
        int m = 0;
        for (int s = 0; s < slots && m < n; s++) {
            if (B->slot[s]) continue;
            Job *j = js[m++];
            B->slot[s] = j;
            // iterations: LP ~ 7, HP ~ 48 (spread); fixed counts honoured
            const int base = (B->k == K_LP16 || B->k == K_LPBF) ? 7 : 48;
            const int it = j->fixed > 0 ? j->fixed : std::max(1, base + (int)(rng() % 9) - 4);
            j->iters = it;
            B->left[s] = it;
        }
        return m;
    }
    int launch(Batch *B)
    {
        if (B->in_flight) fail("launch while a chunk is in flight%s", "");
        if (roll(p_launch)) {
            injected++;
            for (Job *j : B->slot)
                if (j) failed_reqs.insert(j->owner);
            return TM_ERR_HIP;
        }
        // the chunk's duration: per-iteration cost ~ volume and slots in use
        const double t_it = 2e-5 + volume(B->G) * (B->k == K_MIXED || B->k == K_F64 ? 2.2e-9 : 0.8e-9) *
                                       (0.4 + 0.05 * active(B));
        B->t_done = now + B->chunk * t_it;
        B->in_flight = true;
        for (int s = 0; s < slots; s++)
            if (B->slot[s]) B->left[s] -= B->chunk;
        return TM_OK;
    }
    void abort(Batch *B, std::vector<Job *> &js)
    {
        for (Job *&j : B->slot)
            if (j) {
                js.push_back(j);
                failed_reqs.insert(j->owner);
                j = nullptr;
            }
        B->in_flight = false;
    }
    int req_begin(Req &R)
    {
        if (roll(p_begin)) {
            injected++;
            failed_reqs.insert(&R);
            return TM_ERR_HIP;
        }
        R.dev.begun = true;
        return TM_OK;
    }
    void job_done(Req &R, Batch *, bool) { R.dev.jobs_done++; }
    int finalize(Req &R)
    {
        if (!R.dev.begun) fail("finalize of a request that was not set up%s", "");
        if (R.dev.jobs_done != (int)(R.hp.size() + R.lp.size())) fail("finalize before every job was harvested%s", "");
        if (roll(p_fin)) {
            injected++;
            failed_reqs.insert(&R);
            return TM_ERR_HIP;
        }
        R.dev.t_fin = now + 1e-4 + 1e-6 * (R.hp.size() + R.lp.size());
        return TM_OK;
    }
    int fin_poll(Req &R) { return now >= R.dev.t_fin ? 1 : 0; }
    void fin_collect(Req &R, bool ok)
    {
        if (ok) {
            // a result that identifies the request and its sources
            R.res.assign((size_t)TM_N_OPS * R.lt * 4, 0.0);
            R.res[0] = (double)R.tag;
            R.res[1] = (double)(R.hp.size() + R.lp.size());
        }
        R.dev.begun = false;
    }
};

const int SIZES[4][4] = {{8, 8, 8, 16}, {16, 16, 16, 32}, {24, 24, 24, 48}, {32, 32, 32, 64}};

struct Scenario {
    int n_req;
    double budget_factor;  // arena = factor x the largest standalone footprint
    double load;           // arrival rate relative to an estimate of the capacity
    bool failures;
    int slots;
};

using S_ = Sched<SimDev>;
using Req = S_::Req;

void dump(const S_ &Q, const SimDev &dev)
{
    std::fprintf(stderr, "state at t = %.6f: queued %zu, active %zu, finished %zu, outstanding %d, batches %zu, arena %zu/%zu "
                         "(largest free %zu)\n",
                 dev.now, Q.queue.size(), Q.active.size(), Q.finished.size(), Q.outstanding, Q.batches.size(),
                 Q.arena.used, Q.arena.size, Q.arena.largest_free());
    for (Req *R : Q.active)
        std::fprintf(stderr, "  active request %" PRIu64 ": state %d, remaining %d, status %d\n", R->tag, (int)R->state,
                     R->remaining, R->status);
    if (!Q.queue.empty()) {
        const Req *R = Q.queue.front();
        std::fprintf(stderr, "  queue head %" PRIu64 ": footprint %zu\n", R->tag, Q.footprint(R));
    }
    for (auto &kv : Q.batches)
        std::fprintf(stderr, "  batch lt=%d kind %d: in flight %d, active %d, pending %zu\n", kv.second->G->dims[3],
                     (int)kv.second->kind, (int)kv.second->b->in_flight, dev.active(kv.second->b),
                     kv.second->pending.size());
}

// returns requests completed; 0 on failure (g_fail set)
long long run(uint64_t seed, const Scenario &sc)
{
    std::mt19937_64 rng(seed);
    auto ui = [&](int a, int b) { return a + (int)(rng() % (uint64_t)(b - a + 1)); };
    auto ur = [&](double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); };
    std::vector<tm_gauge> gauges;
    for (int s = 0; s < 4; s++)
        for (int k = 0; k < 2; k++) gauges.push_back(tm_gauge{{SIZES[s][0], SIZES[s][1], SIZES[s][2], SIZES[s][3]}});
    SimDev dev;
    dev.rng.seed(seed ^ 0x9E3779B97F4A7C15ull);
    dev.slots = sc.slots;
    if (sc.failures) {
        dev.p_create = 0.02;
        dev.p_launch = 0.002;
        dev.p_poll = 0.002;
        dev.p_begin = 0.02;
        dev.p_fin = 0.02;
    }
    // requests
    struct Sub {
        const tm_gauge *G;
        tm_tsm_params P;
        double t;
    };
    std::vector<Sub> subs;
    double t = 0, work = 0;
    size_t biggest = 0;
    std::vector<tm_tsm_params> ps;
    for (int i = 0; i < sc.n_req; i++) {
        const tm_gauge *G = &gauges[ui(0, (int)gauges.size() - 1)];
        tm_tsm_params P{};
        P.kappa = 0.1636;
        P.two_kappa_mu = (rng() & 1) ? 0.0033 : 0.01;
        P.noise_seed = 1000 + i;
        P.n_hp = (rng() % 8 == 0) ? 0 : ui(4, 24);
        P.n_lp = ui(50, 500);
        P.hp.mode = (rng() % 5 == 0) ? TM_SOLVE_F64 : TM_SOLVE_MIXED;
        P.hp.tol = 1e-10;
        P.hp.max_iter = 100000;
        P.lp.mode = (rng() % 7 == 0) ? TM_SOLVE_F64 : TM_SOLVE_LP;
        P.lp.half_prec = (rng() % 3 == 0) ? TM_PREC_BF16 : TM_PREC_F16;
        P.lp.tol = 1e-2;
        P.lp.max_iter = 100000;
        P.lp.fixed_iters = (rng() % 10 == 0) ? ui(1, 12) : 0;
        P.batch = sc.slots;
        subs.push_back({G, P, 0});
        work += (P.n_hp * 6 + P.n_hp + P.n_lp) * volume(G);
    }
    {
        // the arena: a multiple of the largest standalone footprint
        Arena tmp;
        S_ probe(dev, (char *)(uintptr_t)0x100000000ull, (size_t)1 << 50);
        for (auto &s : subs) biggest = std::max(biggest, probe.standalone_bytes(s.G, s.P));
    }
    const size_t budget = (size_t)(sc.budget_factor * biggest) + 4096;
    // Poisson arrivals at `load` x (an estimate of) the capacity
    const double cap = 1.0 / (0.8e-9 * 8.0 / sc.slots);  // site-iterations per second, LP-equivalent
    const double rate = sc.load * cap / (work / sc.n_req * 8.0);
    for (auto &s : subs) {
        t += -std::log(1.0 - ur(0, 1)) / rate;
        s.t = t;
    }
    S_ Q(dev, (char *)(uintptr_t)0x100000000ull, budget);
    dev.mem.alloc = [](void *self, size_t n) -> void * { return ((Arena *)self)->alloc(n); };
    dev.mem.free = [](void *self, void *p) { ((Arena *)self)->release(p); };
    dev.mem.self = &Q.arena;

    size_t next = 0;
    long long rejected = 0, completed = 0, steps = 0;
    std::map<uint64_t, int> seen;  // tag -> times finished
    std::vector<double> admit_order;
    std::map<uint64_t, double> t_admit;
    double max_stall = 0, prev_busy = 0, prev_slot = 0, prev_now = dev.now, prev_cap = 0;
    const double t_first = dev.now;
    for (;;) {
        while (next < subs.size() && subs[next].t <= dev.now) {
            const Sub &s = subs[next];
            if (Q.standalone_bytes(s.G, s.P) > Q.arena.size) {
                rejected++;
            } else {
                Req *R = new Req();
                R->tag = next;
                R->G = s.G;
                R->P = s.P;
                Q.submit(R, dev.now);
            }
            next++;
        }
        const SchedStep r = Q.step(dev.now);
        steps++;
        // invariants
        if (Q.arena.used > Q.arena.size) fail("arena over its size%s", "");
        for (auto &kv : Q.batches) {
            const auto *br = kv.second;
            if (!dev.live.count(br->b)) fail("scheduler holds a destroyed batch%s", "");
            if (br->G != kv.first.first || (int)br->kind != kv.first.second) fail("batch under the wrong key%s", "");
        }
        if (dev.live.size() != Q.batches.size()) fail("a batch was leaked%s", "");
        std::vector<Req *> done;
        Q.take_finished(done, 1 << 30);
        for (Req *R : done) {
            if (seen[R->tag]++) fail("request %s%lld finished twice", "", (long long)R->tag);
            completed++;
            // a failure is legitimate when it was injected on the request's
            // path: at its set-up or finalization, in a batch that held or
            // queued one of its jobs (the job carries the error), or in the
            // creation of its batch at its admission
            bool job_failed = false;
            for (const Job &j : R->hp) job_failed |= j.status != TM_OK;
            for (const Job &j : R->lp) job_failed |= j.status != TM_OK;
            const bool injected = dev.failed_reqs.count(R) > 0 || (job_failed && dev.injected > 0) ||
                                  (R->hp.empty() && R->lp.empty() && dev.create_fail_t.count(R->t_done) > 0);
            if (R->status == TM_OK) {
                if (R->res.size() != (size_t)TM_N_OPS * R->lt * 4 || R->res[0] != (double)R->tag ||
                    R->res[1] != (double)(R->hp.size() + R->lp.size()))
                    fail("request %s%lld has wrong results", "", (long long)R->tag);
                if (!(R->t_submit <= R->t_admit && R->t_admit <= R->t_done)) fail("request %s%lld times out of order", "",
                                                                                 (long long)R->tag);
                if (job_failed) fail("OK request with a failed job%s", "");
            } else if (!injected) {
                fail("request %s%lld failed (status %lld) with no failure injected on its path", "", (long long)R->tag,
                     R->status);
            }
            if (R->t_admit > 0) t_admit[R->tag] = R->t_admit;
            delete R;
        }
        {
            std::lock_guard<std::mutex> lk(Q.mu);
            max_stall = std::max(max_stall, Q.snap.stall_s);
            // utilisation integrals: non-decreasing, busy time within the
            // elapsed time, and since the last step at most the slots of the
            // batches resident then, for the time since then
            const tm_serve_status &ss = Q.snap;
            if (ss.busy_s < prev_busy || ss.slot_s < prev_slot) fail("utilisation integrals decreased%s", "");
            if (ss.busy_s > dev.now - t_first + 1e-9) fail("busy time beyond the elapsed time%s", "");
            if (ss.slot_s - prev_slot > (dev.now - prev_now) * prev_cap * (1 + 1e-12) + 1e-9)
                fail("slot-seconds beyond the slots of the batches%s", "");
            prev_busy = ss.busy_s;
            prev_slot = ss.slot_s;
            prev_now = dev.now;
            prev_cap = (double)sc.slots * (double)Q.batches.size();
        }
        if (g_fail) {
            dump(Q, dev);
            return 0;
        }
        if (next == subs.size() && completed + rejected == (long long)subs.size()) break;
        if (r.progressed) continue;
        // nothing changed: the next event is an arrival, a chunk or a finalization
        double tn = 1e300;
        if (next < subs.size()) tn = std::min(tn, subs[next].t);
        for (auto *B : dev.live)
            if (B->in_flight) tn = std::min(tn, B->t_done);
        for (Req *R : Q.active)
            if (R->state == RQ_FINALIZING) tn = std::min(tn, R->dev.t_fin);
        if (tn >= 1e299) {
            fail("stuck: no progress and no pending event with %s%lld requests outstanding", "",
                 (long long)(subs.size() - completed - rejected));
            dump(Q, dev);
            return 0;
        }
        if (tn <= dev.now && !r.busy) {
            fail("stuck: an event is due but the step made no progress%s", "");
            dump(Q, dev);
            return 0;
        }
        dev.now = std::max(dev.now, tn);
        if (steps > 50000000) {
            fail("too many steps%s", "");
            dump(Q, dev);
            return 0;
        }
    }
    // FIFO: admission times follow submission order
    double last = -1;
    for (auto &kv : t_admit) {
        if (kv.second + 1e-12 < last) fail("request %s%lld admitted before an earlier one", "", (long long)kv.first);
        last = std::max(last, kv.second);
    }
    if (Q.arena.used != 0 && !Q.batches.empty()) {
        // idle batches may stay; every request buffer must be released
        size_t b = 0;
        for (auto &kv : Q.batches) b += dev.batch_bytes(kv.second->G, kv.second->kind);
        if (Q.arena.used > b + 256 * Q.batches.size()) fail("request buffers leaked in the arena%s", "");
    }
    Q.shutdown();
    if (Q.arena.used != 0) fail("arena not empty after shutdown%s", "");
    std::printf("seed %" PRIu64 ": %d requests (%lld rejected), slots %d, budget %.1fx, load %.2f, failures %s "
                "(%lld injected): %lld steps, virtual %.2f s, max stall %.4f s\n",
                seed, sc.n_req, rejected, sc.slots, sc.budget_factor, sc.load, sc.failures ? "on" : "off",
                dev.injected, steps, dev.now, max_stall);
    return g_fail ? 0 : completed;
}

}  // namespace

int main(int argc, char **argv)
{
    const uint64_t seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
    const int n = argc > 2 ? std::atoi(argv[2]) : 20;
    std::mt19937_64 rng(seed);
    for (int i = 0; i < n; i++) {
        Scenario sc;
        sc.n_req = 20 + (int)(rng() % 181);
        const double bf[] = {1.0, 1.05, 1.5, 2.2, 4.0};
        sc.budget_factor = bf[rng() % 5];
        const double ld[] = {0.5, 0.8, 0.95, 1.5, 4.0};
        sc.load = ld[rng() % 5];
        sc.failures = (i % 2) == 1;
        const int sl[] = {1, 4, 12, 16};
        sc.slots = sl[rng() % 4];
        if (!run(seed * 1000 + i, sc)) {
            std::fprintf(stderr, "scenario %d of seed %" PRIu64 " failed\n", i, seed);
            return 1;
        }
    }
    return 0;
}
