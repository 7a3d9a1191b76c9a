// Slot engine: S independent CG solves on one gauge field share every
// multi-RHS launch.  Each slot follows the even-odd normal-equation CG of
// its own right-hand side; slots finish, are harvested (reconstruction of
// the odd sites, contractions) and refilled independently between chunks
// of iterations.  Per-slot arithmetic never depends on the other slots, so a
// solve gives the same bits alone and inside any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "tm_internal.h"

using namespace tmk;

namespace tmi {

Kind kind_of(const tm_solver_params &p) { return kind_of_mode(p.mode, p.half_prec); }

int kind_prec(Kind k)
{
    switch (k) {
    case K_F64: return P64;
    case K_MIXED: return P32;
    case K_LP16: return P16;
    case K_LPBF: return PBF;
    }
    return P64;
}

static int kind_xr(Kind k) { return kind_prec(k); }  // x, r stored like the Dslash operands

// Pitch between the slots of a multi-slot field: the field plus 17 x 256
// bytes, so the same site of consecutive slots (at power-of-two-sized
// distances otherwise) does not land on one memory channel.
static size_t slot_pitch(size_t field) { return ((field + 255) & ~(size_t)255) + 17 * 256; }

static bool lp_kind(Kind k) { return k == K_LP16 || k == K_LPBF; }

// longest run of slots prepared / harvested / updated together
// (TM_FILL_RUN, TM_HARVEST_RUN, TM_UPDATE_RUN cap it; 1 = slot by slot)
static int run_cap(const char *name)
{
    const char *e = getenv(name);
    return e ? std::max(1, atoi(e)) : MAX_SLOTS;
}

// Preparation / reconstruction precision of the kind's noise solves (LP: FP32).
static int kind_prep(Kind k) { return lp_kind(k) ? P32 : P64; }

// Each scratch array holds an FP64 full field [even | odd], or one
// preparation-precision half field per slot (runs of slots prepared and
// harvested together).
static size_t scratch_bytes(const Geom &g, Kind kind, int S)
{
    return std::max(2 * half_bytes(P64, g), (size_t)S * slot_pitch(half_bytes(kind_prep(kind), g)));
}

size_t batch_footprint(const tm_gauge *G, Kind kind, int S)
{
    const Geom &g = G->g;
    const int sp = kind_prec(kind), xr = kind_xr(kind);
    size_t b = 0;
    b += (size_t)S * 3 * slot_pitch(half_bytes(sp, g));  // p, u, t
    b += (size_t)S * 2 * slot_pitch(half_bytes(xr, g));  // x, r
    if (kind == K_MIXED) b += (size_t)S * 2 * half_bytes(P64, g);  // x64, b64
    b += (size_t)S * 2 * g.vh * sizeof(uint32_t);      // noise codes
    b += (lp_kind(kind) ? 4 : 3) * (scratch_bytes(g, kind, S) + 256);  // scratch FA, FB, FC (, FD)
    b += (size_t)S * ntile_of(g) * sizeof(double) + 4096;
    b += (size_t)(lp_kind(kind) ? S : 1) * contract_part_doubles(g) * sizeof(double) + 256;
    b += (size_t)S * sizeof(SlotState) + 64 * sizeof(double) + 16 * 256;
    return b;
}

int auto_chunk(const tm_gauge *G, Kind k, int S)
{
    // aim at a few milliseconds of device work between host checks
    const int sp = kind_prec(k);
    const double lb = sp == P64 ? 96 : sp == P32 ? 48 : 36, sb = sp == P64 ? 192 : sp == P32 ? 96 : 52;
    const double bytes_it = (double)G->g.vh * S * (32.0 * lb / 4.0 + 20.0 * sb);
    const double secs = bytes_it / 4.0e12 + 8 * 3e-6;
    int c = (int)(3e-3 / secs);
    return std::max(4, std::min(64, c));
}

static char *carve(char *&cur, size_t bytes)
{
    char *p = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return p;
}

int batch_create(tm_context *ctx, const tm_gauge *G, Kind kind, int S, int chunk, hipStream_t stream, Batch **out,
                 const Mem *mem)
{
    if (S < 1 || S > MAX_SLOTS) return set_err(ctx, TM_ERR_ARG, "batch size %d outside 1..%d", S, MAX_SLOTS);
    const int sp = kind_prec(kind);
    if (!(G->precs & (1u << sp)))
        return set_err(ctx, TM_ERR_ARG, "gauge field was not loaded in the precision this solver needs");
    if ((kind == K_LP16 || kind == K_LPBF) && !(G->precs & (1u << P32)))
        return set_err(ctx, TM_ERR_ARG, "low-precision solves also need the FP32 links (preparation)");
    Batch *b = new Batch();
    b->ctx = ctx;
    b->G = G;
    b->kind = kind;
    b->sp = sp;
    b->xr = kind_xr(kind);
    b->S = S;
    const Geom &g = G->g;
    b->hsp = slot_pitch(half_bytes(sp, g));
    b->hxr = slot_pitch(half_bytes(b->xr, g));
    b->h64 = half_bytes(P64, g);
    b->nblk = ntile_of(g);  // per-slot partial sums (64-site tiles)
    b->bytes = batch_footprint(G, kind, S) + 32 * 256;
    if (mem) b->mem = *mem;
    char *base = (char *)(b->mem.alloc ? b->mem.alloc(b->mem.self, b->bytes) : dalloc(ctx, b->bytes));
    if (!base) {
        delete b;
        return set_err(ctx, TM_ERR_NOMEM, "cannot allocate %zu bytes of solver workspace", (size_t)batch_footprint(G, kind, S));
    }
    char *cur = base;
    b->p = carve(cur, S * b->hsp);
    b->u = carve(cur, S * b->hsp);
    b->t = carve(cur, S * b->hsp);
    b->x = carve(cur, S * b->hxr);
    b->r = carve(cur, S * b->hxr);
    if (kind == K_MIXED) {
        b->x64 = carve(cur, S * b->h64);
        b->b64 = carve(cur, S * b->h64);
    }
    b->codes = (uint32_t *)carve(cur, (size_t)S * 2 * g.vh * sizeof(uint32_t));
    const size_t sb = scratch_bytes(g, kind, S);
    b->wpp = kind_prep(kind);
    b->wpitch = slot_pitch(half_bytes(b->wpp, g));
    b->wslots = (int)std::min<size_t>(S, sb / b->wpitch);
    b->FA = carve(cur, sb);
    b->FB = carve(cur, sb);
    b->FC = carve(cur, sb);
    if (lp_kind(kind)) b->FD = carve(cur, sb);
    b->partial = (double *)carve(cur, (size_t)S * b->nblk * sizeof(double) + 4096);
    b->cpart = (double *)carve(cur, (size_t)(lp_kind(kind) ? S : 1) * contract_part_doubles(g) * sizeof(double));
    b->dres = (double *)carve(cur, 64 * sizeof(double));
    b->st = (SlotState *)carve(cur, (size_t)S * sizeof(SlotState));
    b->stream = stream;
    b->slot_job.assign(S, nullptr);
    b->slot_updates.assign(S, 0);
    b->slot_pending_update.assign(S, 0);
    b->chunk = chunk > 0 ? chunk : auto_chunk(G, kind, S);
    hipError_t e = hipHostMalloc((void **)&b->st_h, (size_t)S * sizeof(SlotState), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->hres, 64 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_destroy(b);
        return set_err(ctx, TM_ERR_HIP, "batch setup failed: %s", hipGetErrorString(e));
    }
    // all slots empty
    std::vector<SlotState> init(S);
    for (auto &s : init) {
        std::memset(&s, 0, sizeof(s));
        s.status = ST_EMPTY;
    }
    std::memcpy(b->st_h, init.data(), S * sizeof(SlotState));
    e = hipMemcpyAsync(b->st, b->st_h, S * sizeof(SlotState), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        batch_destroy(b);
        return set_err(ctx, TM_ERR_HIP, "batch init failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return TM_OK;
}

void batch_destroy(Batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->st_h) (void)hipHostFree(b->st_h);
    if (b->hres) (void)hipHostFree(b->hres);
    if (b->p) {
        if (b->mem.free)
            b->mem.free(b->mem.self, b->p);
        else
            dfree(b->ctx, b->p);
    }
    delete b;
}

int batch_active(const Batch *b)
{
    int n = 0;
    for (auto *j : b->slot_job) n += j != nullptr;
    return n;
}

int batch_free_slot(const Batch *b)
{
    for (int s = 0; s < b->S; s++)
        if (!b->slot_job[s]) return s;
    return -1;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static DslashArgs dargs(const Batch *b, int sp)
{
    DslashArgs A;
    std::memset(&A, 0, sizeof(A));
    A.g = b->G->g;
    A.gauge = b->G->links[sp];
    A.nslot = 1;
    A.swz = b->ctx->swz;
    return A;
}

// one FP64 single-slot Dslash with uniform (kappa, a)
static void d64(const Batch *b, bool dag, int epi, int coef, int out_par, const char *in, const char *in2, char *out,
                double kappa, double a, double *partial = nullptr, const char *bvec = nullptr)
{
    DslashArgs A = dargs(b, P64);
    A.in = in;
    A.in2 = in2;
    A.out = out;
    A.out_par = out_par;
    A.coef = coef;
    A.kappa_u = kappa;
    A.a_u = a;
    A.partial = partial;
    A.b = bvec;
    launch_dslash(P64, dag, epi, in2 != nullptr, A, b->stream);
}

// eta of a job into FA = [even | odd] (FP64)
static void load_eta(Batch *b, int slot, Job *j)
{
    const Geom &g = b->G->g;
    uint32_t *codes = b->codes + (size_t)slot * 2 * g.vh;
    if (j->noise) {
        launch_z4_field(g, codes, 0, 0.0, b->FA, b->stream);
        launch_z4_field(g, codes + g.vh, 0, 0.0, b->FA + b->h64, b->stream);
    } else {
        launch_field_import(P64, g, 1, j->b_canon, b->FA, b->stream);
    }
}

// Prep/reconstruction precision class of a job: P32 for LP noise solves
// (their target is a 1e-2 residual: reconstruction and contraction in FP32,
// the preparation in the solve's half precision, see fill_noise_run),
// P64 for everything else.
static int prep_prec(const Batch *b, const Job *j)
{
    return (j->noise && !j->want_true && (b->kind == K_LP16 || b->kind == K_LPBF)) ? P32 : P64;
}

// Dslash with uniform (kappa, a) in precision pp on single fields
static void dsl(const Batch *b, int pp, bool dag, int epi, int coef, int out_par, const char *in, const char *in2,
                char *out, double kappa, double a, double *partial = nullptr)
{
    DslashArgs A = dargs(b, pp);
    A.in = in;
    A.in2 = in2;
    A.out = out;
    A.out_par = out_par;
    A.coef = coef;
    A.kappa_u = kappa;
    A.a_u = a;
    A.partial = partial;
    launch_dslash(pp, dag, epi, in2 != nullptr, A, b->stream);
}

// Dslash whose noise input comes from the slot's Z4 codes (src 3: prep, src 2: reconstruction)
static void dsl_codes(const Batch *b, int pp, int src, int coef, int out_par, int slot, const char *in, char *out,
                      double kappa, double a)
{
    DslashArgs A = dargs(b, pp);
    A.codes = b->codes + (size_t)slot * 2 * b->G->g.vh;
    A.in = in;
    A.out = out;
    A.out_par = out_par;
    A.coef = coef;
    A.kappa_u = kappa;
    A.a_u = a;
    launch_dslash_codes(pp, src, A, b->stream);
}

// Dslash with uniform (kappa, a) over n consecutive slots with the given pitches
static void dsl_run(const Batch *b, int pp, bool dag, int epi, int coef, int out_par, const char *in, size_t in_slot,
                    const char *in2, size_t in2_slot, char *out, size_t out_slot, double kappa, double a, int n,
                    double *partial = nullptr, const char *bvec = nullptr, size_t b_slot = 0)
{
    DslashArgs A = dargs(b, pp);
    A.nslot = n;
    A.in = in;
    A.in_slot = in_slot;
    A.in2 = in2;
    A.in2_slot = in2_slot;
    A.out = out;
    A.out_slot = out_slot;
    A.out_par = out_par;
    A.coef = coef;
    A.kappa_u = kappa;
    A.a_u = a;
    A.partial = partial;
    A.b = bvec;
    A.b_slot = b_slot;
    launch_dslash(pp, dag, epi, in2 != nullptr, A, b->stream);
}

// dsl_codes over the n consecutive slots from s0
static void dsl_codes_run(const Batch *b, int pp, int src, int coef, int out_par, int s0, int n, const char *in,
                          size_t in_slot, char *out, size_t out_slot, double kappa, double a)
{
    DslashArgs A = dargs(b, pp);
    A.nslot = n;
    A.codes = b->codes + (size_t)s0 * 2 * b->G->g.vh;
    A.codes_slot = (size_t)2 * b->G->g.vh * sizeof(uint32_t);
    A.in = in;
    A.in_slot = in_slot;
    A.out = out;
    A.out_slot = out_slot;
    A.out_par = out_par;
    A.coef = coef;
    A.kappa_u = kappa;
    A.a_u = a;
    launch_dslash_codes(pp, src, A, b->stream);
}

static void job_start(Batch *b, int slot, Job *j)
{
    b->slot_job[slot] = j;
    b->slot_updates[slot] = 0;
    b->slot_pending_update[slot] = 0;
    j->t_fill = now_s();
    if (b->t_first == 0) b->t_first = j->t_fill;
}

// Noise solves in the n consecutive slots from s0, equal (kappa, a) and
// precision class pp (prep_prec), prepared together (FP64 for pp = P64,
// else in the batch's half precision):
//   bhat_e = eta_e + kappa D_eo A^-1 eta_o straight from the Z4 codes,
//   rhs = Mhat^dag bhat = A^dag bhat - kappa^2 D'_eo A^-dag D'_oe bhat,
// r = p = rhs (rounded to the CG precisions), x = 0.
static void fill_noise_run(Batch *b, int s0, int n, Job *const *jobs, int pp)
{
    const Geom &g = b->G->g;
    hipStream_t s = b->stream;
    const bool mixed = b->kind == K_MIXED;
    const double kappa = jobs[0]->kappa, a = jobs[0]->a;
    Z4Sources Z{};
    SlotStartParams P{};
    P.mixed = mixed ? 1 : 0;
    for (int i = 0; i < n; i++) {
        Job *j = jobs[i];
        job_start(b, s0 + i, j);
        Z.seed[i] = j->seed;
        Z.src[i] = j->src;
        Z.tmod[i] = j->tmod;
        Z.tph[i] = j->tph;
        P.kappa[i] = j->kappa;
        P.a[i] = j->a;
        P.tol2[i] = j->fixed > 0 ? 0.0 : j->tol * j->tol;
        P.max_iter[i] = j->fixed > 0 ? j->fixed : j->max_iter;
        const double delta = j->delta > 0 ? j->delta : TM_DEFAULT_DELTA;
        P.delta2[i] = delta * delta;
    }
    launch_z4_codes(g, Z, n, b->codes + (size_t)s0 * 2 * g.vh, s);
    // LP runs prepare their right-hand side in the solve's own half precision
    // (FP32 arithmetic): bhat and A^-dag D bhat stored like the CG vectors
    const bool half = !mixed && pp == P32 && b->xr == b->sp && b->hxr == b->hsp && (b->xr == P16 || b->xr == PBF);
    const int pq = half ? b->sp : pp;
    const size_t w = n > 1 ? b->wpitch : half_bytes(pq, g);
    char *Be = b->FB, *To = b->FC, *Ce = b->FA;
    double *part = b->partial + (size_t)s0 * b->nblk;
    dsl_codes_run(b, pq, 3, CM_PREP, 0, s0, n, nullptr, 0, Be, w, kappa, a);
    dsl_run(b, pq, true, EPI_PLAIN, CM_AINV_DAG, 1, Be, w, nullptr, 0, To, w, kappa, a, n);
    // LP runs: the last preparation Dslash writes r = p = rhs and x = 0 in
    // half precision itself (same bits as the rhs converted after it)
    bool fused = false;
    if (half) {
        DslashArgs A = dargs(b, pq);
        A.nslot = n;
        A.in = To;
        A.in_slot = w;
        A.in2 = Be;
        A.in2_slot = w;
        A.out = b->p + s0 * b->hsp;
        A.out_slot = b->hsp;
        A.r = b->r + s0 * b->hxr;
        A.x = b->x + s0 * b->hxr;
        A.xr_slot = b->hxr;
        A.out_par = 0;
        A.coef = CM_MHAT_DAG;
        A.kappa_u = kappa;
        A.a_u = a;
        A.partial = part;
        fused = launch_dslash_start(pq, b->xr, A, s) == 0;
    }
    if (!fused) dsl_run(b, pq, true, EPI_NORM, CM_MHAT_DAG, 0, To, w, Be, w, Ce, w, kappa, a, n, part);
    launch_slot_start(b->st + s0, part, b->nblk, P, n, s);
    if (!fused) {
        if (b->xr == b->sp && b->hxr == b->hsp && (pq == P64 || pq == P32)) {
            launch_cg_start(pq, b->xr, g, Ce, w, b->r + s0 * b->hxr, b->p + s0 * b->hsp, b->x + s0 * b->hxr, b->hxr,
                            n, s);
        } else {
            launch_convert(pq, b->xr, g, Ce, w, b->r + s0 * b->hxr, b->hxr, n, s);
            launch_convert(pq, b->sp, g, Ce, w, b->p + s0 * b->hsp, b->hsp, n, s);
            launch_zero(b->xr, g, b->x + s0 * b->hxr, b->hxr, n, s);
        }
    }
    if (mixed) {
        launch_convert(P64, P64, g, Ce, w, b->b64 + s0 * b->h64, b->h64, n, s);
        launch_zero(P64, g, b->x64 + s0 * b->h64, b->h64, n, s);
    }
}

int batch_fill_many(Batch *b, Job *const *jobs, int njobs)
{
    std::vector<int> fs;
    for (int s = 0; s < b->S && (int)fs.size() < njobs; s++)
        if (!b->slot_job[s]) fs.push_back(s);
    const int m = (int)fs.size();
    int k = 0;
    while (k < m) {
        Job *j = jobs[k];
        if (!j->noise) {
            batch_fill(b, fs[k], j);
            k++;
            continue;
        }
        const int pp = prep_prec(b, j);
        static const int cap_env = run_cap("TM_FILL_RUN");
        const int cap = pp == b->wpp ? std::min(b->wslots, cap_env) : 1;
        int n = 1;
        while (k + n < m && n < cap && fs[k + n] == fs[k] + n && jobs[k + n]->noise &&
               jobs[k + n]->kappa == j->kappa && jobs[k + n]->a == j->a && prep_prec(b, jobs[k + n]) == pp)
            n++;
        fill_noise_run(b, fs[k], n, jobs + k, pp);
        k += n;
    }
    return m;
}

int batch_fill(Batch *b, int slot, Job *j)
{
    if (j->noise) {
        fill_noise_run(b, slot, 1, &j, prep_prec(b, j));
        return TM_OK;
    }
    const Geom &g = b->G->g;
    hipStream_t s = b->stream;
    job_start(b, slot, j);
    const bool mixed = b->kind == K_MIXED;
    const double tol2 = j->fixed > 0 ? 0.0 : j->tol * j->tol;
    const int maxit = j->fixed > 0 ? j->fixed : j->max_iter;
    const double delta = j->delta > 0 ? j->delta : TM_DEFAULT_DELTA;
    double *part = b->partial + (size_t)slot * b->nblk;
    load_eta(b, slot, j);
    char *Ee = b->FA, *Eo = b->FA + b->h64;
    char *Be = b->FB, *Bo = b->FB + b->h64;
    char *Ce = b->FC;
    // bhat_e = eta_e + kappa D_eo A^-1 eta_o
    launch_site_diag(g, 1, j->a, Eo, Bo, s);
    d64(b, false, EPI_PLAIN, CM_PREP, 0, Bo, Ee, Be, j->kappa, j->a);
    // rhs = Mhat^dag bhat = A^dag bhat - kappa^2 D'_eo A^-dag D'_oe bhat
    d64(b, true, EPI_PLAIN, CM_AINV_DAG, 1, Be, nullptr, Bo, j->kappa, j->a);
    d64(b, true, EPI_NORM, CM_MHAT_DAG, 0, Bo, Be, Ce, j->kappa, j->a, part);
    launch_slot_start(b->st + slot, part, b->nblk, j->kappa, j->a, tol2, maxit, delta * delta, mixed ? 1 : 0, s);
    launch_convert(P64, b->xr, g, Ce, 0, b->r + slot * b->hxr, 0, 1, s);
    launch_convert(P64, b->sp, g, Ce, 0, b->p + slot * b->hsp, 0, 1, s);
    launch_zero(b->xr, g, b->x + slot * b->hxr, 0, 1, s);
    if (mixed) {
        launch_convert(P64, P64, g, Ce, 0, b->b64 + slot * b->h64, 0, 1, s);
        launch_zero(P64, g, b->x64 + slot * b->h64, 0, 1, s);
    }
    return TM_OK;
}

// One CG iteration for every running slot:
//   t = A^-1 D_oe p;  u = A p - k^2 D_eo t (= Mhat p), |u|^2;  alpha = rr/|u|^2
//   t = A^-dag D'_oe u;  Ap = A^dag u - k^2 D'_eo t (= Mhat^dag u);
//   x += alpha p; r -= alpha Ap; |r|^2;  beta;  p = r + beta p
static void enqueue_iteration(Batch *b)
{
    const int sp = b->sp;
    DslashArgs A = dargs(b, sp);
    A.nslot = b->S;
    A.st = b->st;
    A.partial = b->partial;
    A.in_slot = A.in2_slot = A.out_slot = b->hsp;
    // D1
    A.in = b->p;
    A.in2 = nullptr;
    A.out = b->t;
    A.out_par = 1;
    A.coef = CM_AINV;
    launch_dslash(sp, false, EPI_PLAIN, false, A, b->stream);
    // D2
    A.in = b->t;
    A.in2 = b->p;
    A.out = b->u;
    A.out_par = 0;
    A.coef = CM_MHAT;
    launch_dslash(sp, false, EPI_NORM, true, A, b->stream);
    launch_cg_alpha(b->st, b->partial, b->S, b->nblk, b->stream);
    // D3
    A.in = b->u;
    A.in2 = nullptr;
    A.out = b->t;
    A.out_par = 1;
    A.coef = CM_AINV_DAG;
    launch_dslash(sp, true, EPI_PLAIN, false, A, b->stream);
    // D4 with the CG update
    A.in = b->t;
    A.in2 = b->u;
    A.out = nullptr;
    A.out_par = 0;
    A.coef = CM_MHAT_DAG;
    A.r = b->r;
    A.xr_slot = b->hxr;
    launch_dslash(sp, true, EPI_CGUPD, true, A, b->stream);
    launch_cg_beta(b->st, b->partial, b->S, b->nblk, b->stream);
    // x += alpha p (for every slot that stepped) and p = r + beta p
    launch_p_update(sp, b->xr, b->G->g, b->p, b->hsp, b->r, b->hxr, b->x, b->hxr, b->st, b->S, b->ctx->swz,
                    b->stream);
}

int batch_launch_chunk(Batch *b)
{
    hipStream_t s = b->stream;
    if (b->ctx->use_graphs) {
        if (!b->gexec || b->g_iters != b->chunk) {
            if (b->gexec) {
                (void)hipGraphExecDestroy(b->gexec);
                b->gexec = nullptr;
            }
            if (b->graph) {
                (void)hipGraphDestroy(b->graph);
                b->graph = nullptr;
            }
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (int i = 0; i < b->chunk; i++) enqueue_iteration(b);
                e = hipStreamEndCapture(s, &b->graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                // fall back to direct launches for this batch
                (void)hipGetLastError();
                b->ctx->use_graphs = 0;
                if (b->graph) (void)hipGraphDestroy(b->graph);
                b->graph = nullptr;
                b->gexec = nullptr;
            } else {
                b->g_iters = b->chunk;
            }
        }
    }
    if (b->gexec) {
        TM_HIP(b->ctx, hipGraphLaunch(b->gexec, s));
    } else {
        for (int i = 0; i < b->chunk; i++) enqueue_iteration(b);
    }
    TM_HIP(b->ctx, hipMemcpyAsync(b->st_h, b->st, b->S * sizeof(SlotState), hipMemcpyDeviceToHost, s));
    TM_HIP(b->ctx, hipEventRecord(b->ev, s));
    b->in_flight = true;
    return TM_OK;
}

// FP64 reliable updates of the n consecutive mixed-precision slots from s0
// (equal kappa, a): x64 += x32, r = b - Mhat^dag Mhat x64 in FP64, r32 = r,
// then each CG direction continues with beta = |r|^2/|r_old|^2.
static void reliable_update_run(Batch *b, int s0, int n)
{
    const Geom &g = b->G->g;
    const Job *j = b->slot_job[s0];
    hipStream_t s = b->stream;
    const size_t w = n > 1 ? b->wpitch : b->h64;
    char *x64 = b->x64 + s0 * b->h64;
    char *x32 = b->x + s0 * b->hxr, *r32 = b->r + s0 * b->hxr;
    char *Bo = b->FB, *Be = b->FA, *Ce = b->FC;
    double *part = b->partial + (size_t)s0 * b->nblk;
    launch_accum_x(g, x64, b->h64, x32, x32, b->hxr, n, s);
    dsl_run(b, P64, false, EPI_PLAIN, CM_AINV, 1, x64, b->h64, nullptr, 0, Bo, w, j->kappa, j->a, n);
    dsl_run(b, P64, false, EPI_PLAIN, CM_MHAT, 0, Bo, w, x64, b->h64, Be, w, j->kappa, j->a, n);
    dsl_run(b, P64, true, EPI_PLAIN, CM_AINV_DAG, 1, Be, w, nullptr, 0, Bo, w, j->kappa, j->a, n);
    dsl_run(b, P64, true, EPI_RESID, CM_MHAT_DAG, 0, Bo, w, Be, w, Ce, w, j->kappa, j->a, n, part,
            b->b64 + s0 * b->h64, b->h64);
    launch_convert(P64, b->xr, g, Ce, w, r32, b->hxr, n, s);
    launch_reliable_finish(b->st + s0, part, b->nblk, n, s);
    launch_p_update(b->sp, b->xr, g, b->p + s0 * b->hsp, b->hsp, r32, b->hxr, nullptr, 0, b->st + s0, n, b->ctx->swz,
                    s);
    for (int i = 0; i < n; i++) b->slot_updates[s0 + i]++;
}

static void harvest64(Batch *b, int slot, const SlotState &S, Job *j);
static int true_residual(Batch *b, int slot, Job *j);

// LP noise solves in the n consecutive slots from s0 (equal kappa, a):
// s_e = x widened to FP32, s_o = A^-1 (eta_o + kappa D_oe s_e) from the codes,
// contractions on FP32 s and FP32 links with FP64 sums.
static void harvest_lp_run(Batch *b, int s0, int n)
{
    const Geom &g = b->G->g;
    const Job *j = b->slot_job[s0];
    hipStream_t s = b->stream;
    const size_t w = n > 1 ? b->wpitch : half_bytes(P32, g);
    char *se32 = b->FB, *so32 = b->FC;
    launch_convert(b->xr, P32, g, b->x + s0 * b->hxr, b->hxr, se32, w, n, s);
    dsl_codes_run(b, P32, 2, CM_RECON, 1, s0, n, se32, w, so32, w, j->kappa, j->a);
    RawOuts R{}, R2{};
    for (int i = 0; i < n; i++) {
        R.p[i] = b->slot_job[s0 + i]->raw_out;
        R2.p[i] = b->slot_job[s0 + i]->raw_out2;
    }
    if (j->oet) {
        // one-end trick: isovector -2ia s^dag g5 X s, isoscalar 2 s^dag g5 X g5 D_W s with
        // D_W s = (s_e - kappa D_eo s_o, s_o - kappa D_oe s_e)
        char *re = b->FA, *ro = b->FD;
        dsl_run(b, P32, false, EPI_PLAIN, CM_M, 0, so32, w, se32, w, re, w, j->kappa, 0.0, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_M, 1, se32, w, so32, w, ro, w, j->kappa, 0.0, n);
        launch_contract_lr(P32, g, b->G->links[P32], se32, so32, w, se32, so32, w, b->cpart, R, n, 0.0, -2.0 * j->a,
                           s, j->local_only);
        launch_contract_lr(P32, g, b->G->links[P32], re, ro, w, se32, so32, w, b->cpart, R2, n, 2.0, 0.0, s,
                           j->local_only);
        return;
    }
    const uint32_t *codes = b->codes + (size_t)s0 * 2 * g.vh;
    if (j->local_only) launch_contract_local(P32, g, se32, so32, w, codes, b->cpart, R, n, s);
    else launch_contract(P32, g, b->G->links[P32], se32, so32, w, codes, b->cpart, R, n, s);
    if (j->hpe) {
        // (BH)^4 s: even part ((BH)_eo (BH)_oe)^2 s_e via FA (odd) into FD,
        // odd part ((BH)_oe (BH)_eo)^2 s_o via FA (even) into FB
        char *ta = b->FA, *we = b->FD, *wo = b->FB;
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 1, se32, w, nullptr, 0, ta, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 0, ta, w, nullptr, 0, we, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 1, we, w, nullptr, 0, ta, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 0, ta, w, nullptr, 0, we, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 0, so32, w, nullptr, 0, ta, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 1, ta, w, nullptr, 0, wo, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 0, wo, w, nullptr, 0, ta, w, j->kappa, j->a, n);
        dsl_run(b, P32, false, EPI_PLAIN, CM_BH, 1, ta, w, nullptr, 0, wo, w, j->kappa, j->a, n);
        launch_contract_local(P32, g, we, wo, w, codes, b->cpart, R2, n, s);
    }
}

// results of a finished slot: status, counts, optional true residual; frees the slot
static int harvest_done(Batch *b, int slot, const SlotState &S)
{
    Job *j = b->slot_job[slot];
    j->iters = S.iter;
    j->end = S;
    j->updates = b->slot_updates[slot];
    j->cg_rel = S.rr0 > 0 ? std::sqrt(std::max(S.status == ST_CONVERGED || S.status == ST_MAXITER ? S.rr : S.rr_new, 0.0) / S.rr0) : 0.0;
    j->status = S.status == ST_CONVERGED ? TM_OK
                : S.status == ST_MAXITER ? (j->fixed > 0 ? TM_OK : TM_ERR_NOCONV)
                                         : TM_ERR_NUMERIC;
    if (j->want_true) {
        int e = true_residual(b, slot, j);
        if (e != TM_OK) return e;
    }
    b->iters_done += S.iter;
    j->t_done = now_s();
    b->t_last = j->t_done;
    b->slot_job[slot] = nullptr;
    return TM_OK;
}

// LP noise solves harvested in FP32 (their contraction needs a raw output)
static bool lp_harvest(const Batch *b, const Job *j) { return prep_prec(b, j) == P32 && j->raw_out; }

// reconstruct s = (s_e, s_o), contract or export, optional true residual
static int harvest(Batch *b, int slot, const SlotState &S)
{
    Job *j = b->slot_job[slot];
    if (lp_harvest(b, j)) harvest_lp_run(b, slot, 1);
    else if (prep_prec(b, j) != P32) harvest64(b, slot, S, j);
    return harvest_done(b, slot, S);
}

// FP64 reconstruction and contraction / export
static void harvest64(Batch *b, int slot, const SlotState &S, Job *j)
{
    const Geom &g = b->G->g;
    hipStream_t s = b->stream;
    // s_e (FP64) into FC even half
    char *se = b->FC, *so = b->FC + b->h64;
    if (b->kind == K_F64) {
        launch_convert(P64, P64, g, b->x + slot * b->hxr, 0, se, 0, 1, s);
    } else if (b->kind == K_MIXED) {
        char *x64 = b->x64 + slot * b->h64;
        if (S.status != ST_CONVERGED) launch_accum_x(g, x64, 0, b->x + slot * b->hxr, nullptr, 0, 1, s);
        launch_convert(P64, P64, g, x64, 0, se, 0, 1, s);
    } else {
        launch_convert(b->xr, P64, g, b->x + slot * b->hxr, 0, se, 0, 1, s);
    }
    char *Eo = b->FA + b->h64;
    if (j->noise) {
        // s_o = A^-1 (eta_o + kappa D_oe s_e) with eta_o from the codes
        dsl_codes(b, P64, 2, CM_RECON, 1, slot, se, so, j->kappa, j->a);
        if (j->raw_out && j->oet) {
            // one-end trick (see harvest_lp_run), D_W s in FA = [even | odd]
            char *re = b->FA, *ro = b->FA + b->h64;
            d64(b, false, EPI_PLAIN, CM_M, 0, so, se, re, j->kappa, 0.0);
            d64(b, false, EPI_PLAIN, CM_M, 1, se, so, ro, j->kappa, 0.0);
            RawOuts R{}, R2{};
            R.p[0] = j->raw_out;
            R2.p[0] = j->raw_out2;
            launch_contract_lr(P64, g, b->G->links[P64], se, so, 0, se, so, 0, b->cpart, R, 1, 0.0, -2.0 * j->a, s,
                               j->local_only);
            launch_contract_lr(P64, g, b->G->links[P64], re, ro, 0, se, so, 0, b->cpart, R2, 1, 2.0, 0.0, s,
                               j->local_only);
        } else if (j->raw_out) {
            const uint32_t *codes = b->codes + (size_t)slot * 2 * g.vh;
            if (j->local_only) {
                RawOuts R{};
                R.p[0] = j->raw_out;
                launch_contract_local(P64, g, se, so, 0, codes, b->cpart, R, 1, s);
            } else {
                launch_contract(P64, g, b->G->links[P64], se, so, codes, b->cpart, j->raw_out, s);
            }
            if (j->hpe) {
                // (BH)^4 s into FB = [even | odd] through FA (see harvest_lp_run)
                char *ae = b->FA, *ao = b->FA + b->h64, *we = b->FB, *wo = b->FB + b->h64;
                d64(b, false, EPI_PLAIN, CM_BH, 1, se, nullptr, ao, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 0, ao, nullptr, we, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 1, we, nullptr, ao, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 0, ao, nullptr, we, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 0, so, nullptr, ae, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 1, ae, nullptr, wo, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 0, wo, nullptr, ae, j->kappa, j->a);
                d64(b, false, EPI_PLAIN, CM_BH, 1, ae, nullptr, wo, j->kappa, j->a);
                RawOuts R2{};
                R2.p[0] = j->raw_out2;
                launch_contract_local(P64, g, we, wo, 0, codes, b->cpart, R2, 1, s);
            }
        }
    } else {
        load_eta(b, slot, j);
        d64(b, false, EPI_PLAIN, CM_RECON, 1, se, Eo, so, j->kappa, j->a);
        launch_field_export(P64, g, 1, b->FC, j->x_canon, s);
    }
}

// |eta - M s| / |eta| in FP64 (s in FC, eta rebuilt in FA)
static int true_residual(Batch *b, int slot, Job *j)
{
    const Geom &g = b->G->g;
    hipStream_t s = b->stream;
    char *se = b->FC, *so = b->FC + b->h64;
    load_eta(b, slot, j);
    char *Ee = b->FA, *Eo = b->FA + b->h64;
    char *Be = b->FB, *Bo = b->FB + b->h64;
    double *p0 = b->partial + (size_t)slot * b->nblk;
    // even: eta_e - (A s_e - kappa D_eo s_o); odd: eta_o - (A s_o - kappa D_oe s_e)
    d64(b, false, EPI_RESID, CM_M, 0, so, se, Be, j->kappa, j->a, p0, Ee);
    launch_reduce(p0, b->nblk, 1, b->dres + 0, s);
    d64(b, false, EPI_RESID, CM_M, 1, se, so, Bo, j->kappa, j->a, p0, Eo);
    launch_reduce(p0, b->nblk, 1, b->dres + 1, s);
    launch_norm_partial(g, Ee, p0, s);
    launch_reduce(p0, b->nblk, 1, b->dres + 2, s);
    launch_norm_partial(g, Eo, p0, s);
    launch_reduce(p0, b->nblk, 1, b->dres + 3, s);
    TM_HIP(b->ctx, hipMemcpyAsync(b->hres, b->dres, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    TM_HIP(b->ctx, hipStreamSynchronize(s));
    const double num = b->hres[0] + b->hres[1], den = b->hres[2] + b->hres[3];
    j->true_rel = den > 0 ? std::sqrt(num / den) : 0.0;
    return TM_OK;
}

static bool same_params(const Job *a, const Job *b) { return a->kappa == b->kappa && a->a == b->a; }

int batch_process(Batch *b, std::vector<Job *> &finished)
{
    b->in_flight = false;
    int rc = TM_OK;
    const int S = b->S;
    // reliable updates, run over consecutive slots with equal (kappa, a)
    for (int s = 0; s < S;) {
        Job *j = b->slot_job[s];
        if (!j || b->st_h[s].status != ST_NEED_UPDATE) {
            s++;
            continue;
        }
        static const int cap = run_cap("TM_UPDATE_RUN");
        int n = 1;
        while (s + n < S && n < std::min(b->wslots, cap) && b->slot_job[s + n] && b->st_h[s + n].status == ST_NEED_UPDATE &&
               same_params(b->slot_job[s + n], j))
            n++;
        reliable_update_run(b, s, n);
        s += n;
    }
    // finished slots; LP noise solves harvested together
    auto done = [&](int s) {
        const int st = b->st_h[s].status;
        return b->slot_job[s] && st != ST_RUNNING && st != ST_NEED_UPDATE;
    };
    for (int s = 0; s < S;) {
        if (!done(s)) {
            s++;
            continue;
        }
        Job *j = b->slot_job[s];
        int n = 1;
        if (lp_harvest(b, j)) {
            static const int cap = run_cap("TM_HARVEST_RUN");
            while (s + n < S && n < std::min(b->wslots, cap) && done(s + n) && lp_harvest(b, b->slot_job[s + n]) &&
                   same_params(b->slot_job[s + n], j) && b->slot_job[s + n]->oet == j->oet &&
                   b->slot_job[s + n]->hpe == j->hpe && b->slot_job[s + n]->local_only == j->local_only)
                n++;
            harvest_lp_run(b, s, n);
        } else if (prep_prec(b, j) != P32) {
            harvest64(b, s, b->st_h[s], j);
        }
        for (int i = 0; i < n; i++) {
            Job *ji = b->slot_job[s + i];
            int e = harvest_done(b, s + i, b->st_h[s + i]);
            if (e != TM_OK) rc = e;
            finished.push_back(ji);
        }
        s += n;
    }
    return rc;
}

int run_jobs(std::vector<Batch *> &batches, std::vector<std::vector<Job *>> &queues)
{
    std::vector<size_t> next(batches.size(), 0);
    int rc = TM_OK;
    for (;;) {
        bool any = false, progressed = false;
        for (size_t k = 0; k < batches.size(); k++) {
            Batch *b = batches[k];
            if (b->in_flight) {
                hipError_t q = hipEventQuery(b->ev);
                if (q == hipErrorNotReady) {
                    any = true;
                    continue;
                }
                if (q != hipSuccess) return set_err(b->ctx, TM_ERR_HIP, "event query: %s", hipGetErrorString(q));
                std::vector<Job *> fin;
                int e = batch_process(b, fin);
                if (e != TM_OK && rc == TM_OK) rc = e;
                progressed = true;
            }
            // refill free slots
            if (next[k] < queues[k].size() && batch_free_slot(b) >= 0) {
                next[k] += batch_fill_many(b, queues[k].data() + next[k], (int)(queues[k].size() - next[k]));
                progressed = true;
            }
            if (batch_active(b) > 0) {
                int e = batch_launch_chunk(b);
                if (e != TM_OK) return e;
                any = true;
            }
        }
        if (!any) break;
        if (!progressed) {
            // wait for the first batch to finish its chunk, whichever it is,
            // so that its stream is refilled while the others still run
            int nflight = 0;
            for (Batch *b : batches) nflight += b->in_flight ? 1 : 0;
            if (nflight == 1) {
                for (Batch *b : batches)
                    if (b->in_flight) {
                        (void)hipEventSynchronize(b->ev);
                        break;
                    }
            } else if (nflight > 1) {
                for (bool ready = false; !ready;) {
                    for (Batch *b : batches)
                        if (b->in_flight && hipEventQuery(b->ev) != hipErrorNotReady) {
                            ready = true;
                            break;
                        }
                    if (!ready) std::this_thread::yield();
                }
            }
        }
    }
    for (Batch *b : batches) (void)hipStreamSynchronize(b->stream);
    return rc;
}

}  // namespace tmi
