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
#include <cstring>
#include <thread>

#include "tm_internal.h"

using namespace tmk;

namespace tmi {

Kind kind_of(const tm_solver_params &p)
{
    if (p.mode == TM_SOLVE_MIXED) return K_MIXED;
    if (p.mode == TM_SOLVE_LP) return p.half_prec == TM_PREC_BF16 ? K_LPBF : K_LP16;
    return K_F64;
}

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

size_t batch_footprint(const tm_gauge *G, Kind kind, int S)
{
    const Geom &g = G->g;
    const int sp = kind_prec(kind), xr = kind_xr(kind);
    size_t b = 0;
    b += (size_t)S * 3 * slot_pitch(half_bytes(sp, g));  // p, u, t
    b += (size_t)S * 2 * slot_pitch(half_bytes(xr, g));  // x, r
    if (kind == K_MIXED) b += (size_t)S * 2 * half_bytes(P64, g);  // x64, b64
    b += (size_t)S * 2 * g.vh * sizeof(uint32_t);      // noise codes
    b += 3 * 2 * half_bytes(P64, g);                   // FP64 scratch FA, FB, FC
    b += (size_t)S * ntile_of(g) * sizeof(double) + 4096;
    b += (size_t)g.L[3] * contract_nchunk(g) * 288 * sizeof(double);
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
    b->FA = carve(cur, 2 * b->h64);
    b->FB = carve(cur, 2 * b->h64);
    b->FC = carve(cur, 2 * b->h64);
    b->partial = (double *)carve(cur, (size_t)S * b->nblk * sizeof(double) + 4096);
    b->cpart = (double *)carve(cur, (size_t)g.L[3] * contract_nchunk(g) * 288 * sizeof(double));
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

// Prep/reconstruction precision of a job: LP noise solves run them in FP32
// (their target is a 1e-2 residual), everything else in FP64.
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

int batch_fill(Batch *b, int slot, Job *j)
{
    const Geom &g = b->G->g;
    hipStream_t s = b->stream;
    b->slot_job[slot] = j;
    b->slot_updates[slot] = 0;
    b->slot_pending_update[slot] = 0;
    j->t_fill = now_s();
    if (b->t_first == 0) b->t_first = j->t_fill;
    const bool mixed = b->kind == K_MIXED;
    const double tol2 = j->fixed > 0 ? 0.0 : j->tol * j->tol;
    const int maxit = j->fixed > 0 ? j->fixed : j->max_iter;
    const double delta = j->delta > 0 ? j->delta : 0.1;
    double *part = b->partial + (size_t)slot * b->nblk;
    const int pp = prep_prec(b, j);
    if (j->noise) {
        // bhat_e = eta_e + kappa D_eo A^-1 eta_o straight from the Z4 codes,
        // rhs = Mhat^dag bhat = A^dag bhat - kappa^2 D'_eo A^-dag D'_oe bhat
        launch_z4_codes(g, j->seed, j->src, b->codes + (size_t)slot * 2 * g.vh, s);
        char *Be = b->FB, *To = b->FC;  // scratch fields in precision pp
        dsl_codes(b, pp, 3, CM_PREP, 0, slot, nullptr, Be, j->kappa, j->a);
        dsl(b, pp, true, EPI_PLAIN, CM_AINV_DAG, 1, Be, nullptr, To, j->kappa, j->a);
        if (pp == P32) {
            // LP: the FP32 right-hand side is rounded once into r and p (half precision)
            char *rhs = b->FA;
            dsl(b, P32, true, EPI_NORM, CM_MHAT_DAG, 0, To, Be, rhs, j->kappa, j->a, part);
            launch_slot_start(b->st + slot, part, b->nblk, j->kappa, j->a, tol2, maxit, delta * delta, 0, s);
            launch_convert(P32, b->xr, g, rhs, 0, b->r + slot * b->hxr, 0, 1, s);
            launch_convert(P32, b->sp, g, rhs, 0, b->p + slot * b->hsp, 0, 1, s);
            launch_zero(b->xr, g, b->x + slot * b->hxr, 0, 1, s);
            return TM_OK;
        }
        char *Ce = b->FA;
        dsl(b, P64, true, EPI_NORM, CM_MHAT_DAG, 0, To, Be, Ce, j->kappa, j->a, part);
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
    A.x = b->x;
    A.r = b->r;
    A.p = b->p;
    A.xr_slot = b->hxr;
    A.p_slot = b->hsp;
    launch_dslash(sp, true, EPI_CGUPD, true, A, b->stream);
    launch_cg_beta(b->st, b->partial, b->S, b->nblk, b->stream);
    launch_p_update(sp, b->xr, b->G->g, b->p, b->hsp, b->r, b->hxr, b->st, b->S, b->ctx->swz, b->stream);
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

// FP64 reliable update of a mixed-precision slot: x64 += x32, r = b - Mhat^dag Mhat x64
// in FP64, r32 = r, then the CG direction continues with beta = |r|^2/|r_old|^2.
static void reliable_update(Batch *b, int slot)
{
    const Geom &g = b->G->g;
    Job *j = b->slot_job[slot];
    hipStream_t s = b->stream;
    char *x64 = b->x64 + slot * b->h64;
    char *x32 = b->x + slot * b->hxr;
    char *Be = b->FB, *Bo = b->FB + b->h64, *Ce = b->FC;
    launch_accum_x(g, x64, x32, x32, s);
    d64(b, false, EPI_PLAIN, CM_AINV, 1, x64, nullptr, Bo, j->kappa, j->a);
    d64(b, false, EPI_PLAIN, CM_MHAT, 0, Bo, x64, Be, j->kappa, j->a);
    d64(b, true, EPI_PLAIN, CM_AINV_DAG, 1, Be, nullptr, Bo, j->kappa, j->a);
    double *part = b->partial + (size_t)slot * b->nblk;
    d64(b, true, EPI_RESID, CM_MHAT_DAG, 0, Bo, Be, Ce, j->kappa, j->a, part, b->b64 + slot * b->h64);
    launch_convert(P64, P32, g, Ce, 0, b->r + slot * b->hxr, 0, 1, s);
    launch_reliable_finish(b->st + slot, part, b->nblk, s);
    launch_p_update(b->sp, b->xr, g, b->p + slot * b->hsp, b->hsp, b->r + slot * b->hxr, b->hxr, b->st + slot, 1,
                    b->ctx->swz, s);
    b->slot_updates[slot]++;
}

static void harvest64(Batch *b, int slot, const SlotState &S, Job *j);
static int true_residual(Batch *b, int slot, Job *j);

// reconstruct s = (s_e, s_o), contract or export, optional true residual
static int harvest(Batch *b, int slot, const SlotState &S)
{
    const Geom &g = b->G->g;
    Job *j = b->slot_job[slot];
    hipStream_t s = b->stream;
    if (prep_prec(b, j) == P32) {
        // LP noise solve: s_e = x widened to FP32, s_o = A^-1 (eta_o + kappa D_oe s_e) from the
        // codes, contraction on FP32 s and FP32 links with FP64 accumulation
        char *se32 = b->FB, *so32 = b->FC;
        launch_convert(b->xr, P32, g, b->x + slot * b->hxr, 0, se32, 0, 1, s);
        dsl_codes(b, P32, 2, CM_RECON, 1, slot, se32, so32, j->kappa, j->a);
        if (j->raw_out)
            launch_contract(P32, g, b->G->links[P32], se32, so32, b->codes + (size_t)slot * 2 * g.vh, b->cpart,
                            j->raw_out, s);
    } else {
        harvest64(b, slot, S, j);
    }
    j->iters = S.iter;
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
        if (S.status != ST_CONVERGED) launch_accum_x(g, x64, b->x + slot * b->hxr, nullptr, s);
        launch_convert(P64, P64, g, x64, 0, se, 0, 1, s);
    } else {
        launch_convert(b->xr, P64, g, b->x + slot * b->hxr, 0, se, 0, 1, s);
    }
    char *Eo = b->FA + b->h64;
    if (j->noise) {
        // s_o = A^-1 (eta_o + kappa D_oe s_e) with eta_o from the codes
        dsl_codes(b, P64, 2, CM_RECON, 1, slot, se, so, j->kappa, j->a);
        if (j->raw_out)
            launch_contract(P64, g, b->G->links[P64], se, so, b->codes + (size_t)slot * 2 * g.vh, b->cpart,
                            j->raw_out, s);
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

int batch_process(Batch *b, std::vector<Job *> &finished)
{
    b->in_flight = false;
    int rc = TM_OK;
    for (int s = 0; s < b->S; s++) {
        Job *j = b->slot_job[s];
        if (!j) continue;
        const SlotState &S = b->st_h[s];
        if (S.status == ST_RUNNING) continue;
        if (S.status == ST_NEED_UPDATE) {
            reliable_update(b, s);
            continue;
        }
        int e = harvest(b, s, S);
        if (e != TM_OK) rc = e;
        finished.push_back(j);
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
            int slot;
            while (next[k] < queues[k].size() && (slot = batch_free_slot(b)) >= 0) {
                batch_fill(b, slot, queues[k][next[k]++]);
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
            // block on the first batch still in flight
            for (Batch *b : batches)
                if (b->in_flight) {
                    (void)hipEventSynchronize(b->ev);
                    break;
                }
        }
    }
    for (Batch *b : batches) (void)hipStreamSynchronize(b->stream);
    return rc;
}

}  // namespace tmi
