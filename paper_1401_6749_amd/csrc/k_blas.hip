// CG scalar kernels (FP64, fixed-order reductions of per-block partials),
// site-local vector kernels, conversions between storage precisions and the
// streaming copy probe.
#include "tm_dev.h"
#include "tm_launch.h"

#include <algorithm>

namespace tmk {

// Fixed-order sum of n doubles by one block of BLOCK threads: thread i keeps
// four running sums, of v[i + (4k + j) BLOCK] for j = 0..3, so four loads
// are in flight per step of its loop; then (s0 + s1) + (s2 + s3) and the
// block tree.  Valid in thread 0; the same bits for the same n and v.
__device__ __forceinline__ double sum_fixed(const double *v, int n, double *lds)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
#pragma unroll 2
    for (; i + 3 * BLOCK < n; i += 4 * BLOCK) {
        a0 += v[i];
        a1 += v[i + BLOCK];
        a2 += v[i + 2 * BLOCK];
        a3 += v[i + 3 * BLOCK];
    }
    // at most three more
    if (i < n) a0 += v[i];
    if (i + BLOCK < n) a1 += v[i + BLOCK];
    if (i + 2 * BLOCK < n) a2 += v[i + 2 * BLOCK];
    return block_sum<BLOCK>((a0 + a1) + (a2 + a3), lds);
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < 1.0e300; }

__global__ __launch_bounds__(BLOCK) void k_cg_alpha(SlotState *st, const double *partial, int nblk)
{
    __shared__ double lds[BLOCK / 64];
    const int slot = blockIdx.x;
    SlotState &S = st[slot];
    if (S.status != ST_RUNNING) {
        if (threadIdx.x == 0) S.xpend = 0;  // no step this iteration
        return;
    }
    const double pap = sum_fixed(partial + (size_t)slot * nblk, nblk, lds);
    if (threadIdx.x == 0) {
        S.pap = pap;
        if (!finite_pos(pap)) {
            S.status = ST_NUMERIC;
            S.alpha = 0.0;
            S.xpend = 0;
        } else {
            S.alpha = S.rr / pap;
            S.xpend = 1;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_cg_beta(SlotState *st, const double *partial, int nblk)
{
    __shared__ double lds[BLOCK / 64];
    const int slot = blockIdx.x;
    SlotState &S = st[slot];
    if (S.status != ST_RUNNING) return;
    const double rr = sum_fixed(partial + (size_t)slot * nblk, nblk, lds);
    if (threadIdx.x == 0) {
        S.iter += 1;
        S.rr_new = rr;
        if (!(rr >= 0.0 && rr < 1.0e300)) {
            S.status = ST_NUMERIC;
        } else if (S.tol2 > 0.0 && rr <= S.tol2 * S.rr0) {
            // mixed precision confirms convergence on the true residual
            S.status = S.mixed ? ST_NEED_UPDATE : ST_CONVERGED;
            if (!S.mixed) S.rr = rr;
        } else if (S.mixed && rr <= S.delta2 * S.rr_ref) {
            S.status = ST_NEED_UPDATE;
        } else if (S.iter >= S.max_iter) {
            S.status = ST_MAXITER;
            S.rr = rr;
        } else {
            S.beta = rr / S.rr;
            S.rr = rr;
        }
    }
}

// block i starts slot st[i] from partial[i*nblk ..]
__global__ void k_slot_start(SlotState *st, const double *partial, int nblk, SlotStartParams P)
{
    __shared__ double lds[BLOCK / 64];
    const int i = blockIdx.x;
    const double rr0 = sum_fixed(partial + (size_t)i * nblk, nblk, lds);
    if (threadIdx.x == 0) {
        SlotState &S = st[i];
        const int max_iter = P.max_iter[i];
        S.kappa = P.kappa[i];
        S.a = P.a[i];
        S.tol2 = P.tol2[i];
        S.max_iter = max_iter;
        S.delta2 = P.delta2[i];
        S.mixed = P.mixed;
        S.iter = 0;
        S.rr0 = rr0;
        S.rr = rr0;
        S.rr_new = rr0;
        S.rr_ref = rr0;
        S.alpha = S.beta = S.pap = 0.0;
        S.xpend = 0;
        if (!(rr0 >= 0.0 && rr0 < 1.0e300))
            S.status = ST_NUMERIC;
        else if (rr0 == 0.0)
            S.status = ST_CONVERGED;
        else if (max_iter <= 0)
            S.status = ST_MAXITER;
        else
            S.status = ST_RUNNING;
    }
}

// block i finishes the reliable update of slot st[i] from partial[i*nblk ..]
__global__ void k_reliable_finish(SlotState *st, const double *partial, int nblk)
{
    __shared__ double lds[BLOCK / 64];
    const int i = blockIdx.x;
    const double rr = sum_fixed(partial + (size_t)i * nblk, nblk, lds);
    if (threadIdx.x == 0) {
        SlotState &S = st[i];
        S.rr_new = rr;
        if (!(rr >= 0.0 && rr < 1.0e300)) {
            S.status = ST_NUMERIC;
        } else if (S.tol2 > 0.0 && rr <= S.tol2 * S.rr0) {
            S.status = ST_CONVERGED;
            S.rr = rr;
        } else if (S.iter >= S.max_iter) {
            S.status = ST_MAXITER;
            S.rr = rr;
        } else {
            S.beta = rr / S.rr;
            S.rr = rr;
            S.rr_ref = rr;
            S.status = ST_RUNNING;
        }
    }
}

__global__ void k_reduce(const double *partial, int nblk, double *out)
{
    __shared__ double lds[BLOCK / 64];
    const double v = sum_fixed(partial + (size_t)blockIdx.x * nblk, nblk, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

void launch_cg_alpha(SlotState *st, const double *partial, int nslot, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_alpha, dim3(nslot), dim3(BLOCK), 0, s, st, partial, nblk);
}
void launch_cg_beta(SlotState *st, const double *partial, int nslot, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_beta, dim3(nslot), dim3(BLOCK), 0, s, st, partial, nblk);
}
void launch_slot_start(SlotState *st, const double *partial, int nblk, const SlotStartParams &P, int n,
                       hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_slot_start, dim3(n), dim3(BLOCK), 0, s, st, partial, nblk, P);
}

void launch_slot_start(SlotState *st, const double *partial, int nblk, double kappa, double a, double tol2,
                       int max_iter, double delta2, int mixed, hipStream_t s)
{
    SlotStartParams P{};
    P.kappa[0] = kappa;
    P.a[0] = a;
    P.tol2[0] = tol2;
    P.delta2[0] = delta2;
    P.max_iter[0] = max_iter;
    P.mixed = mixed;
    launch_slot_start(st, partial, nblk, P, 1, s);
}

void launch_reliable_finish(SlotState *st, const double *partial, int nblk, int n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_reliable_finish, dim3(n), dim3(BLOCK), 0, s, st, partial, nblk);
}
void launch_reduce(const double *partial, int nblk, int n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(n), dim3(BLOCK), 0, s, partial, nblk, out);
}

// ---------------------------------------------------------------------------
// p = r + beta p
// ---------------------------------------------------------------------------
// End of a CG iteration per slot: x += alpha p if the iteration took a step
// (x != nullptr and the slot's step is owed), then p = r + beta p if the slot
// keeps running.  Both read the old p.  The coefficients come from the
// slot's device state (the solver) or, for a standalone update, from the
// kernel's arguments.
struct UpdCoef {
    bool step, run;
    double alpha, beta;
};
struct SlotCoef {
    const SlotState *st;
    __device__ __forceinline__ UpdCoef operator()(int slot, bool has_x) const
    {
        const SlotState &S = st[slot];
        return {has_x && S.xpend != 0, S.status == ST_RUNNING, S.alpha, S.beta};
    }
};
struct ArgCoef {
    UpdateCoefs c;
    __device__ __forceinline__ UpdCoef operator()(int slot, bool has_x) const
    {
        return {has_x, true, c.alpha[slot], c.beta[slot]};
    }
};
template <int SP, int XR, class Coef>
__global__ __launch_bounds__(BLOCK) void k_p_update(Geom g, char *p, size_t p_slot, const char *r, size_t r_slot,
                                                    char *x, size_t x_slot, Coef coef, int nslot, int nblk,
                                                    int swz)
{
    using T = typename Real<SP>::T;
    int sblk, slot;
    if (!map_block(nblk, nslot, swz, sblk, slot)) return;
    const UpdCoef S = coef(slot, x != nullptr);
    const bool step = S.step, run = S.run;
    if (!step && !run) return;
    const int cb = sblk * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    cpx<T> pv[12];
    char *ps = p + (size_t)slot * p_slot;
    char *xs = step ? x + (size_t)slot * x_slot : nullptr;
    SpinorIO<SP>::load(ps, g.vh, cb, pv);
    // x and p are written with non-temporal stores: each is next read by a
    // later kernel, after far more data than the caches hold has passed
    if (step) {
        cpx<T> xv[12];
        SpinorIO<XR>::load(xs, g.vh, cb, xv);
        const T al = (T)S.alpha;
#pragma unroll
        for (int k = 0; k < 12; k++) xv[k] = xv[k] + cscale(al, pv[k]);
        SpinorIO<XR>::template store<T, true>(xs, g.vh, cb, xv);
    }
    if (run) {
        cpx<T> rv[12];
        SpinorIO<XR>::load(r + (size_t)slot * r_slot, g.vh, cb, rv);
        const T beta = (T)S.beta;
#pragma unroll
        for (int k = 0; k < 12; k++) pv[k] = rv[k] + cscale(beta, pv[k]);
        SpinorIO<SP>::template store<T, true>(ps, g.vh, cb, pv);
    }
}

template <class Coef>
static void launch_p_update_t(int sp, int xr, const Geom &g, char *p, size_t p_slot, const char *r, size_t r_slot,
                              char *x, size_t x_slot, const Coef &coef, int nslot, int swz, hipStream_t s)
{
    const int nblk = nblk_of(g);
    const int total = nblk * nslot;
    const int grid = swz ? 8 * ((total + 7) / 8) : total;
#define TMK_P(SP, XR)                                                                                         \
    if (sp == SP && xr == XR) {                                                                              \
        hipLaunchKernelGGL((k_p_update<SP, XR, Coef>), dim3(grid), dim3(BLOCK), 0, s, g, p, p_slot, r, r_slot, \
                           x, x_slot, coef, nslot, nblk, swz);                                                \
        return;                                                                                               \
    }
    TMK_P(P64, P64)
    TMK_P(P32, P32)
    TMK_P(P16, P16)
    TMK_P(PBF, PBF)
#undef TMK_P
}

void launch_p_update(int sp, int xr, const Geom &g, char *p, size_t p_slot, const char *r, size_t r_slot, char *x,
                     size_t x_slot, SlotState *st, int nslot, int swz, hipStream_t s)
{
    launch_p_update_t(sp, xr, g, p, p_slot, r, r_slot, x, x_slot, SlotCoef{st}, nslot, swz, s);
}

void launch_p_update_coefs(int sp, const Geom &g, char *p, const char *r, char *x, size_t slot_bytes,
                           const UpdateCoefs &c, int nslot, int swz, hipStream_t s)
{
    launch_p_update_t(sp, sp, g, p, slot_bytes, r, slot_bytes, x, slot_bytes, ArgCoef{c}, nslot, swz, s);
}

// ---------------------------------------------------------------------------
// Conversions and site-local kernels
// ---------------------------------------------------------------------------
template <int PI, int PO>
__global__ __launch_bounds__(BLOCK) void k_convert(Geom g, const char *in, size_t in_slot, char *out,
                                                   size_t out_slot)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    const int slot = blockIdx.y;
    cpx<double> v[12];
    SpinorIO<PI>::load(in + (size_t)slot * in_slot, g.vh, cb, v);
    SpinorIO<PO>::store(out + (size_t)slot * out_slot, g.vh, cb, v);
}

template <int PI>
static void conv_from(int pout, const Geom &g, const char *in, size_t is, char *out, size_t os, int nslot,
                      hipStream_t s)
{
    dim3 grid(nblk_of(g), nslot);
    switch (pout) {
    case P64: hipLaunchKernelGGL((k_convert<PI, P64>), grid, dim3(BLOCK), 0, s, g, in, is, out, os); break;
    case P32: hipLaunchKernelGGL((k_convert<PI, P32>), grid, dim3(BLOCK), 0, s, g, in, is, out, os); break;
    case P16: hipLaunchKernelGGL((k_convert<PI, P16>), grid, dim3(BLOCK), 0, s, g, in, is, out, os); break;
    case PBF: hipLaunchKernelGGL((k_convert<PI, PBF>), grid, dim3(BLOCK), 0, s, g, in, is, out, os); break;
    }
}

void launch_convert(int pin, int pout, const Geom &g, const char *in, size_t in_slot, char *out, size_t out_slot,
                    int nslot, hipStream_t s)
{
    switch (pin) {
    case P64: conv_from<P64>(pout, g, in, in_slot, out, out_slot, nslot, s); break;
    case P32: conv_from<P32>(pout, g, in, in_slot, out, out_slot, nslot, s); break;
    case P16: conv_from<P16>(pout, g, in, in_slot, out, out_slot, nslot, s); break;
    case PBF: conv_from<PBF>(pout, g, in, in_slot, out, out_slot, nslot, s); break;
    }
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k_zero(Geom g, char *f, size_t slot_bytes)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    cpx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) v[k] = cpx<double>{0.0, 0.0};
    SpinorIO<P>::store(f + (size_t)blockIdx.y * slot_bytes, g.vh, cb, v);
}

void launch_zero(int p, const Geom &g, char *f, size_t slot, int nslot, hipStream_t s)
{
    dim3 grid(nblk_of(g), nslot);
    switch (p) {
    case P64: hipLaunchKernelGGL((k_zero<P64>), grid, dim3(BLOCK), 0, s, g, f, slot); break;
    case P32: hipLaunchKernelGGL((k_zero<P32>), grid, dim3(BLOCK), 0, s, g, f, slot); break;
    case P16: hipLaunchKernelGGL((k_zero<P16>), grid, dim3(BLOCK), 0, s, g, f, slot); break;
    case PBF: hipLaunchKernelGGL((k_zero<PBF>), grid, dim3(BLOCK), 0, s, g, f, slot); break;
    }
}

// Start of a CG solve: r = p = rhs (rounded to precision PO, as k_convert
// rounds), x = 0 (as k_zero), reading rhs once.
template <int PI, int PO>
__global__ __launch_bounds__(BLOCK) void k_cg_start(Geom g, const char *in, size_t in_slot, char *r, char *p, char *x,
                                                    size_t o_slot)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    const size_t so = (size_t)blockIdx.y * o_slot;
    cpx<double> v[12];
    SpinorIO<PI>::load(in + (size_t)blockIdx.y * in_slot, g.vh, cb, v);
    SpinorIO<PO>::store(r + so, g.vh, cb, v);
    SpinorIO<PO>::store(p + so, g.vh, cb, v);
#pragma unroll
    for (int k = 0; k < 12; k++) v[k] = cpx<double>{0.0, 0.0};
    SpinorIO<PO>::store(x + so, g.vh, cb, v);
}

template <int PI>
static void cg_start_from(int po, const Geom &g, const char *in, size_t is, char *r, char *p, char *x, size_t os,
                          int nslot, hipStream_t s)
{
    dim3 grid(nblk_of(g), nslot);
    switch (po) {
    case P64: hipLaunchKernelGGL((k_cg_start<PI, P64>), grid, dim3(BLOCK), 0, s, g, in, is, r, p, x, os); break;
    case P32: hipLaunchKernelGGL((k_cg_start<PI, P32>), grid, dim3(BLOCK), 0, s, g, in, is, r, p, x, os); break;
    case P16: hipLaunchKernelGGL((k_cg_start<PI, P16>), grid, dim3(BLOCK), 0, s, g, in, is, r, p, x, os); break;
    case PBF: hipLaunchKernelGGL((k_cg_start<PI, PBF>), grid, dim3(BLOCK), 0, s, g, in, is, r, p, x, os); break;
    }
}

void launch_cg_start(int pin, int pout, const Geom &g, const char *in, size_t in_slot, char *r, char *p, char *x,
                     size_t out_slot, int nslot, hipStream_t s)
{
    if (pin == P64) cg_start_from<P64>(pout, g, in, in_slot, r, p, x, out_slot, nslot, s);
    else cg_start_from<P32>(pout, g, in, in_slot, r, p, x, out_slot, nslot, s);
}

__global__ __launch_bounds__(BLOCK) void k_accum_x(Geom g, char *x64, const char *x32, char *x32z, size_t s64,
                                                   size_t s32)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    x64 += (size_t)blockIdx.y * s64;
    x32 += (size_t)blockIdx.y * s32;
    if (x32z) x32z += (size_t)blockIdx.y * s32;
    cpx<double> a[12], b[12];
    SpinorIO<P64>::load(x64, g.vh, cb, a);
    SpinorIO<P32>::load(x32, g.vh, cb, b);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        a[k] = a[k] + b[k];
        b[k] = cpx<double>{0.0, 0.0};
    }
    SpinorIO<P64>::store(x64, g.vh, cb, a);
    if (x32z) SpinorIO<P32>::store(x32z, g.vh, cb, b);
}

void launch_accum_x(const Geom &g, char *x64, size_t s64, const char *x32_in, char *x32_zero, size_t s32, int n,
                    hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_accum_x, dim3(nblk_of(g), n), dim3(BLOCK), 0, s, g, x64, x32_in, x32_zero, s64, s32);
}

// per-tile |f|^2 of one FP64 half field: partial[tile], 64-site tiles
__global__ __launch_bounds__(BLOCK) void k_norm_partial(Geom g, const char *f, double *partial)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    double part = 0.0;
    if (cb < g.vh) {
        cpx<double> v[12];
        SpinorIO<P64>::load(f, g.vh, cb, v);
#pragma unroll
        for (int k = 0; k < 12; k++) part += norm2(v[k]);
    }
    part = wave_sum(part);
    const int tile = cb / TILE;
    if ((threadIdx.x & 63) == 0 && tile < ntile_of(g)) partial[tile] = part;
}

void launch_norm_partial(const Geom &g, const char *f, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm_partial, dim3(nblk_of(g)), dim3(BLOCK), 0, s, g, f, partial);
}

__global__ __launch_bounds__(BLOCK) void k_site_diag(Geom g, int mode, double a, const char *in, char *out)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    cpx<double> v[12];
    SpinorIO<P64>::load(in, g.vh, cb, v);
    if (mode == 1) {
        const double den = 1.0 / (1.0 + a * a);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double ch = k < 6 ? 1.0 : -1.0;
            v[k] = cmul(cpx<double>{den, -ch * a * den}, v[k]);
        }
    }
    SpinorIO<P64>::store(out, g.vh, cb, v);
}

void launch_site_diag(const Geom &g, int mode, double a, const char *in, char *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_site_diag, dim3(nblk_of(g)), dim3(BLOCK), 0, s, g, mode, a, in, out);
}

// ---------------------------------------------------------------------------
// Streaming copy, the measured HBM ceiling: each block moves CU_VEC * BLOCK
// consecutive 16-byte vectors, every thread issuing its CU_VEC loads before
// any store (several loads in flight per lane), streamed past the caches.
// ---------------------------------------------------------------------------
constexpr int CU_VEC = 4;

__global__ __launch_bounds__(BLOCK) void k_stream_copy(const tm_u32x4 *__restrict__ src, tm_u32x4 *__restrict__ dst,
                                                       size_t n)
{
    const size_t base = (size_t)blockIdx.x * BLOCK * CU_VEC + threadIdx.x;
    tm_u32x4 v[CU_VEC];
#pragma unroll
    for (int u = 0; u < CU_VEC; u++) {
        const size_t i = base + (size_t)u * BLOCK;
        if (i < n) v[u] = __builtin_nontemporal_load(&src[i]);
    }
#pragma unroll
    for (int u = 0; u < CU_VEC; u++) {
        const size_t i = base + (size_t)u * BLOCK;
        if (i < n) __builtin_nontemporal_store(v[u], &dst[i]);
    }
}

void launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (n == 0) return;
    const size_t blocks = (n + (size_t)BLOCK * CU_VEC - 1) / ((size_t)BLOCK * CU_VEC);
    for (size_t b0 = 0; b0 < blocks; b0 += 0x7FFFFFFF) {
        const size_t nb = std::min<size_t>(blocks - b0, 0x7FFFFFFF);
        const size_t off = b0 * BLOCK * CU_VEC;
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)nb), dim3(BLOCK), 0, s, (const tm_u32x4 *)src + off,
                           (tm_u32x4 *)dst + off, n - off);
    }
}

}  // namespace tmk
