// Even-odd hopping kernel (the hot loop of every CG iteration) with fused
// site-local epilogues.
//
// For an output site x of parity p it sums the eight neighbours of parity
// 1 - p:
//   hop(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)
// and, with DAG, the projectors swapped, which is g5 hop g5 (the hop of
// M^dagger).  Each projector (1 + s g_mu) has rank two in spin: the kernel
// forms the two independent spin rows ("half spinor"), multiplies them by the
// link and rebuilds the other two rows, so each neighbour costs two SU(3)
// products.  The epilogue then forms P*in2 + Q*hop per chirality.
#include "tm_dev.h"
#include "tm_launch.h"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#ifndef TM_DSLASH_WAVES_F64
#define TM_DSLASH_WAVES_F64 2
#endif
#ifndef TM_DSLASH_WAVES_F32
#define TM_DSLASH_WAVES_F32 3
#endif
#ifndef TM_DSLASH_WAVES_F16
#define TM_DSLASH_WAVES_F16 4
#endif

namespace tmk {

// Rebuild the four spin rows of (1 + S g_mu) psi from the transported half
// spinor w and add them to acc.
template <class T, int MU, int S>
__device__ __forceinline__ void accum(cpx<T> acc[12], const cpx<T> w[6])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cpx<T> w0 = w[c], w1 = w[3 + c];
        acc[c] = acc[c] + w0;
        acc[3 + c] = acc[3 + c] + w1;
        if (MU == 0) {  // rows 2,3 = iS w1, iS w0
            acc[6 + c] = S > 0 ? acc[6 + c] + ti(w1) : acc[6 + c] - ti(w1);
            acc[9 + c] = S > 0 ? acc[9 + c] + ti(w0) : acc[9 + c] - ti(w0);
        } else if (MU == 1) {  // S w1, -S w0
            acc[6 + c] = S > 0 ? acc[6 + c] + w1 : acc[6 + c] - w1;
            acc[9 + c] = S > 0 ? acc[9 + c] - w0 : acc[9 + c] + w0;
        } else if (MU == 2) {  // iS w0, -iS w1
            acc[6 + c] = S > 0 ? acc[6 + c] + ti(w0) : acc[6 + c] - ti(w0);
            acc[9 + c] = S > 0 ? acc[9 + c] - ti(w1) : acc[9 + c] + ti(w1);
        } else {  // S w0, S w1
            acc[6 + c] = S > 0 ? acc[6 + c] + w0 : acc[6 + c] - w0;
            acc[9 + c] = S > 0 ? acc[9 + c] + w1 : acc[9 + c] - w1;
        }
    }
}

// Buffer loads: one uniform resource per field (SGPRs), the component-group
// stride in the scalar offset and a single 32-bit lane offset per neighbour,
// so the eight neighbours do not each hold seven 64-bit lane addresses.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mkrsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ u32x4 bld16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ u32x2 bld8(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ uint32_t bld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ double2 as_d2(u32x4 v)
{
    double2 d;
    __builtin_memcpy(&d, &v, 16);
    return d;
}
__device__ __forceinline__ float4 as_f4(u32x4 v)
{
    float4 f;
    __builtin_memcpy(&f, &v, 16);
    return f;
}

// Neighbour spinor kept in its storage form (packed halves stay packed) and
// decoded one colour at a time.  lane: byte offset of the lane's slot field
// from the resource base; i: site within the parity.
template <int SP, class T>
struct Raw;
template <class T>
struct Raw<P64, T> {
    double2 q[12];
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t lane, int vh, int i)
    {
        const uint32_t vo = lane + (uint32_t)i * 16u;
#pragma unroll
        for (int k = 0; k < 12; k++) q[k] = as_d2(bld16(rs, vo, (uint32_t)k * (uint32_t)vh * 16u));
    }
    __device__ __forceinline__ cpx<T> get(int k) const { return cpx<T>{(T)q[k].x, (T)q[k].y}; }
};
template <class T>
struct Raw<P32, T> {
    float4 q[6];
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t lane, int vh, int i)
    {
        const uint32_t vo = lane + (uint32_t)i * 16u;
#pragma unroll
        for (int g = 0; g < 6; g++) q[g] = as_f4(bld16(rs, vo, (uint32_t)g * (uint32_t)vh * 16u));
    }
    __device__ __forceinline__ cpx<T> get(int k) const
    {
        const float4 &v = q[k >> 1];
        return (k & 1) ? cpx<T>{(T)v.z, (T)v.w} : cpx<T>{(T)v.x, (T)v.y};
    }
};
template <int P, class T>
struct RawHalf {
    u32x4 q[3];
    float sc;
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t lane, int vh, int i)
    {
        const uint32_t vo = lane + (uint32_t)i * 16u;
#pragma unroll
        for (int g = 0; g < 3; g++) q[g] = bld16(rs, vo, (uint32_t)g * (uint32_t)vh * 16u);
        sc = __uint_as_float(bld4(rs, lane + (uint32_t)i * 4u, 3u * (uint32_t)vh * 16u));
    }
    __device__ __forceinline__ cpx<T> get(int k) const
    {
        const u32x4 &v = q[k >> 2];
        const uint32_t w = v[k & 3];
        return cpx<T>{(T)(HalfCodec<P>::dec((uint16_t)(w & 0xFFFFu)) * sc),
                      (T)(HalfCodec<P>::dec((uint16_t)(w >> 16)) * sc)};
    }
};
template <int SP, class T>
struct RawSel {
    using type = Raw<SP, T>;
};
template <class T>
struct RawSel<P16, T> {
    using type = RawHalf<P16, T>;
};
template <class T>
struct RawSel<PBF, T> {
    using type = RawHalf<PBF, T>;
};

// Noise neighbour generated from its 4-byte Z4 code: c * eta with c = A^-1
// per chirality (a prep hop over A^-1 eta_o without any stored spinor).
template <class T>
struct RawZ4 {
    uint32_t code;
    cpx<T> c[2];
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t lane, int vh, int i)
    {
        code = bld4(rs, lane + (uint32_t)i * 4u, 0);
    }
    __device__ __forceinline__ cpx<T> get(int k) const
    {
        const T h = (code & Z4_ZERO) ? (T)0 : (T)0.70710678118654752440;
        const cpx<T> e{((code >> (2 * k)) & 1u) ? -h : h, ((code >> (2 * k + 1)) & 1u) ? -h : h};
        return cmul(c[k / 6], e);
    }
};

// link (par, mu) of site i through the gauge resource
template <int SP, class T>
__device__ __forceinline__ void load_link(__amdgpu_buffer_rsrc_t rs, int vh, int par, int mu, int i, Link<T> &L)
{
    const uint32_t pm = (uint32_t)(par * 4 + mu);
    if constexpr (SP == P64) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const double2 q = as_d2(bld16(rs, (uint32_t)i * 16u, (pm * 6u + k) * (uint32_t)vh * 16u));
            L.u[k / 3][k % 3] = cpx<T>{(T)q.x, (T)q.y};
        }
    } else if constexpr (SP == P32) {
#pragma unroll
        for (int g = 0; g < 3; g++) {
            const float4 q = as_f4(bld16(rs, (uint32_t)i * 16u, (pm * 3u + g) * (uint32_t)vh * 16u));
            L.u[(2 * g) / 3][(2 * g) % 3] = cpx<T>{(T)q.x, (T)q.y};
            L.u[(2 * g + 1) / 3][(2 * g + 1) % 3] = cpx<T>{(T)q.z, (T)q.w};
        }
    } else {
        // packed complex halves: all nine entries, or rows 0 and 1
        const uint32_t base = (uint32_t)(par * 4 + mu) * (uint32_t)HALF_LINK_BYTES * (uint32_t)vh;
        constexpr int NW = TM_HALF_LINK12 ? 6 : 9;
        uint32_t w[9];
        const u32x4 q = bld16(rs, (uint32_t)i * 16u, base);
#pragma unroll
        for (int k = 0; k < 4; k++) w[k] = q[k];
        if constexpr (NW == 6) {
            const u32x2 r = bld8(rs, (uint32_t)i * 8u, base + 16u * (uint32_t)vh);
            w[4] = r[0];
            w[5] = r[1];
        } else {
            const u32x4 q1 = bld16(rs, (uint32_t)i * 16u, base + 16u * (uint32_t)vh);
#pragma unroll
            for (int k = 0; k < 4; k++) w[4 + k] = q1[k];
            w[8] = bld4(rs, (uint32_t)i * 4u, base + 32u * (uint32_t)vh);
        }
#pragma unroll
        for (int k = 0; k < NW; k++)
            L.u[k / 3][k % 3] = cpx<T>{(T)HalfCodec<SP>::dec(w[k] & 0xFFFFu), (T)HalfCodec<SP>::dec(w[k] >> 16)};
        if constexpr (NW == 9) return;
    }
    rebuild_row2(L);
}

// half spinor of colour c for the projector (1 + S g_mu)
template <class T, int MU, int S, class R>
__device__ __forceinline__ void project_c(const R &raw, int c, cpx<T> &h0, cpx<T> &h1)
{
    const cpx<T> p0 = raw.get(c), p1 = raw.get(3 + c), p2 = raw.get(6 + c), p3 = raw.get(9 + c);
    if (MU == 0) {
        h0 = S > 0 ? p0 - ti(p3) : p0 + ti(p3);
        h1 = S > 0 ? p1 - ti(p2) : p1 + ti(p2);
    } else if (MU == 1) {
        h0 = S > 0 ? p0 - p3 : p0 + p3;
        h1 = S > 0 ? p1 + p2 : p1 - p2;
    } else if (MU == 2) {
        h0 = S > 0 ? p0 - ti(p2) : p0 + ti(p2);
        h1 = S > 0 ? p1 + ti(p3) : p1 - ti(p3);
    } else {
        h0 = S > 0 ? p0 + p2 : p0 - p2;
        h1 = S > 0 ? p1 + p3 : p1 - p3;
    }
}

// w = U h (FWD) or U^dagger h, accumulated colour by colour of h
// entry a of U h (FWD) or U^dagger h as two multiply-add chains: one
// multiply and five multiply-adds per real part
template <class T, bool FWD>
__device__ __forceinline__ cpx<T> link_row(const Link<T> &L, int a, const cpx<T> h[3])
{
    T re = 0, im = 0;
#pragma unroll
    for (int b = 0; b < 3; b++) {
        const cpx<T> u = FWD ? L.u[a][b] : L.u[b][a];
        const T ui = FWD ? u.im : -u.im;
        if (b == 0) {
            re = u.re * h[0].re;
            im = u.re * h[0].im;
        } else {
            re = fma(u.re, h[b].re, re);
            im = fma(u.re, h[b].im, im);
        }
        re = fma(-ui, h[b].im, re);
        im = fma(ui, h[b].re, im);
    }
    return {re, im};
}
template <class T, int MU, int S, bool FWD, class R>
__device__ __forceinline__ void transport(const Link<T> &L, const R &raw, cpx<T> w[6])
{
    cpx<T> h0[3], h1[3];
#pragma unroll
    for (int b = 0; b < 3; b++) project_c<T, MU, S>(raw, b, h0[b], h1[b]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        w[a] = link_row<T, FWD>(L, a, h0);
        w[3 + a] = link_row<T, FWD>(L, a, h1);
    }
}

// Resources of one Dslash application (uniform per block).
struct HopRes {
    __amdgpu_buffer_rsrc_t in, gauge;
    uint32_t lane;  // byte offset of this lane's input field from the input resource base
};

template <class RawT>
__device__ __forceinline__ void raw_setup(RawT &, double, double) {}
template <class T>
__device__ __forceinline__ void raw_setup(RawZ4<T> &z, double den, double a)
{
    // A^-1 = (1 - i a g5) / (1 + a^2): chirality + then -
    z.c[0] = cpx<T>{(T)den, (T)(-a * den)};
    z.c[1] = cpx<T>{(T)den, (T)(a * den)};
}

// ---------------------------------------------------------------------------
// FP16 hop with FP32 arithmetic on the stored halves.  A stored spinor
// component and a stored link entry are each one 32-bit word holding a
// complex number as two halves (re low, im high).  Every operation is an FP32
// fused multiply-add whose FP16 operands are widened exactly inside the
// instruction (v_fma_mix_f32), so neither the neighbour spinor nor the link
// is decoded into registers first: the spin projection is one FP32 add per
// real component and the colour transport four FP32 multiply-adds per complex
// product, the same arithmetic as the FP32 kernel.  The neighbour's per-site
// scale enters in the FP32 accumulation.
// ---------------------------------------------------------------------------
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2 as_h2(uint32_t x)
{
    h2 r;
    __builtin_memcpy(&r, &x, 4);
    return r;
}
__device__ __forceinline__ float lo_f(uint32_t x) { return (float)as_h2(x).x; }
__device__ __forceinline__ float hi_f(uint32_t x) { return (float)as_h2(x).y; }

// FP16 link (par, mu) of site i for the packed-operand transport: the
// stored entries as packed complex halves (re low, im high), all nine or,
// with TM_HALF_LINK12, rows 0 and 1 with row 2 rebuilt in FP32 as the
// conjugated cross product of the two
struct LinkPk {
    uint32_t w[TM_HALF_LINK12 ? 6 : 9];
    float r2[TM_HALF_LINK12 ? 6 : 1];
};
// entry (row, col) of a packed link as FP32 (re, im)
__device__ __forceinline__ void link_entry(const LinkPk &L, int row, int col, float &re, float &im)
{
    if (TM_HALF_LINK12 != 0 && row == 2) {
        re = L.r2[2 * col];
        im = L.r2[2 * col + 1];
    } else {
        re = lo_f(L.w[3 * row + col]);
        im = hi_f(L.w[3 * row + col]);
    }
}
__device__ __forceinline__ void load_link_words(__amdgpu_buffer_rsrc_t rs, int vh, int par, int mu, int i, LinkPk &L)
{
    const uint32_t base = (uint32_t)(par * 4 + mu) * (uint32_t)HALF_LINK_BYTES * (uint32_t)vh;
    const u32x4 q = bld16(rs, (uint32_t)i * 16u, base);
#pragma unroll
    for (int k = 0; k < 4; k++) L.w[k] = q[k];
    if constexpr (TM_HALF_LINK12 != 0) {
        const u32x2 r = bld8(rs, (uint32_t)i * 8u, base + 16u * (uint32_t)vh);
        L.w[4] = r[0];
        L.w[5] = r[1];
        // row 2 = conj(row 0 x row 1): entry j from columns k = j+1, l = j+2 (mod 3)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int k = (j + 1) % 3, l = (j + 2) % 3;
            const float ar = lo_f(L.w[k]), ai = hi_f(L.w[k]), br = lo_f(L.w[3 + l]), bi = hi_f(L.w[3 + l]);
            const float cr = lo_f(L.w[l]), ci = hi_f(L.w[l]), dr = lo_f(L.w[3 + k]), di = hi_f(L.w[3 + k]);
            // a b - c d, then conjugated
            L.r2[2 * j] = fmaf(ar, br, fmaf(-ai, bi, fmaf(-cr, dr, ci * di)));
            L.r2[2 * j + 1] = -fmaf(ar, bi, fmaf(ai, br, fmaf(-cr, di, -(ci * dr))));
        }
    } else {
        const u32x4 q1 = bld16(rs, (uint32_t)i * 16u, base + 16u * (uint32_t)vh);
#pragma unroll
        for (int k = 0; k < 4; k++) L.w[4 + k] = q1[k];
        L.w[8] = bld4(rs, (uint32_t)i * 4u, base + 32u * (uint32_t)vh);
    }
}

// sc times the half spinor of colour c for the projector (1 + S g_mu), FP32,
// from the stored words p[3*spin + colour]: two mixed-precision FMAs per real
// component, so the neighbour's scale costs nothing later
template <int MU, int S>
__device__ __forceinline__ void project_pk(const uint32_t p[12], int c, float sc, cpx<float> &h0, cpx<float> &h1)
{
    const uint32_t p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    const float s = S > 0 ? sc : -sc;
    if (MU == 0) {  // p0 - i S p3, p1 - i S p2
        h0 = {fmaf(sc, lo_f(p0), fmaf(s, hi_f(p3), 0.f)), fmaf(sc, hi_f(p0), fmaf(-s, lo_f(p3), 0.f))};
        h1 = {fmaf(sc, lo_f(p1), fmaf(s, hi_f(p2), 0.f)), fmaf(sc, hi_f(p1), fmaf(-s, lo_f(p2), 0.f))};
    } else if (MU == 1) {  // p0 - S p3, p1 + S p2
        h0 = {fmaf(sc, lo_f(p0), fmaf(-s, lo_f(p3), 0.f)), fmaf(sc, hi_f(p0), fmaf(-s, hi_f(p3), 0.f))};
        h1 = {fmaf(sc, lo_f(p1), fmaf(s, lo_f(p2), 0.f)), fmaf(sc, hi_f(p1), fmaf(s, hi_f(p2), 0.f))};
    } else if (MU == 2) {  // p0 - i S p2, p1 + i S p3
        h0 = {fmaf(sc, lo_f(p0), fmaf(s, hi_f(p2), 0.f)), fmaf(sc, hi_f(p0), fmaf(-s, lo_f(p2), 0.f))};
        h1 = {fmaf(sc, lo_f(p1), fmaf(-s, hi_f(p3), 0.f)), fmaf(sc, hi_f(p1), fmaf(s, lo_f(p3), 0.f))};
    } else {  // p0 + S p2, p1 + S p3
        h0 = {fmaf(sc, lo_f(p0), fmaf(s, lo_f(p2), 0.f)), fmaf(sc, hi_f(p0), fmaf(s, hi_f(p2), 0.f))};
        h1 = {fmaf(sc, lo_f(p1), fmaf(s, lo_f(p3), 0.f)), fmaf(sc, hi_f(p1), fmaf(s, hi_f(p3), 0.f))};
    }
}

// w = U h (FWD) or U^dagger h from the link entries
template <bool FWD>
__device__ __forceinline__ void transport_pk(const LinkPk &u, const cpx<float> h[3], float wr[3], float wi[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            float ur, ui;
            link_entry(u, FWD ? a : b, FWD ? b : a, ur, ui);
            if (!FWD) ui = -ui;
            re = fmaf(ur, h[b].re, fmaf(-ui, h[b].im, re));
            im = fmaf(ur, h[b].im, fmaf(ui, h[b].re, im));
        }
        wr[a] = re;
        wi[a] = im;
    }
}

// One FP16 neighbour n of site s on packed operands (see above); raw holds
// the neighbour's stored words.
template <int MU, bool FWD, bool DAG>
__device__ __forceinline__ void hop_compute_pk(const DslashArgs &A, __amdgpu_buffer_rsrc_t gauge, const Site &s, int n,
                                               const RawHalf<P16, float> &raw, cpx<float> acc[12])
{
    const int vh = A.g.vh;
    constexpr int S = (FWD != DAG) ? -1 : 1;
    uint32_t p[12];
#pragma unroll
    for (int k = 0; k < 12; k++) p[k] = raw.q[k >> 2][k & 3];
    float sc = raw.sc;
    LinkPk u;
    load_link_words(gauge, vh, FWD ? A.out_par : 1 - A.out_par, MU, FWD ? s.cb : n, u);
    if (MU == 3 && A.g.tbc < 0 && s.t == (FWD ? A.g.L[3] - 1 : 0)) sc = -sc;
    cpx<float> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; c++) project_pk<MU, S>(p, c, sc, h0[c], h1[c]);
    cpx<float> w[6];
    {
        float wr[3], wi[3];
        transport_pk<FWD>(u, h0, wr, wi);
#pragma unroll
        for (int a = 0; a < 3; a++) w[a] = cpx<float>{wr[a], wi[a]};
        transport_pk<FWD>(u, h1, wr, wi);
#pragma unroll
        for (int a = 0; a < 3; a++) w[3 + a] = cpx<float>{wr[a], wi[a]};
    }
    accum<float, MU, S>(acc, w);
}

// The two transported spin rows of neighbour n of site s (FP64/FP32 storage),
// before they are added into the output spinor: the projector, the link
// product and the antiperiodic sign of a temporal hop that wraps.  For the
// backward t neighbour only s.t is read.
template <class T, int SP, int MU, bool FWD, bool DAG, class RawT>
__device__ __forceinline__ void hop_w(const DslashArgs &A, __amdgpu_buffer_rsrc_t gauge, const Site &s, int n,
                                      const RawT &raw, cpx<T> w[6])
{
    constexpr int S = (FWD != DAG) ? -1 : 1;
    Link<T> L;
    load_link<SP, T>(gauge, A.g.vh, FWD ? A.out_par : 1 - A.out_par, MU, FWD ? s.cb : n, L);
    transport<T, MU, S, FWD>(L, raw, w);
    if (MU == 3 && A.g.tbc < 0 && s.t == (FWD ? A.g.L[3] - 1 : 0)) {
#pragma unroll
        for (int k = 0; k < 6; k++) w[k] = cpx<T>{-w[k].re, -w[k].im};
    }
}

// One neighbour n of site s from its loaded storage form raw: forward x+mu
// with (1 - g_mu) U_mu(x), or backward x-mu with (1 + g_mu) U_mu(x-mu)^dagger
// (projectors swapped for DAG).
template <class T, int SP, int MU, bool FWD, bool DAG, class RawT>
__device__ __forceinline__ void hop_compute(const DslashArgs &A, __amdgpu_buffer_rsrc_t gauge, const Site &s, int n,
                                            const RawT &raw, cpx<T> acc[12])
{
    if constexpr (SP == P16 && std::is_same<RawT, RawHalf<P16, float>>::value) {
        hop_compute_pk<MU, FWD, DAG>(A, gauge, s, n, raw, acc);
        return;
    }
    constexpr int S = (FWD != DAG) ? -1 : 1;
    cpx<T> w[6];
    hop_w<T, SP, MU, FWD, DAG, RawT>(A, gauge, s, n, raw, w);
    accum<T, MU, S>(acc, w);
}

// One neighbour read from the input resource.
template <class T, int SP, int MU, bool FWD, bool DAG, class RawT>
__device__ __forceinline__ void hop_dir(const DslashArgs &A, const HopRes &R, const Site &s, cpx<T> acc[12],
                                        double den, double a)
{
    const int n = nbr<MU, FWD ? 1 : -1>(A.g, s);
    RawT raw;
    raw_setup(raw, den, a);
    raw.load(R.in, R.lane, A.g.vh, n);
    hop_compute<T, SP, MU, FWD, DAG, RawT>(A, R.gauge, s, n, raw, acc);
}

// The eight neighbours as a runtime loop of uniform branches: each stage is
// its own basic block, so only one neighbour's operands are live at a time
// and occupancy (not load hoisting) hides memory latency.
template <class T, int SP, bool DAG, class RawT>
__device__ __forceinline__ void hop_all(const DslashArgs &A, const HopRes &R, const Site &s, cpx<T> acc[12],
                                        double den, double a)
{
#pragma unroll 1
    for (int d = 0; d < 8; d++) {
        switch (__builtin_amdgcn_readfirstlane(d)) {  // opaque: keeps the stages apart
        case 0: hop_dir<T, SP, 0, true, DAG, RawT>(A, R, s, acc, den, a); break;
        case 1: hop_dir<T, SP, 0, false, DAG, RawT>(A, R, s, acc, den, a); break;
        case 2: hop_dir<T, SP, 1, true, DAG, RawT>(A, R, s, acc, den, a); break;
        case 3: hop_dir<T, SP, 1, false, DAG, RawT>(A, R, s, acc, den, a); break;
        case 4: hop_dir<T, SP, 2, true, DAG, RawT>(A, R, s, acc, den, a); break;
        case 5: hop_dir<T, SP, 2, false, DAG, RawT>(A, R, s, acc, den, a); break;
        case 6: hop_dir<T, SP, 3, true, DAG, RawT>(A, R, s, acc, den, a); break;
        default: hop_dir<T, SP, 3, false, DAG, RawT>(A, R, s, acc, den, a); break;
        }
    }
}

// Epilogue coefficients per chirality c = 0 (spins 0,1: g5 = +1) and
// c = 1 (spins 2,3: g5 = -1); A = 1 + i a g5, A^-1 = (1 - i a g5)/(1 + a^2).
template <class T>
__device__ __forceinline__ void coefs(int mode, double kappa, double a, cpx<T> P[2], cpx<T> Q[2])
{
    const double den = 1.0 / (1.0 + a * a);
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const double ch = c == 0 ? 1.0 : -1.0;
        double pr = 0, pi = 0, qr = 0, qi = 0;
        switch (mode) {
        case CM_HOP: qr = 1; break;
        case CM_AINV: qr = den; qi = -ch * a * den; break;
        case CM_AINV_DAG: qr = den; qi = ch * a * den; break;
        case CM_MHAT: pr = 1; pi = ch * a; qr = -kappa * kappa; break;
        case CM_MHAT_DAG: pr = 1; pi = -ch * a; qr = -kappa * kappa; break;
        case CM_PREP: pr = 1; qr = kappa; break;
        case CM_RECON: pr = den; pi = -ch * a * den; qr = kappa * den; qi = -kappa * ch * a * den; break;
        case CM_M: pr = 1; pi = ch * a; qr = -kappa; break;
        case CM_MDAG: pr = 1; pi = -ch * a; qr = -kappa; break;
        case CM_BH: qr = -kappa * den; qi = kappa * ch * a * den; break;
        default: break;
        }
        P[c] = cpx<T>{(T)pr, (T)pi};
        Q[c] = cpx<T>{(T)qr, (T)qi};
    }
}

// Registers per lane are capped so that several waves per SIMD keep enough
// loads in flight: minimum waves per execution unit by storage precision.
template <int SP>
constexpr int dslash_waves()
{
    return SP == P64 ? TM_DSLASH_WAVES_F64 : SP == P32 ? TM_DSLASH_WAVES_F32 : TM_DSLASH_WAVES_F16;
}

// Site-local epilogue of output site cb of slot: out = P in2 + Q hop with the
// CG update / residual variants; returns the site's contribution to the
// slot's reduction (0 for EPI_PLAIN).
template <int SP, int EPI, bool IN2, int SRC, bool NT = false, int PO = SP>
__device__ __forceinline__ double epilogue(const DslashArgs &A, int slot, int cb, const cpx<typename Real<SP>::T> acc[12],
                                           double kappa, double a, double alpha)
{
    using T = typename Real<SP>::T;
    constexpr int XR = SP;  // x and r share the storage precision of the Dslash operands
    const int vh = A.g.vh;
    double part = 0.0;
    cpx<T> P[2], Q[2];
    coefs<T>(A.coef, kappa, a, P, Q);
    cpx<T> v[12];
    if (IN2) {
        cpx<T> y[12];
        if constexpr (SRC & 2) {
            const uint32_t c = A.codes[(size_t)slot * A.codes_slot / 4 + (size_t)A.out_par * vh + cb];
            const T h = (c & Z4_ZERO) ? (T)0 : (T)0.70710678118654752440;
#pragma unroll
            for (int k = 0; k < 12; k++)
                y[k] = cpx<T>{((c >> (2 * k)) & 1u) ? -h : h, ((c >> (2 * k + 1)) & 1u) ? -h : h};
        } else {
            SpinorIO<SP>::load(A.in2 + (size_t)slot * A.in2_slot, vh, cb, y);
        }
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = cmul(P[k / 6], y[k]) + cmul(Q[k / 6], acc[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = cmul(Q[k / 6], acc[k]);
    }
    if (EPI == EPI_PLAIN || EPI == EPI_NORM) {
        SpinorIO<SP>::template store<T, NT>(A.out + (size_t)slot * A.out_slot, vh, cb, v);
        if (EPI == EPI_NORM) {
#pragma unroll
            for (int k = 0; k < 12; k++) part += (double)norm2(v[k]);
        }
    } else if (EPI == EPI_CGUPD) {
        // r -= alpha Ap; x += alpha p waits for the direction update, which
        // reads p anyway, so this kernel touches two fields fewer
        cpx<T> rr[12];
        char *rs = A.r + (size_t)slot * A.xr_slot;
        SpinorIO<XR>::load(rs, vh, cb, rr);
        const T al = (T)alpha;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            rr[k] = rr[k] - cscale(al, v[k]);
            part += (double)norm2(rr[k]);
        }
        SpinorIO<XR>::store(rs, vh, cb, rr);
    } else if (EPI == EPI_START) {
        // start of a CG solve: r = p = v and x = 0 in the CG storage
        // precision PO, each rounded from the FP64 widening of v exactly as a
        // separate conversion of the stored FP32 v rounds it; the norm is
        // that of v, as EPI_NORM forms it
        cpx<double> vd[12], zd[12];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            vd[k] = cpx<double>{(double)v[k].re, (double)v[k].im};
            zd[k] = cpx<double>{0.0, 0.0};
            part += (double)norm2(v[k]);
        }
        SpinorIO<PO>::template store<double, NT>(A.r + (size_t)slot * A.xr_slot, vh, cb, vd);
        SpinorIO<PO>::template store<double, NT>(A.out + (size_t)slot * A.out_slot, vh, cb, vd);
        SpinorIO<PO>::template store<double, NT>(A.x + (size_t)slot * A.xr_slot, vh, cb, zd);
    } else {  // EPI_RESID (FP64 only)
        cpx<T> b[12];
        SpinorIO<P64>::load(A.b + (size_t)slot * A.b_slot, vh, cb, b);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            v[k] = b[k] - v[k];
            part += (double)norm2(v[k]);
        }
        SpinorIO<SP>::template store<T, NT>(A.out + (size_t)slot * A.out_slot, vh, cb, v);
    }
    return part;
}

// Thread mapping: a block holds BLOCK/R sites x R right-hand sides ("slots")
// of one slot group, lane = site * R + r, so the R lanes of a site sit in the
// same wave and their link loads hit the same addresses: each link is
// fetched once per R right-hand sides.  Per-slot reductions are over fixed
// 64-site tiles (one butterfly per tile), independent of R and of the
// number of slots, so a slot's sums have the same bits in any batch.
// SLOT: per-slot solver state (CG chunks) or uniform parameters (operator calls).
// SRC bit 0: the hop input is A^-1 eta decoded from Z4 codes (parity 1 - out_par);
// SRC bit 1: the site-local input is eta decoded from codes (parity out_par).
template <int SP, bool DAG, int EPI, bool IN2, bool SLOT, int R, int SRC = 0>
__global__ __launch_bounds__(BLOCK, dslash_waves<SP>()) void k_dslash(const DslashArgs A)
{
    using T = typename Real<SP>::T;
    constexpr int SPB = BLOCK / R;  // sites per block
    __shared__ double red[EPI == EPI_PLAIN ? 1 : BLOCK];
    const int ngroups = (A.nslot + R - 1) / R;
    int sb, grp;
    if (!map_block(A.nblk_site, ngroups, A.swz, sb, grp, A.gouter != 0)) return;
    const int r = threadIdx.x % R, sl = threadIdx.x / R;
    const int slot = grp * R + r;
    bool live = slot < A.nslot;
    double kappa = A.kappa_u, a = A.a_u, alpha = 0;
    if constexpr (SLOT) {
        // the block leaves only if none of its R slots is running
        bool any = false;
#pragma unroll
        for (int q = 0; q < R; q++) {
            const int sq = grp * R + q;
            any |= sq < A.nslot && A.st[sq].status == ST_RUNNING;
        }
        if (!any) return;
        if (live) {
            const SlotState &st = A.st[slot];
            live = st.status == ST_RUNNING;
            kappa = st.kappa;
            a = st.a;
            alpha = st.alpha;
        }
    }
    const int vh = A.g.vh;
    // t-walk: the block keeps one spatial chunk of SPB sites and walks tw
    // consecutive timeslices, so its t+-1 and spatial neighbours come back
    // from its own recent L2 lines instead of HBM.
    const int tw = A.twalk;
    int cb0, tstep;
    if (tw > 1) {
        const int zs_per_slice = A.g.v3h / SPB;
        const int tb = sb / zs_per_slice, zs = sb - tb * zs_per_slice;
        cb0 = tb * tw * A.g.v3h + zs * SPB + sl;
        tstep = A.g.v3h;
    } else {
        cb0 = sb * SPB + sl;
        tstep = 0;
    }
    for (int it = 0; it < (tw > 1 ? tw : 1); it++) {
    const int cb = cb0 + it * tstep;
    double part = 0.0;
    if (live && cb < vh) {
        const Site s = site_of(A.g, cb, A.out_par);
        HopRes res;
        res.gauge = mkrsrc(A.gauge, A.gauge_span);
        cpx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = cpx<T>{(T)0, (T)0};
        if constexpr (SRC & 1) {
            res.in = mkrsrc(A.codes + (size_t)slot * A.codes_slot / 4 + (size_t)(1 - A.out_par) * vh,
                            (uint32_t)vh * 4u);
            res.lane = 0;
            hop_all<T, SP, DAG, RawZ4<T>>(A, res, s, acc, 1.0 / (1.0 + a * a), a);
        } else {
            res.in = mkrsrc(A.in + (size_t)grp * R * A.in_slot, A.in_span);
            res.lane = (uint32_t)r * (uint32_t)A.in_slot;
            hop_all<T, SP, DAG, typename RawSel<SP, T>::type>(A, res, s, acc, 0.0, 0.0);
        }
        part = epilogue<SP, EPI, IN2, SRC>(A, slot, cb, acc, kappa, a, alpha);
    }
    if constexpr (EPI != EPI_PLAIN) {
        // tile sums: wave w reduces (slot r_w, tile t_w) of this block
        __syncthreads();  // red[] of the previous t-step fully consumed
        red[r * SPB + sl] = part;
        __syncthreads();
        constexpr int TPS = SPB / 64;  // tiles per slot in this block
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int rw = w / TPS, tw_ = w % TPS;
        const double v = wave_sum(red[rw * SPB + tw_ * 64 + lane]);
        const int sw = grp * R + rw;
        const int tile = (cb - sl) / 64 + tw_;
        if (lane == 0 && sw < A.nslot && tile < A.ntile) A.partial[(size_t)sw * A.ntile + tile] = v;
    }
    }
}


// ---------------------------------------------------------------------------
// Timeslice walk through LDS (FP32 and half storage, one slot per block).
//
// A block owns a chunk of one timeslice, cy rows (y) x cz planes (z) of full
// x rows, one site per thread (at most walk_max), for one right-hand side and
// walks tw consecutive timeslices.
// Every input site the walk touches is read from HBM (or L2) once: at each
// step the thread loads its own site of timeslice t+1, which is at once its
// forward t neighbour; the block stages that timeslice in LDS for the next
// step's x, y (and, for small planes, z) neighbours; the backward t
// neighbour is the thread's own site of t-1, from a second LDS buffer (half
// precision) or transported one step early (FP64, FP32: one buffer, see
// walk_nbuf).  Only neighbours outside the chunk (the z planes above and
// below, and y rows at the chunk's edges) are read from global memory, where
// the blocks working on those chunks have just fetched them into L2.  The
// chunk shape is picked on the host to minimise the halo; each 64-thread
// wave covers one 64-site reduction tile.  The arithmetic per neighbour is
// that of k_dslash, in the same order (backward t first, forward t last), so
// both buffer schemes give the same bits.
// ---------------------------------------------------------------------------
#ifndef TM_WALK_MAX_HALF
#define TM_WALK_MAX_HALF 256
#endif
#ifndef TM_WALK_MAX_F32
#define TM_WALK_MAX_F32 256
#endif
#ifndef TM_WALK_MAX_F64
#define TM_WALK_MAX_F64 256
#endif
// LDS buffers per block: one timeslice or two.  With two, the thread's own
// site of t+1 goes into the second buffer while the block still reads
// timeslice t, and the buffer of t-1 serves the backward t neighbour: one
// barrier per step.  With one (FP64 and FP32, whose sites take 192 and 96
// bytes), the backward t neighbour of the next step's output is transported
// while the thread's own site of t is at hand and carried in registers (six
// complex numbers), the thread's own site of t+1 stays in registers for the
// forward t neighbour, and the block overwrites the buffer between two
// barriers: half the LDS per block, so twice the blocks fit a CU.
#ifndef TM_WALK_NB_F64
#define TM_WALK_NB_F64 1
#endif
#ifndef TM_WALK_NB_F32
#define TM_WALK_NB_F32 1
#endif
template <int SP>
constexpr int walk_nbuf()
{
    return SP == P64 ? TM_WALK_NB_F64 : SP == P32 ? TM_WALK_NB_F32 : 2;
}
// largest chunk (threads per block) per storage precision: FP64 256 sites
// (48 KB, one buffer), FP32 256 (24 KB, one buffer), FP16/BF16 256 (26 KB,
// two buffers: 512-site chunks, 52 KB, read fewer halo neighbours, 0.75
// against 1.0 per site at 32^3x64, but their eight-wave blocks start less
// readily beside a concurrent stream's kernels: TSM step 273.9 against 278.7
// sources/s, same bits)
template <int SP>
constexpr int walk_max()
{
    return SP == P64 ? TM_WALK_MAX_F64 : SP == P32 ? TM_WALK_MAX_F32 : TM_WALK_MAX_HALF;
}

template <int SP>
struct WalkBuf;
template <>
struct WalkBuf<P64> {
    u32x4 q[walk_nbuf<P64>()][12][walk_max<P64>()];
    __device__ __forceinline__ void get(int b, int d, Raw<P64, double> &r) const
    {
#pragma unroll
        for (int k = 0; k < 12; k++) r.q[k] = as_d2(q[b][k][d]);
    }
    __device__ __forceinline__ void put(int b, int d, const Raw<P64, double> &r)
    {
#pragma unroll
        for (int k = 0; k < 12; k++) __builtin_memcpy(&q[b][k][d], &r.q[k], 16);
    }
};
template <>
struct WalkBuf<P32> {
    u32x4 q[walk_nbuf<P32>()][6][walk_max<P32>()];
    __device__ __forceinline__ void get(int b, int d, Raw<P32, float> &r) const
    {
#pragma unroll
        for (int g = 0; g < 6; g++) r.q[g] = as_f4(q[b][g][d]);
    }
    __device__ __forceinline__ void put(int b, int d, const Raw<P32, float> &r)
    {
#pragma unroll
        for (int g = 0; g < 6; g++) __builtin_memcpy(&q[b][g][d], &r.q[g], 16);
    }
};
template <int SP>
struct WalkBufHalf {
    u32x4 q[2][3][walk_max<SP>()];
    float sc[2][walk_max<SP>()];
    __device__ __forceinline__ void get(int b, int d, RawHalf<SP, float> &r) const
    {
#pragma unroll
        for (int g = 0; g < 3; g++) r.q[g] = q[b][g][d];
        r.sc = sc[b][d];
    }
    __device__ __forceinline__ void put(int b, int d, const RawHalf<SP, float> &r)
    {
#pragma unroll
        for (int g = 0; g < 3; g++) q[b][g][d] = r.q[g];
        sc[b][d] = r.sc;
    }
};
template <>
struct WalkBuf<P16> : WalkBufHalf<P16> {};
template <>
struct WalkBuf<PBF> : WalkBufHalf<PBF> {};

struct WalkPos {
    int buf;     // LDS buffer holding the current timeslice
    int yy, zz;  // the thread's row and plane within the chunk
};

// Halo prefetch of the half-precision walk (bit 0: z halo, bit 1: y halo):
// a thread on the chunk's edge loads its neighbour outside the chunk for the
// next timeslice at the end of a step, when the block owning that
// neighbour has just fetched it (its own next timeslice), instead of one
// step later, when the L2 has usually dropped the line.
#ifndef TM_WALK_HALO_PF
#define TM_WALK_HALO_PF 0
#endif

// t neighbours (two-buffer walk only): this thread's own site in timeslices
// t+-1, both in the other LDS buffer (t-1 until the backward neighbour is
// done, t+1 after).
// y/z neighbours outside the chunk come from the prefetched halo (hy, hz)
// when there is one, else from global memory.
template <int SP, int MU, bool FWD, bool DAG, class RawT>
__device__ __forceinline__ void walk_dir(const DslashArgs &A, const HopRes &R, const Site &s, const WalkBuf<SP> &W,
                                         const WalkPos &w, cpx<typename Real<SP>::T> acc[12], const RawT &hy,
                                         const RawT &hz, int pf)
{
    using T = typename Real<SP>::T;
    const int n = nbr<MU, FWD ? 1 : -1>(A.g, s);
    if constexpr (MU == 3) {
        RawT raw;
        W.get(w.buf ^ 1, threadIdx.x, raw);
        hop_compute<T, SP, MU, FWD, DAG, RawT>(A, R.gauge, s, n, raw, acc);
    } else {
        RawT raw;
        const int l = (int)threadIdx.x;
        bool in = true;
        int d = l;
        if (MU == 0) {
            d = l + (n - s.cb);  // same x row
        } else {
            const int c = MU == 1 ? A.wcy : A.wcz, full = MU == 1 ? A.g.L[1] : A.g.L[2];
            int q = (MU == 1 ? w.yy : w.zz) + (FWD ? 1 : -1);
            if (c == full) q = q < 0 ? c - 1 : (q == c ? 0 : q);  // the chunk spans the dimension
            else in = (unsigned)q < (unsigned)c;
            d = l + (q - (MU == 1 ? w.yy : w.zz)) * (MU == 1 ? A.g.lxh : A.g.lxh * A.wcy);
        }
        if (in) W.get(w.buf, d, raw);
        else if (MU == 1 && (pf & 2)) raw = hy;
        else if (MU == 2 && (pf & 1)) raw = hz;
        else raw.load(R.in, 0, A.g.vh, n);
        hop_compute<T, SP, MU, FWD, DAG, RawT>(A, R.gauge, s, n, raw, acc);
    }
}

#ifndef TM_WALK_WAVES_F64
#define TM_WALK_WAVES_F64 2
#endif
#ifndef TM_WALK_WAVES_F32
#define TM_WALK_WAVES_F32 3
#endif
#ifndef TM_WALK_WAVES_F16
#define TM_WALK_WAVES_F16 4
#endif
#ifndef TM_WALK_WAVES_F16_CG
#define TM_WALK_WAVES_F16_CG 4
#endif
template <int SP, int EPI>
constexpr int walk_waves()
{
    return SP == P64 ? TM_WALK_WAVES_F64
           : SP == P32 ? TM_WALK_WAVES_F32
                       : EPI == EPI_CGUPD ? TM_WALK_WAVES_F16_CG : TM_WALK_WAVES_F16;
}

// SRC bit 1: the site-local input is eta decoded from Z4 codes (the
// reconstruction of noise solves), as in k_dslash.
template <int SP, bool DAG, int EPI, bool IN2, bool SLOT, bool NT, int SRC = 0, int PO = SP>
__global__ __launch_bounds__(walk_max<SP>(), (walk_waves<SP, EPI>())) void k_dslash_walk(const DslashArgs A)
{
    using T = typename Real<SP>::T;
    using RawT = typename RawSel<SP, T>::type;
    __shared__ WalkBuf<SP> W;
    int sb, slot;
    if (!map_block(A.nblk_site, A.nslot, A.swz, sb, slot, A.gouter != 0)) return;
    double kappa = A.kappa_u, a = A.a_u, alpha = 0;
    if constexpr (SLOT) {
        const SlotState &st = A.st[slot];
        if (st.status != ST_RUNNING) return;  // uniform over the block
        kappa = st.kappa;
        a = st.a;
        alpha = st.alpha;
    }
    const Geom &g = A.g;
    const int vh = g.vh, lt = g.L[3], tw = A.twalk;
    const int ncy = g.L[1] / A.wcy, chunks = ncy * (g.L[2] / A.wcz);
    const int tb = sb / chunks, c = sb - tb * chunks;
    const int l = (int)threadIdx.x, xh = l % g.lxh, rz = l / g.lxh;
    const int yy = rz % A.wcy, zz = rz / A.wcy;
    // the thread's site within a timeslice
    const int o = xh + g.sy * ((c % ncy) * A.wcy + yy) + g.sz * ((c / ncy) * A.wcz + zz);
    const int t0 = tb * tw;
    HopRes R;
    R.gauge = mkrsrc(A.gauge, A.gauge_span);
    R.in = mkrsrc(A.in + (size_t)slot * A.in_slot, A.in_span);
    R.lane = 0;
    // halo prefetch roles: the one y (z) neighbour of this thread outside the
    // chunk, if the chunk is at least two rows (planes) deep and does not
    // span the dimension; pf bit set only for threads that have one
    constexpr int PF = (SP == P16 || SP == PBF) ? TM_WALK_HALO_PF : 0;
    int ydir = 0, zdir = 0, pf = 0;
    if constexpr ((PF & 2) != 0)
        if (A.wcy >= 2 && A.wcy < g.L[1]) ydir = yy == 0 ? -1 : (yy == A.wcy - 1 ? 1 : 0);
    if constexpr ((PF & 1) != 0)
        if (A.wcz >= 2 && A.wcz < g.L[2]) zdir = zz == 0 ? -1 : (zz == A.wcz - 1 ? 1 : 0);
    pf = (ydir ? 2 : 0) | (zdir ? 1 : 0);
    RawT hy{}, hz{};
    // halo sites of timeslice t (same o) into hy / hz
    auto halo_load = [&](int t) {
        const Site s1 = site_of(g, t * g.st + o, A.out_par);
        if (ydir) hy.load(R.in, 0, vh, ydir > 0 ? nbr<1, 1>(g, s1) : nbr<1, -1>(g, s1));
        if (zdir) hz.load(R.in, 0, vh, zdir > 0 ? nbr<2, 1>(g, s1) : nbr<2, -1>(g, s1));
    };
    constexpr int NB = walk_nbuf<SP>();
    // the backward t neighbour's projector sign (FWD = false)
    constexpr int SB = DAG ? -1 : 1;
    cpx<T> carry[NB == 1 ? 6 : 1];
    {
        RawT r0, r1;
        r0.load(R.in, 0, vh, ((t0 + lt - 1) % lt) * g.st + o);
        r1.load(R.in, 0, vh, t0 * g.st + o);
        if constexpr (PF != 0) halo_load(t0);
        if constexpr (NB == 1) {
            const Site s0 = site_of(g, t0 * g.st + o, A.out_par);
            hop_w<T, SP, 3, false, DAG, RawT>(A, R.gauge, s0, ((t0 + lt - 1) % lt) * g.st + o, r0, carry);
            W.put(0, threadIdx.x, r1);
        } else {
            W.put(1, threadIdx.x, r0);
            W.put(0, threadIdx.x, r1);
        }
    }
    __syncthreads();
    for (int k = 0; k < tw; k++) {
        const int t = t0 + k;
        const int cb = t * g.st + o;
        RawT nxt;
        if constexpr (NB != 1) nxt.load(R.in, 0, vh, ((t + 1) % lt) * g.st + o);
        const WalkPos w{NB == 1 ? 0 : (k & 1), yy, zz};
        const Site s = site_of(g, cb, A.out_par);
        cpx<T> acc[12];
#pragma unroll
        for (int q = 0; q < 12; q++) acc[q] = cpx<T>{(T)0, (T)0};
        if constexpr (NB == 1) {
            // the neighbours in the same order as with two buffers: backward
            // t (carried), x, y, z, forward t (nxt, still in registers)
            accum<T, 3, SB>(acc, carry);
#pragma unroll 1
            for (int d = 0; d < 6; d++) {
                switch (__builtin_amdgcn_readfirstlane(d)) {
                case 0: walk_dir<SP, 0, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 1: walk_dir<SP, 0, false, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 2: walk_dir<SP, 1, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 3: walk_dir<SP, 1, false, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 4: walk_dir<SP, 2, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                default: walk_dir<SP, 2, false, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                }
            }
            // the thread's own site of t+1, loaded only now so that it is not
            // held in registers through the spatial neighbours
            nxt.load(R.in, 0, vh, ((t + 1) % lt) * g.st + o);
            hop_compute<T, SP, 3, true, DAG, RawT>(A, R.gauge, s, nbr<3, 1>(g, s), nxt, acc);
            if (k + 1 < tw) {
                __syncthreads();  // every read of timeslice t is done
                // only this thread writes its slot: its own site of t (the
                // next output's backward t neighbour, input index cb) is read
                // back, then replaced by its site of t+1; the backward hop
                // reads only the output's t
                RawT own;
                W.get(0, threadIdx.x, own);
                W.put(0, threadIdx.x, nxt);
                Site s1 = s;
                s1.t = t + 1 == lt ? 0 : t + 1;
                hop_w<T, SP, 3, false, DAG, RawT>(A, R.gauge, s1, cb, own, carry);
            }
        } else {
            // backward t neighbour first: it frees this thread's slot of
            // timeslice t-1, which then takes timeslice t+1 (the forward t
            // neighbour now and the next step's spatial neighbours), so nxt is
            // not held in registers through the other seven neighbours.
            walk_dir<SP, 3, false, DAG>(A, R, s, W, w, acc, hy, hz, pf);
            W.put(w.buf ^ 1, threadIdx.x, nxt);
#pragma unroll 1
            for (int d = 0; d < 7; d++) {
                switch (__builtin_amdgcn_readfirstlane(d)) {
                case 0: walk_dir<SP, 0, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 1: walk_dir<SP, 0, false, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 2: walk_dir<SP, 1, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 3: walk_dir<SP, 1, false, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 4: walk_dir<SP, 2, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                case 5: walk_dir<SP, 2, false, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                default: walk_dir<SP, 3, true, DAG>(A, R, s, W, w, acc, hy, hz, pf); break;
                }
            }
        }
        // next timeslice's halo, while its owners are reading it
        if constexpr (PF != 0)
            if (k + 1 < tw) halo_load(t + 1);
        const double part = epilogue<SP, EPI, IN2, SRC, NT, PO>(A, slot, cb, acc, kappa, a, alpha);
        if constexpr (EPI != EPI_PLAIN) {
            // one wave = one 64-site reduction tile
            const double v = wave_sum(part);
            if ((threadIdx.x & 63) == 0) A.partial[(size_t)slot * A.ntile + cb / TILE] = v;
        }
        __syncthreads();
    }
}

template <int SP, bool DAG, int EPI, bool IN2, int R>
static void launch_r(const DslashArgs &A, hipStream_t s)
{
    const int ngroups = (A.nslot + R - 1) / R;
    const int total = A.nblk_site * ngroups;
    const int grid = A.swz ? 8 * ((total + 7) / 8) : total;
    if (A.st)
        hipLaunchKernelGGL((k_dslash<SP, DAG, EPI, IN2, true, R>), dim3(grid), dim3(BLOCK), 0, s, A);
    else
        hipLaunchKernelGGL((k_dslash<SP, DAG, EPI, IN2, false, R>), dim3(grid), dim3(BLOCK), 0, s, A);
}

// timeslices walked per block (TM_TWALK overrides; 1 = no walk)
inline int dslash_twalk()
{
    static int tw = [] {
        const char *e = getenv("TM_TWALK");
        return e ? std::max(1, atoi(e)) : 4;
    }();
    return tw;
}

// integer tuning knob from the environment (read once)
inline int env_knob(const char *name, int dflt)
{
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

// lanes per site: one per slot up to 4 (TM_DSLASH_R caps it)
inline int lanes_per_site(int nslot)
{
    static const int cap = std::max(1, std::min(4, env_knob("TM_DSLASH_R", 4)));
    int r = nslot >= 3 ? 4 : nslot;
    while (r > cap) r /= 2;
    return r;
}

// Chunk shape of the walk: cy rows x cz planes of full x rows with cy | Ly,
// cz | Lz, a multiple of 64 sites up to maxcs, each 64 threads one aligned
// 64-site tile (cy = Ly, or cy * Lx/2 a multiple of 64); the fewest halo
// neighbours per site (2/cy + 2/cz, no term for a dimension the chunk spans),
// then the largest chunk.  False if no shape fits.
inline bool walk_chunk(const Geom &g, int maxcs, int &cy, int &cz)
{
    double best = 1e30;
    int bs = 0;
    for (int y = 1; y <= g.L[1]; y++) {
        if (g.L[1] % y) continue;
        for (int z = 1; z <= g.L[2]; z++) {
            if (g.L[2] % z) continue;
            const int cs = y * z * g.lxh;
            if (cs > maxcs || cs % 64) continue;
            if (y != g.L[1] && (y * g.lxh) % 64) continue;
            const double halo = (y < g.L[1] ? 2.0 / y : 0.0) + (z < g.L[2] ? 2.0 / z : 0.0);
            if (halo < best - 1e-12 || (halo < best + 1e-12 && cs > bs)) {
                best = halo;
                bs = cs;
                cy = y;
                cz = z;
            }
        }
    }
    return bs > 0;
}

// timeslices per block of the LDS walk (TM_LDS_TWALK; TM_LDS_WALK=0 disables the walk)
inline int lds_twalk()
{
    static const int tw = env_knob("TM_LDS_WALK", 1) ? std::max(1, env_knob("TM_LDS_TWALK", 8)) : 0;
    return tw;
}

template <int SP, bool DAG, int EPI, bool IN2, int SRC = 0, int PO = SP>
static bool launch_walk(DslashArgs A, hipStream_t s)
{
    {
        int tw = lds_twalk();
        const uint64_t field = (uint64_t)A.g.vh * (SP == P64 ? 192 : SP == P32 ? 96 : 52);
        if (tw < 1 || field >= (1ull << 32) || !walk_chunk(A.g, walk_max<SP>(), A.wcy, A.wcz)) return false;
        while (A.g.L[3] % tw) tw--;
        A.twalk = tw;
        A.in_span = (uint32_t)field;
        A.gauge_span = (uint32_t)std::min<uint64_t>(
            (uint64_t)2 * 4 * A.g.vh * (SP == P64 ? 96 : SP == P32 ? 48 : HALF_LINK_BYTES), 0xFFFFFFFFull);
        static const int gouter = env_knob("TM_GROUP_OUTER", 0);
        A.gouter = gouter;
        const int cs = A.wcy * A.wcz * A.g.lxh;
        A.nblk_site = (A.g.v3h / cs) * (A.g.L[3] / tw);
        A.ntile = ntile_of(A.g);
        const int total = A.nblk_site * A.nslot;
        const int grid = A.swz ? 8 * ((total + 7) / 8) : total;
        // outputs are streamed past L2 (non-temporal), keeping it for the halo lines
        if constexpr (SRC != 0 || PO != SP)
            hipLaunchKernelGGL((k_dslash_walk<SP, DAG, EPI, IN2, false, true, SRC, PO>), dim3(grid), dim3(cs), 0, s,
                               A);
        else if (A.st)
            hipLaunchKernelGGL((k_dslash_walk<SP, DAG, EPI, IN2, true, true>), dim3(grid), dim3(cs), 0, s, A);
        else
            hipLaunchKernelGGL((k_dslash_walk<SP, DAG, EPI, IN2, false, true>), dim3(grid), dim3(cs), 0, s, A);
        return true;
    }
}

template <int SP, bool DAG, int EPI, bool IN2>
static void launch_t(DslashArgs A, hipStream_t s)
{
    if (launch_walk<SP, DAG, EPI, IN2>(A, s)) return;
    int R = lanes_per_site(A.nslot);
    // 32-bit buffer offsets: the R input fields of a group must span < 4 GiB
    const uint64_t field = (uint64_t)A.g.vh * (SP == P64 ? 192 : SP == P32 ? 96 : 52);
    if (R > 1 && ((uint64_t)(R - 1) * A.in_slot + field >= (1ull << 32) || A.in_slot % 16)) R = 1;
    A.in_span = (uint32_t)std::min<uint64_t>((uint64_t)(R - 1) * A.in_slot + field, 0xFFFFFFFFull);
    A.gauge_span = (uint32_t)std::min<uint64_t>((uint64_t)2 * 4 * A.g.vh * (SP == P64 ? 96 : SP == P32 ? 48 : HALF_LINK_BYTES),
                                                0xFFFFFFFFull);
    const int spb = BLOCK / R;
    int tw = dslash_twalk();
    if (tw > 1 && (A.g.v3h % spb != 0 || A.g.L[3] % tw != 0)) tw = 1;
    A.twalk = tw;
    static const int gouter = env_knob("TM_GROUP_OUTER", 0);
    A.gouter = gouter;
    A.nblk_site = tw > 1 ? A.g.vh / spb / tw : (A.g.vh + spb - 1) / spb;
    A.ntile = ntile_of(A.g);
    if (R == 1) launch_r<SP, DAG, EPI, IN2, 1>(A, s);
    else if (R == 2) launch_r<SP, DAG, EPI, IN2, 2>(A, s);
    else launch_r<SP, DAG, EPI, IN2, 4>(A, s);
}

template <int SP>
static void launch_sp(bool dag, int epi, bool in2, const DslashArgs &A, hipStream_t s)
{
#define TMK_CASE(D, E, I) \
    if (dag == D && epi == E && in2 == I) return launch_t<SP, D, E, I>(A, s);
    TMK_CASE(false, EPI_PLAIN, false)
    TMK_CASE(true, EPI_PLAIN, false)
    TMK_CASE(false, EPI_PLAIN, true)
    TMK_CASE(true, EPI_PLAIN, true)
    TMK_CASE(false, EPI_NORM, true)
    TMK_CASE(true, EPI_NORM, true)
    TMK_CASE(false, EPI_CGUPD, true)
    TMK_CASE(true, EPI_CGUPD, true)
    if constexpr (SP == P64) {
        TMK_CASE(true, EPI_RESID, true)
        TMK_CASE(false, EPI_RESID, true)
    }
#undef TMK_CASE
}

// Z4-code sources (prep and reconstruction of noise solves), FP32 and FP64.
// The reconstruction (hop input a field, site-local input the codes) runs on
// the timeslice walk where a chunk fits; the preparation (hop input decoded
// from codes) and small lattices on the register kernel.
template <int SP, int SRC>
static void launch_src(DslashArgs A, hipStream_t s)
{
    A.st = nullptr;  // uniform parameters
    if constexpr (SRC == 2)
        if (launch_walk<SP, false, EPI_PLAIN, true, 2>(A, s)) return;
    A.twalk = 1;
    A.gouter = 0;
    A.nblk_site = (A.g.vh + BLOCK - 1) / BLOCK;
    A.ntile = ntile_of(A.g);
    A.gauge_span = (uint32_t)std::min<uint64_t>((uint64_t)2 * 4 * A.g.vh * link_bytes(SP), 0xFFFFFFFFull);
    A.in_span = (uint32_t)std::min<uint64_t>((uint64_t)A.g.vh * (SP == P64 ? 192 : SP == P32 ? 96 : 52), 0xFFFFFFFFull);
    const int total = A.nblk_site * A.nslot;
    const int grid = A.swz ? 8 * ((total + 7) / 8) : total;
    hipLaunchKernelGGL((k_dslash<SP, false, EPI_PLAIN, true, false, 1, SRC>), dim3(grid), dim3(BLOCK), 0, s, A);
}

int launch_dslash_codes(int sp, int src, const DslashArgs &A, hipStream_t s)
{
    if (src == 3) {
        switch (sp) {
        case P64: launch_src<P64, 3>(A, s); break;
        case P32: launch_src<P32, 3>(A, s); break;
        case P16: launch_src<P16, 3>(A, s); break;
        case PBF: launch_src<PBF, 3>(A, s); break;
        default: return -1;
        }
    } else if (src == 2 && (sp == P64 || sp == P32)) {
        sp == P64 ? launch_src<P64, 2>(A, s) : launch_src<P32, 2>(A, s);
    } else {
        return -1;
    }
    return 0;
}

int launch_dslash_start(int sp, int po, const DslashArgs &A, hipStream_t s)
{
    if (A.nslot < 1) return 0;
    DslashArgs B = A;
    B.st = nullptr;  // uniform parameters
    bool ok = false;
    if (sp == P32 && po == P16) ok = launch_walk<P32, true, EPI_START, true, 0, P16>(B, s);
    else if (sp == P32 && po == PBF) ok = launch_walk<P32, true, EPI_START, true, 0, PBF>(B, s);
    else if (sp == P16 && po == P16) ok = launch_walk<P16, true, EPI_START, true, 0, P16>(B, s);
    else if (sp == PBF && po == PBF) ok = launch_walk<PBF, true, EPI_START, true, 0, PBF>(B, s);
    return ok ? 0 : -1;
}

int launch_dslash(int sp, bool dag, int epi, bool in2, const DslashArgs &A, hipStream_t s)
{
    if (A.nslot < 1) return 0;
    if (epi == EPI_RESID && sp != P64) return -1;
    if ((epi == EPI_NORM || epi == EPI_CGUPD || epi == EPI_RESID) && !in2) return -1;
    switch (sp) {
    case P64: launch_sp<P64>(dag, epi, in2, A, s); break;
    case P32: launch_sp<P32>(dag, epi, in2, A, s); break;
    case P16: launch_sp<P16>(dag, epi, in2, A, s); break;
    case PBF: launch_sp<PBF>(dag, epi, in2, A, s); break;
    default: return -1;
    }
    return 0;
}

}  // namespace tmk
