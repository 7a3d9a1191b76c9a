// Device-side building blocks of libtm: complex arithmetic, lattice geometry
// in the even-odd site-major layout, storage formats of spinors and links,
// the counter-based Z4 generator and deterministic block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tm_types.h"

namespace tmk {

// ---------------------------------------------------------------------------
// Complex numbers
// ---------------------------------------------------------------------------
template <class T>
struct cpx {
    T re, im;
};

template <class T>
__device__ __forceinline__ cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <class T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <class T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T>
__device__ __forceinline__ cpx<T> cscale(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
// i * a and -i * a
template <class T>
__device__ __forceinline__ cpx<T> ti(cpx<T> a) { return {-a.im, a.re}; }
template <class T>
__device__ __forceinline__ cpx<T> tmi(cpx<T> a) { return {a.im, -a.re}; }
template <class T>
__device__ __forceinline__ T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// Lattice geometry.  Sites of one parity are indexed by cb = lex / 2; the
// sites of parity p in timeslice t occupy cb in [t*V3h, (t+1)*V3h).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d)
{
    return (uint32_t)(((uint64_t)__umulhi(n, d.m) + n) >> d.l);
}

struct Site {
    int x, y, z, t, xh, cb;
};

__device__ __forceinline__ Site site_of(const Geom &g, int cb, int par)
{
    Site s;
    s.cb = cb;
    uint32_t q1 = fdiv((uint32_t)cb, g.div_xh);
    s.xh = cb - (int)q1 * g.lxh;
    uint32_t q2 = fdiv(q1, g.div_y);
    s.y = (int)q1 - (int)q2 * g.L[1];
    uint32_t q3 = fdiv(q2, g.div_z);
    s.z = (int)q2 - (int)q3 * g.L[2];
    s.t = (int)q3;
    s.x = 2 * s.xh + ((par + s.y + s.z + s.t) & 1);
    return s;
}

// cb index (in the other parity) of the neighbour x + dir*mu
template <int MU, int DIR>
__device__ __forceinline__ int nbr(const Geom &g, const Site &s)
{
    if (MU == 0) {
        int xn = DIR > 0 ? (s.x + 1 == g.L[0] ? 0 : s.x + 1) : (s.x == 0 ? g.L[0] - 1 : s.x - 1);
        return s.cb - s.xh + (xn >> 1);
    } else if (MU == 1) {
        return s.cb + (DIR > 0 ? (s.y == g.L[1] - 1 ? -(g.L[1] - 1) : 1) : (s.y == 0 ? g.L[1] - 1 : -1)) * g.sy;
    } else if (MU == 2) {
        return s.cb + (DIR > 0 ? (s.z == g.L[2] - 1 ? -(g.L[2] - 1) : 1) : (s.z == 0 ? g.L[2] - 1 : -1)) * g.sz;
    } else {
        return s.cb + (DIR > 0 ? (s.t == g.L[3] - 1 ? -(g.L[3] - 1) : 1) : (s.t == 0 ? g.L[3] - 1 : -1)) * g.st;
    }
}

// full lexicographic index of a site
__device__ __forceinline__ uint64_t lex_of(const Geom &g, const Site &s)
{
    return (uint64_t)s.x + (uint64_t)g.L[0] * ((uint64_t)s.y + (uint64_t)g.L[1] * ((uint64_t)s.z + (uint64_t)g.L[2] * s.t));
}

// ---------------------------------------------------------------------------
// Half-precision helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float f)
{
    // round to nearest even (inputs here are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float h16_to_f(uint16_t h)
{
    _Float16 v;
    __builtin_memcpy(&v, &h, 2);
    return (float)v;
}
__device__ __forceinline__ uint16_t f_to_h16(float f)
{
    _Float16 v = (_Float16)f;
    uint16_t h;
    __builtin_memcpy(&h, &v, 2);
    return h;
}

template <int P>
struct Real {
    using T = float;
};
template <>
struct Real<P64> {
    using T = double;
};

// ---------------------------------------------------------------------------
// Spinor storage.  One field = the sites of one parity of one right-hand side.
//   P64: 12 double2 components, component k at [k][Vh]
//   P32: 6 float4 groups at [g][Vh]
//   P16/PBF: 3 groups of 8 halves at [g][Vh] (uint4), then float scale[Vh]
// ---------------------------------------------------------------------------
template <int P>
struct SpinorIO;

// 16- and 4-byte global stores; NT marks them non-temporal (streamed past
// the caches), for outputs no kernel of the same pass reads again.
typedef unsigned int tm_u32x4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ void st16(void *p, tm_u32x4 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, (tm_u32x4 *)p);
    else *(tm_u32x4 *)p = v;
}
template <bool NT>
__device__ __forceinline__ void st4(void *p, uint32_t v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, (uint32_t *)p);
    else *(uint32_t *)p = v;
}
template <bool NT, class V>
__device__ __forceinline__ void st16v(void *p, const V &v)
{
    tm_u32x4 u;
    __builtin_memcpy(&u, &v, 16);
    st16<NT>(p, u);
}

template <>
struct SpinorIO<P64> {
    static constexpr size_t bytes_per_site = 192;
    template <class T>
    __device__ static __forceinline__ void load(const void *f, int vh, int i, cpx<T> v[12])
    {
        const double2 *p = (const double2 *)f;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 q = p[(size_t)k * vh + i];
            v[k] = cpx<T>{(T)q.x, (T)q.y};
        }
    }
    template <class T, bool NT = false>
    __device__ static __forceinline__ void store(void *f, int vh, int i, const cpx<T> v[12])
    {
        double2 *p = (double2 *)f;
#pragma unroll
        for (int k = 0; k < 12; k++) st16v<NT>(&p[(size_t)k * vh + i], make_double2((double)v[k].re, (double)v[k].im));
    }
};

template <>
struct SpinorIO<P32> {
    static constexpr size_t bytes_per_site = 96;
    template <class T>
    __device__ static __forceinline__ void load(const void *f, int vh, int i, cpx<T> v[12])
    {
        const float4 *p = (const float4 *)f;
#pragma unroll
        for (int g = 0; g < 6; g++) {
            float4 q = p[(size_t)g * vh + i];
            v[2 * g] = cpx<T>{(T)q.x, (T)q.y};
            v[2 * g + 1] = cpx<T>{(T)q.z, (T)q.w};
        }
    }
    template <class T, bool NT = false>
    __device__ static __forceinline__ void store(void *f, int vh, int i, const cpx<T> v[12])
    {
        float4 *p = (float4 *)f;
#pragma unroll
        for (int g = 0; g < 6; g++)
            st16v<NT>(&p[(size_t)g * vh + i], make_float4((float)v[2 * g].re, (float)v[2 * g].im,
                                                          (float)v[2 * g + 1].re, (float)v[2 * g + 1].im));
    }
};

template <int P>
struct HalfCodec;
template <>
struct HalfCodec<P16> {
    __device__ static __forceinline__ float dec(uint16_t h) { return h16_to_f(h); }
    __device__ static __forceinline__ uint16_t enc(float f) { return f_to_h16(f); }
};
template <>
struct HalfCodec<PBF> {
    __device__ static __forceinline__ float dec(uint16_t h) { return bf16_to_f(h); }
    __device__ static __forceinline__ uint16_t enc(float f) { return f_to_bf16(f); }
};

template <int P>
struct SpinorHalfIO {
    static constexpr size_t bytes_per_site = 52;
    template <class T>
    __device__ static __forceinline__ void load(const void *f, int vh, int i, cpx<T> v[12])
    {
        const uint4 *p = (const uint4 *)f;
        const float sc = ((const float *)(p + 3 * (size_t)vh))[i];
#pragma unroll
        for (int g = 0; g < 3; g++) {
            uint4 q = p[(size_t)g * vh + i];
            uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int c = 0; c < 4; c++) {
                float re = HalfCodec<P>::dec((uint16_t)(w[c] & 0xFFFFu));
                float im = HalfCodec<P>::dec((uint16_t)(w[c] >> 16));
                v[4 * g + c] = cpx<T>{(T)(re * sc), (T)(im * sc)};
            }
        }
    }
    template <class T, bool NT = false>
    __device__ static __forceinline__ void store(void *f, int vh, int i, const cpx<T> v[12])
    {
        uint4 *p = (uint4 *)f;
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < 12; k++) mx = fmaxf(mx, fmaxf(fabsf((float)v[k].re), fabsf((float)v[k].im)));
        // A site whose largest component is below the smallest normal FP32
        // number is stored as zero: 1/mx would overflow.  Such sites arise in
        // the tails of fields with exact zeros (time-diluted sources), where
        // rounding in half storage leaves residues of the spin projections
        // that shrink by orders of magnitude per Dslash application.
        if (!(mx >= 1.17549435e-38f)) mx = 0.f;
        const float inv = mx > 0.f ? 1.0f / mx : 0.f;
#pragma unroll
        for (int g = 0; g < 3; g++) {
            uint32_t w[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                uint32_t lo = HalfCodec<P>::enc((float)v[4 * g + c].re * inv);
                uint32_t hi = HalfCodec<P>::enc((float)v[4 * g + c].im * inv);
                w[c] = lo | (hi << 16);
            }
            st16<NT>(&p[(size_t)g * vh + i], tm_u32x4{w[0], w[1], w[2], w[3]});
        }
        st4<NT>(&((float *)(p + 3 * (size_t)vh))[i], __float_as_uint(mx));
    }
};
template <>
struct SpinorIO<P16> : SpinorHalfIO<P16> {};
template <>
struct SpinorIO<PBF> : SpinorHalfIO<PBF> {};

__host__ __device__ constexpr size_t spinor_site_bytes(int p) { return p == P64 ? 192 : p == P32 ? 96 : 52; }
__host__ __device__ constexpr size_t link_bytes(int p) { return p == P64 ? 96 : p == P32 ? 48 : HALF_LINK_BYTES; }

// ---------------------------------------------------------------------------
// Links.  P64/P32: first two rows (12 reals) per link, third row rebuilt as
// the complex conjugate of the cross product of the first two (det U = 1).
// P16/PBF: all nine entries (18 halves), so the half-precision hop needs no
// arithmetic to rebuild a row.
// Per precision the array is [parity 2][mu 4][group][Vh]:
//   P64: 6 double2 groups (entries 3*row+col), P32: 3 float4 (entries 2g, 2g+1),
//   P16/PBF: 2 groups of 4 packed complex halves (entries 4g..4g+3) then entry 8
//   (one packed complex) per site
// ---------------------------------------------------------------------------
template <class T>
struct Link {
    cpx<T> u[3][3];
};

template <class T>
__device__ __forceinline__ void rebuild_row2(Link<T> &L)
{
    const cpx<T> *a = L.u[0], *b = L.u[1];
    // row2 = conj(a x b): entry j = conj(a_k b_l - a_l b_k), (j, k, l) cyclic,
    // each real part one multiply and three multiply-adds
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int k = (j + 1) % 3, l = (j + 2) % 3;
        const cpx<T> p = a[k], q = b[l], r = a[l], t = b[k];
        T re = p.re * q.re, im = p.re * q.im;
        re = fma(-p.im, q.im, re);
        re = fma(-r.re, t.re, re);
        re = fma(r.im, t.im, re);
        im = fma(p.im, q.re, im);
        im = fma(-r.re, t.im, im);
        im = fma(-r.im, t.re, im);
        L.u[2][j] = cpx<T>{re, -im};
    }
}

template <int P>
struct LinkIO;

template <>
struct LinkIO<P64> {
    template <class T>
    __device__ static __forceinline__ void load(const void *G, int vh, int par, int mu, int i, Link<T> &L)
    {
        const double2 *p = (const double2 *)G + (size_t)(par * 4 + mu) * 6 * vh;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 q = p[(size_t)k * vh + i];
            L.u[k / 3][k % 3] = cpx<T>{(T)q.x, (T)q.y};
        }
        rebuild_row2(L);
    }
};
template <>
struct LinkIO<P32> {
    template <class T>
    __device__ static __forceinline__ void load(const void *G, int vh, int par, int mu, int i, Link<T> &L)
    {
        const float4 *p = (const float4 *)G + (size_t)(par * 4 + mu) * 3 * vh;
#pragma unroll
        for (int g = 0; g < 3; g++) {
            float4 q = p[(size_t)g * vh + i];
            L.u[(2 * g) / 3][(2 * g) % 3] = cpx<T>{(T)q.x, (T)q.y};
            L.u[(2 * g + 1) / 3][(2 * g + 1) % 3] = cpx<T>{(T)q.z, (T)q.w};
        }
        rebuild_row2(L);
    }
};
template <int P>
struct LinkHalfIO {
    template <class T>
    __device__ static __forceinline__ void load(const void *G, int vh, int par, int mu, int i, Link<T> &L)
    {
        const char *base = (const char *)G + (size_t)(par * 4 + mu) * HALF_LINK_BYTES * vh;
        if constexpr (TM_HALF_LINK12 != 0) {
            const uint4 q = ((const uint4 *)base)[i];
            const uint2 r = ((const uint2 *)(base + (size_t)16 * vh))[i];
            const uint32_t w[6] = {q.x, q.y, q.z, q.w, r.x, r.y};
#pragma unroll
            for (int k = 0; k < 6; k++)
                L.u[k / 3][k % 3] = cpx<T>{(T)HalfCodec<P>::dec(w[k] & 0xFFFFu), (T)HalfCodec<P>::dec(w[k] >> 16)};
            rebuild_row2(L);
            return;
        }
        uint32_t w[9];
#pragma unroll
        for (int g = 0; g < 2; g++) {
            const uint4 q = ((const uint4 *)base)[(size_t)g * vh + i];
            w[4 * g] = q.x;
            w[4 * g + 1] = q.y;
            w[4 * g + 2] = q.z;
            w[4 * g + 3] = q.w;
        }
        w[8] = ((const uint32_t *)(base + (size_t)32 * vh))[i];
#pragma unroll
        for (int k = 0; k < 9; k++)
            L.u[k / 3][k % 3] = cpx<T>{(T)HalfCodec<P>::dec(w[k] & 0xFFFFu), (T)HalfCodec<P>::dec(w[k] >> 16)};
    }
};
template <>
struct LinkIO<P16> : LinkHalfIO<P16> {};
template <>
struct LinkIO<PBF> : LinkHalfIO<PBF> {};

// U h and U^dagger h for colour 3-vectors
template <class T>
__device__ __forceinline__ void umul(const Link<T> &L, const cpx<T> h[3], cpx<T> o[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) o[a] = cmul(L.u[a][0], h[0]) + cmul(L.u[a][1], h[1]) + cmul(L.u[a][2], h[2]);
}
template <class T>
__device__ __forceinline__ void udagmul(const Link<T> &L, const cpx<T> h[3], cpx<T> o[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) o[a] = cmulc(L.u[0][a], h[0]) + cmulc(L.u[1][a], h[1]) + cmulc(L.u[2][a], h[2]);
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the Z4 code of a site: 24 bits,
// bit 2k = sign of Re eta_k, bit 2k+1 = sign of Im eta_k, k = 3*spin+colour.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t philox_w0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1)
{
    const uint64_t MA = 0xD2E7470EE14C6C93ull, MB = 0xCA5A826395121157ull;
    const uint64_t WA = 0x9E3779B97F4A7C15ull, WB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint64_t hA = __umul64hi(MA, c0), lA = MA * c0;
        const uint64_t hB = __umul64hi(MB, c2), lB = MB * c2;
        const uint64_t n0 = hB ^ c1 ^ k0, n2 = hA ^ c3 ^ k1;
        c0 = n0;
        c1 = lB;
        c2 = n2;
        c3 = lA;
        k0 += WA;
        k1 += WB;
    }
    return c0;
}

__device__ __forceinline__ uint32_t z4_code(uint64_t lex, uint64_t src, uint64_t seed)
{
    return (uint32_t)(philox_w0(lex, src, 0, 0, seed, 0) & 0xFFFFFFull);
}

// A code with this bit set is a site where the source is zero (a time-diluted
// source outside its timeslices); the 24 noise bits are kept.
constexpr uint32_t Z4_ZERO = 0x80000000u;

// unscaled eta component k: (+-1, +-1), or 0 at a zero site; multiply by
// 2^-1/2 for the value
template <class T>
__device__ __forceinline__ cpx<T> z4_unscaled(uint32_t code, int k)
{
    const T u = (code & Z4_ZERO) ? (T)0 : (T)1;
    return cpx<T>{((code >> (2 * k)) & 1u) ? -u : u, ((code >> (2 * k + 1)) & 1u) ? -u : u};
}

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed order; every lane ends with the same sum).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a block of NT threads; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds /* NT/64 doubles */)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (NT > 64) {
        if (l == 0) lds[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0;
#pragma unroll
            for (int k = 0; k < NT / 64; k++) s += lds[k];
            v = s;
        }
        __syncthreads();
    }
    return v;
}

// XCD-aware block mapping.  Consecutive hardware block ids are dealt out to
// the 8 XCDs in turn; remap so that each XCD walks a contiguous range of
// (site block, slot) pairs, slots of the same site block back to back, so
// the links and neighbour spinors of a range stay in that XCD's L2.
// gouter: slot (group) index slowest instead of fastest
__device__ __forceinline__ bool map_block(int nblk_site, int nslot, int swz, int &sblk, int &slot,
                                          bool gouter = false)
{
    const int total = nblk_site * nslot;
    const int bid = blockIdx.x;
    int l = bid;
    if (swz) {
        const int per = (total + 7) >> 3;
        l = (bid & 7) * per + (bid >> 3);
    }
    if (l >= total) return false;
    if (gouter) {
        slot = l / nblk_site;
        sblk = l - slot * nblk_site;
    } else {
        sblk = l / nslot;
        slot = l - sblk * nslot;
    }
    return true;
}

}  // namespace tmk
