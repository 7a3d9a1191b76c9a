// Z4 noise from a counter-based generator, loop contractions at every
// timeslice, projection onto the local / one-derivative insertions and the
// truncated-solver combination.
#include "tm_dev.h"
#include "tm_launch.h"

namespace tmk {

// ---------------------------------------------------------------------------
// Z4 noise
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_z4_codes(Geom g, uint64_t seed, uint64_t src, uint32_t *codes)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    const int par = blockIdx.y;
    if (cb >= g.vh) return;
    const Site s = site_of(g, cb, par);
    codes[(size_t)par * g.vh + cb] = z4_code(lex_of(g, s), src, seed);
}

void launch_z4_codes(const Geom &g, uint64_t seed, uint64_t src, uint32_t *codes, hipStream_t s)
{
    hipLaunchKernelGGL(k_z4_codes, dim3(nblk_of(g), 2), dim3(BLOCK), 0, s, g, seed, src, codes);
}

__global__ __launch_bounds__(BLOCK) void k_z4_codes_n(Geom g, Z4Sources Z, uint32_t *codes)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    const int par = blockIdx.y & 1, i = blockIdx.y >> 1;
    if (cb >= g.vh) return;
    const Site s = site_of(g, cb, par);
    uint32_t c = z4_code(lex_of(g, s), Z.src[i], Z.seed[i]);
    // time dilution: the source lives on the timeslices t = tph mod tmod only
    if (Z.tmod[i] > 0 && s.t % Z.tmod[i] != Z.tph[i]) c |= Z4_ZERO;
    codes[((size_t)i * 2 + par) * g.vh + cb] = c;
}

void launch_z4_codes(const Geom &g, const Z4Sources &Z, int n, uint32_t *codes, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_z4_codes_n, dim3(nblk_of(g), 2 * n), dim3(BLOCK), 0, s, g, Z, codes);
}

#define TM_RSQRT2 0.70710678118654752440

__global__ __launch_bounds__(BLOCK) void k_z4_field(Geom g, const uint32_t *codes, int ainv, double a, char *out)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.vh) return;
    const uint32_t c = codes[cb];
    cpx<double> v[12];
    const double den = 1.0 / (1.0 + a * a);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        cpx<double> e = z4_unscaled<double>(c, k);
        e = cpx<double>{e.re * TM_RSQRT2, e.im * TM_RSQRT2};
        if (ainv) {
            const double ch = k < 6 ? 1.0 : -1.0;
            e = cmul(cpx<double>{den, -ch * a * den}, e);
        }
        v[k] = e;
    }
    SpinorIO<P64>::store(out, g.vh, cb, v);
}

void launch_z4_field(const Geom &g, const uint32_t *codes_par, int ainv, double a, char *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_z4_field, dim3(nblk_of(g)), dim3(BLOCK), 0, s, g, codes_par, ainv, a, out);
}

__global__ __launch_bounds__(BLOCK) void k_z4_canonical(Geom g, uint64_t seed, uint64_t src, double *out)
{
    const size_t lex = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (lex >= (size_t)2 * g.vh) return;
    const uint32_t c = z4_code(lex, src, seed);
    double2 *o = (double2 *)out + 12 * lex;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const cpx<double> e = z4_unscaled<double>(c, k);
        o[k] = make_double2(e.re * TM_RSQRT2, e.im * TM_RSQRT2);
    }
}

void launch_z4_canonical(const Geom &g, uint64_t seed, uint64_t src, double *out, hipStream_t s)
{
    const size_t v = (size_t)2 * g.vh;
    hipLaunchKernelGGL(k_z4_canonical, dim3((unsigned)((v + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, g, seed, src,
                       out);
}

// ---------------------------------------------------------------------------
// Contractions.  A block owns a chunk of CPB sites of one timeslice (sites
// of parity 0, then parity 1, each in cb order) for one source.  Each kind
// of spin matrix has a one-wave block of its own (the nine blocks of a chunk
// and source are consecutive, so they run together on one XCD and the other
// kinds find a site's solution, links and codes in its L2); single-wave
// blocks fill the four SIMDs of a CU evenly and fit beside the Dslash blocks
// of a concurrent stream.  Each lane
// accumulates its sites, the wave reduces in a fixed order and writes one
// partial per (timeslice, chunk, kind); a second kernel sums the chunks of
// each timeslice in order and applies one complex factor.
//   kind 0:      P_ab  = sum conj(l_a) . s_b
//   kind 1+nu:   F_ab  = sum conj(l_a(x)) . [U_nu(x) s(x+nu)]_b
//   kind 5+nu:   B_ab  = sum conj([U_nu(x) l(x+nu)]_a) . s_b(x)
// The left vector l is the noise from its Z4 codes (unscaled +-1 +- i; factor
// 2^-1/2), or, for the one-end trick, a field: the solution itself (factor
// -2ia, isovector) with s the solution or D_W applied to it (factor 2).
// ---------------------------------------------------------------------------
// waves per SIMD the register allocation of the FP32 kinds must allow
#ifndef TM_CONTRACT_WAVES
#define TM_CONTRACT_WAVES 3
#endif
constexpr int SPT = 16;        // sites per lane (amortises the wave reductions)
constexpr int CPB = 64 * SPT;  // sites per block

int contract_nchunk(const Geom &g) { return (2 * g.v3h + CPB - 1) / CPB; }

// Wave sums of a lane's 32 accumulators by recursive halving: in the
// exchange over lane bit b (b = 5 down to 1) a lane keeps the half of its
// values that bit selects and adds its partner's copy of that half; then
// lanes 2i and 2i+1 hold the total of value i, and lane 2i writes it.  The
// order is fixed, so every call gives the same bits.
__device__ __forceinline__ void wave_write32(double (&v)[32], double *dst)
{
    const int l = (int)threadIdx.x & 63;
#pragma unroll
    for (int e = 4; e >= 0; e--) {
        const int h = 1 << e;  // values kept
        const bool up = (l & (2 * h)) != 0;
#pragma unroll
        for (int j = 0; j < h; j++) {
            const double send = up ? v[j] : v[j + h];
            const double keep = up ? v[j + h] : v[j];
            v[j] = keep + __shfl_xor(send, 2 * h, 64);
        }
    }
    const double tot = v[0] + __shfl_xor(v[0], 1, 64);
    if ((l & 1) == 0) dst[l >> 1] = tot;
}

__device__ __forceinline__ bool contract_site(const Geom &g, int t, int q, int &par, int &cb)
{
    if (q >= 2 * g.v3h) return false;
    par = q < g.v3h ? 0 : 1;
    cb = t * g.v3h + (q - par * g.v3h);
    return true;
}

// Arithmetic of the contraction as explicit multiply-add chains: a colour
// sum of three complex products is one multiply and five multiply-adds per
// real part (written as sums of separate products, each needs two more
// instructions).
template <class T>
__device__ __forceinline__ T tfma(T a, T b, T c)
{
    if constexpr (sizeof(T) == 8) return fma(a, b, c);
    else return fmaf(a, b, c);
}
// sum_c conj(l[c * sl]) w[c * sw], c = 0..2
template <class T>
__device__ __forceinline__ cpx<T> cdot3(const cpx<T> *l, int sl, const cpx<T> *w, int sw)
{
    T re = l[0].re * w[0].re, im = l[0].re * w[0].im;
    re = tfma(l[0].im, w[0].im, re);
    im = tfma(-l[0].im, w[0].re, im);
#pragma unroll
    for (int c = 1; c < 3; c++) {
        const cpx<T> a = l[c * sl], b = w[c * sw];
        re = tfma(a.re, b.re, re);
        re = tfma(a.im, b.im, re);
        im = tfma(a.re, b.im, im);
        im = tfma(-a.im, b.re, im);
    }
    return {re, im};
}
// o = U h (colour vectors), U's rows as multiply-add chains
template <class T>
__device__ __forceinline__ void umul_chain(const Link<T> &L, const cpx<T> h[3], cpx<T> o[3])
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const cpx<T> u0 = L.u[a][0];
        T re = u0.re * h[0].re, im = u0.re * h[0].im;
        re = tfma(-u0.im, h[0].im, re);
        im = tfma(u0.im, h[0].re, im);
#pragma unroll
        for (int b = 1; b < 3; b++) {
            const cpx<T> u = L.u[a][b];
            re = tfma(u.re, h[b].re, re);
            re = tfma(-u.im, h[b].im, re);
            im = tfma(u.re, h[b].im, im);
            im = tfma(u.im, h[b].re, im);
        }
        o[a] = {re, im};
    }
}

// One kind of spin matrix for the thread's sites, 32 FP64 accumulators:
//   KIND 0: local; KIND 1+nu: F^nu; KIND 5+nu: B^nu.
// Products in the precision of s (FP64 for HP and FP64 solves, FP32 for LP
// solves, with links of the same precision); sums always in FP64.
// left vector: Z4 codes (unscaled noise) or a field of precision SPS.  The
// antiperiodic sign of a hop across the time boundary multiplies the noise:
// for codes it flips their 24 sign bits (the code itself), for a field it
// multiplies the transported vector.
template <int SPS, bool FIELD>
struct LeftVec {
    const uint32_t *codes;
    const char *fld[2];
    // unscaled Z4 value of component k: (+-1, +-1), (0, 0) at flagged sites
    template <class T>
    __device__ static __forceinline__ T z4_part(uint32_t c, int bit, uint32_t one_hi)
    {
        const uint32_t sgn = (c << (31 - bit)) & 0x80000000u;
        if constexpr (sizeof(T) == 8) return __hiloint2double((int)(sgn | one_hi), 0);
        else return __uint_as_float(sgn | one_hi);
    }
    template <class T>
    __device__ __forceinline__ void get(const Geom &g, int par, int cb, cpx<T> l[12], bool neg = false) const
    {
        if constexpr (FIELD) {
            SpinorIO<SPS>::load(fld[par], g.vh, cb, l);
        } else {
            uint32_t c = codes[(size_t)par * g.vh + cb];
            const bool zero = (c & Z4_ZERO) != 0;
            if (neg) c ^= 0x00FFFFFFu;
            // high word of 1.0 (FP64) or its bits (FP32); zero at flagged sites
            const uint32_t one_hi = zero ? 0u : (sizeof(T) == 8 ? 0x3FF00000u : 0x3F800000u);
#pragma unroll
            for (int k = 0; k < 12; k++) l[k] = cpx<T>{z4_part<T>(c, 2 * k, one_hi), z4_part<T>(c, 2 * k + 1, one_hi)};
        }
    }
};

template <int KIND, int SPS, bool FIELD>
__device__ __forceinline__ void contract_kind(const Geom &g, const void *G, const char *s_fld[2],
                                              const LeftVec<SPS, FIELD> &left, int t, int chunk, double (&acc)[32])
{
    using T = typename Real<SPS>::T;
#pragma unroll
    for (int k = 0; k < 32; k++) acc[k] = 0.0;
    const int lane = (int)threadIdx.x & 63;
#pragma unroll 1
    for (int k = 0; k < SPT; k++) {
        int par, cb;
        if (!contract_site(g, t, chunk * CPB + k * 64 + lane, par, cb)) continue;
        if constexpr (KIND == 0) {
            cpx<T> lv[12], sv[12];
            left.get(g, par, cb, lv);
            SpinorIO<SPS>::load(s_fld[par], g.vh, cb, sv);
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const cpx<T> f = cdot3(&lv[3 * a], 1, &sv[3 * b], 1);
                    acc[2 * (4 * a + b)] += (double)f.re;
                    acc[2 * (4 * a + b) + 1] += (double)f.im;
                }
        } else {
            constexpr int NU = (KIND - 1) % 4;
            const Site s = site_of(g, cb, par);
            const int nf = nbr<NU, 1>(g, s);
            Link<T> L;
            LinkIO<SPS>::load(G, g.vh, par, NU, cb, L);
            const bool neg = NU == 3 && g.tbc < 0 && s.t == g.L[3] - 1;
            if constexpr (KIND <= 4) {
                // F: conj(l_a(x)) . (U s(x+nu))_b, the boundary sign on l
                cpx<T> lv[12], snb[12];
                left.get(g, par, cb, lv, !FIELD && neg);
                SpinorIO<SPS>::load(s_fld[1 - par], g.vh, nf, snb);
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    cpx<T> w[3];
                    umul_chain(L, &snb[3 * b], w);
                    if (FIELD && neg) {
#pragma unroll
                        for (int c = 0; c < 3; c++) w[c] = cpx<T>{-w[c].re, -w[c].im};
                    }
#pragma unroll
                    for (int a = 0; a < 4; a++) {
                        const cpx<T> f = cdot3(&lv[3 * a], 1, w, 1);
                        acc[2 * (4 * a + b)] += (double)f.re;
                        acc[2 * (4 * a + b) + 1] += (double)f.im;
                    }
                }
            } else {
                // B: conj((U l(x+nu))_a) . s_b(x), the boundary sign on l
                cpx<T> lf[12], sv[12];
                left.get(g, 1 - par, nf, lf, !FIELD && neg);
                SpinorIO<SPS>::load(s_fld[par], g.vh, cb, sv);
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    cpx<T> v[3];
                    umul_chain(L, &lf[3 * a], v);
                    if (FIELD && neg) {
#pragma unroll
                        for (int c = 0; c < 3; c++) v[c] = cpx<T>{-v[c].re, -v[c].im};
                    }
#pragma unroll
                    for (int b = 0; b < 4; b++) {
                        const cpx<T> f = cdot3(v, 1, &sv[3 * b], 1);
                        acc[2 * (4 * a + b)] += (double)f.re;
                        acc[2 * (4 * a + b) + 1] += (double)f.im;
                    }
                }
            }
        }
    }
}

// Contraction blocks: FP32 solutions take TM_CONTRACT_KPB kinds per block,
// one wave per kind (the 9 kinds in 9 / KPB blocks; measured at 32^3x64, 12
// sources: 9 kinds per block 3.70 ms, 3 kinds 3.25 ms, 1 kind 3.20 ms, same
// bits); FP64 ones one kind per single-wave block (before, one wave computed
// the nine kinds in turn: 0.99 ms per source against 0.51 ms).
#ifndef TM_CONTRACT_KPB
#define TM_CONTRACT_KPB 1
#endif
static_assert(9 % TM_CONTRACT_KPB == 0, "kinds per block must divide 9");
template <int SPS, int NK>
constexpr int contract_waves()
{
    return SPS == P32 && NK == 9 ? TM_CONTRACT_KPB : 1;
}
// blocks per source and site chunk
template <int SPS, int NK>
constexpr int contract_groups()
{
    return NK == 9 ? 9 / contract_waves<SPS, NK>() : 1;
}

// partial layout: cpart[(t * nchunk + chunk) * 288 + kind * 32 + ab * 2 + re/im]
// Logical block lb handles kind group lb mod NG of logical unit l = lb / NG,
// and l source i = l mod n of site chunk l / n: the n
// sources of a chunk run back to back on one XCD (the hardware hands block b
// to XCD b mod 8, so lb = (b mod 8) * per + b / 8 gives each XCD a contiguous
// range of logical blocks) and share the chunk's links in its L2.  The left
// vector is the source's codes (FIELD false) or the field pair
// (l_even, l_odd) + i * l_stride; NK = 9 (all kinds) or 1 (local only).
template <int SPS, bool FIELD, int NK>
__global__ __launch_bounds__((64 * contract_waves<SPS, NK>()), (SPS == P32 && NK == 9 ? TM_CONTRACT_WAVES : 2))
void k_contract(Geom g, const void *G, const char *s_even, const char *s_odd, size_t s_stride, const char *l_even,
                const char *l_odd, size_t l_stride, const uint32_t *codes, double *cpart, int nchunk,
                size_t part_stride, int n, int total)
{
    constexpr int NG = contract_groups<SPS, NK>();
    const int per = (total + 7) >> 3;
    const int lb = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (lb >= total) return;  // uniform over the block
    const int kg = lb % NG, l = lb / NG;
    const int i = l % n, tc = l / n;
    const int t = tc / nchunk, chunk = tc - t * nchunk;
    const char *s_fld[2] = {s_even + (size_t)i * s_stride, s_odd + (size_t)i * s_stride};
    LeftVec<SPS, FIELD> left;
    left.codes = FIELD ? nullptr : codes + (size_t)i * 2 * g.vh;
    left.fld[0] = FIELD ? l_even + (size_t)i * l_stride : nullptr;
    left.fld[1] = FIELD ? l_odd + (size_t)i * l_stride : nullptr;
    double *dst = cpart + (size_t)i * part_stride + (size_t)tc * 288;
    double acc[32];
#define TMK_KIND(K)                                                     \
    contract_kind<K, SPS, FIELD>(g, G, s_fld, left, t, chunk, acc);     \
    wave_write32(acc, dst + (K) * 32);
    if constexpr (NK == 1) {
        TMK_KIND(0)
    } else {
        // wave w of group kg computes kind kg * waves + w
        switch (__builtin_amdgcn_readfirstlane(kg * contract_waves<SPS, NK>() + ((int)threadIdx.x >> 6))) {
        case 0: TMK_KIND(0) break;
        case 1: TMK_KIND(1) break;
        case 2: TMK_KIND(2) break;
        case 3: TMK_KIND(3) break;
        case 4: TMK_KIND(4) break;
        case 5: TMK_KIND(5) break;
        case 6: TMK_KIND(6) break;
        case 7: TMK_KIND(7) break;
        default: TMK_KIND(8) break;
        }
    }
#undef TMK_KIND
}

// raw[kind][t][ab] = (sr + i si) * sum_chunk cpart[t][chunk][kind][ab] (complex) for the
// first nk kinds; blockIdx.y = source
__global__ void k_contract_final(const double *cpart, int nchunk, int lt, RawOuts R, size_t part_stride, double sr,
                                 double si, int nk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over lt * nk * 16 complex entries
    if (i >= lt * nk * 16) return;
    cpart += (size_t)blockIdx.y * part_stride;
    double *raw = R.p[blockIdx.y];
    const int t = i / (nk * 16), e = 2 * (i - t * nk * 16);
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nchunk; c++) {
        re += cpart[((size_t)t * nchunk + c) * 288 + e];
        im += cpart[((size_t)t * nchunk + c) * 288 + e + 1];
    }
    const int kind = e / 32, ab = e - kind * 32;
    raw[((size_t)kind * lt + t) * 32 + ab] = re * sr - im * si;
    raw[((size_t)kind * lt + t) * 32 + ab + 1] = re * si + im * sr;
}

size_t contract_part_doubles(const Geom &g) { return (size_t)g.L[3] * contract_nchunk(g) * 288; }

template <bool FIELD, int NK = 9>
static void contract_t(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                       size_t s_stride, const char *l_even, const char *l_odd, size_t l_stride,
                       const uint32_t *codes, double *cpart, const RawOuts &raw, int n, double sr, double si,
                       hipStream_t s)
{
    if (n < 1) return;
    const int nchunk = contract_nchunk(g);
    const int lt = g.L[3];
    const size_t ps = contract_part_doubles(g);
    const int total = lt * nchunk * n * (sps == P32 ? contract_groups<P32, NK>() : contract_groups<P64, NK>());
    const unsigned nb = (unsigned)(8 * ((total + 7) / 8));
    if (sps == P32)
        hipLaunchKernelGGL((k_contract<P32, FIELD, NK>), dim3(nb), dim3(64 * contract_waves<P32, NK>()), 0, s, g,
                           gauge, s_even, s_odd, s_stride, l_even, l_odd, l_stride, codes, cpart, nchunk, ps, n,
                           total);
    else
        hipLaunchKernelGGL((k_contract<P64, FIELD, NK>), dim3(nb), dim3(64 * contract_waves<P64, NK>()), 0, s, g,
                           gauge, s_even, s_odd, s_stride, l_even, l_odd, l_stride, codes, cpart, nchunk, ps, n,
                           total);
    const int m = lt * NK * 16;
    hipLaunchKernelGGL(k_contract_final, dim3((m + 255) / 256, n), dim3(256), 0, s, cpart, nchunk, lt, raw, ps, sr,
                       si, NK);
}

void launch_contract(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                     size_t s_stride, const uint32_t *codes, double *cpart, const RawOuts &raw, int n, hipStream_t s)
{
    contract_t<false>(sps, g, gauge, s_even, s_odd, s_stride, nullptr, nullptr, 0, codes, cpart, raw, n, TM_RSQRT2,
                      0.0, s);
}

void launch_contract(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                     const uint32_t *codes, double *cpart, double *raw_out, hipStream_t s)
{
    RawOuts R{};
    R.p[0] = raw_out;
    launch_contract(sps, g, gauge, s_even, s_odd, 0, codes, cpart, R, 1, s);
}

void launch_contract_lr(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                        size_t s_stride, const char *l_even, const char *l_odd, size_t l_stride, double *cpart,
                        const RawOuts &raw, int n, double sr, double si, hipStream_t s, bool local_only)
{
    if (local_only)
        contract_t<true, 1>(sps, g, gauge, s_even, s_odd, s_stride, l_even, l_odd, l_stride, nullptr, cpart, raw, n,
                            sr, si, s);
    else
        contract_t<true>(sps, g, gauge, s_even, s_odd, s_stride, l_even, l_odd, l_stride, nullptr, cpart, raw, n, sr,
                         si, s);
}

void launch_contract_local(int sps, const Geom &g, const char *s_even, const char *s_odd, size_t s_stride,
                           const uint32_t *codes, double *cpart, const RawOuts &raw, int n, hipStream_t s)
{
    contract_t<false, 1>(sps, g, nullptr, s_even, s_odd, s_stride, nullptr, nullptr, 0, codes, cpart, raw, n,
                         TM_RSQRT2, 0.0, s);
}

// ---------------------------------------------------------------------------
// Exact part of the hopping parameter expansion (Sec. 2.4, Eq. HPE) as local
// spin matrices raw[0][t][a][b] (kinds 1..8 untouched): the site-diagonal
// blocks of B - BHB + (BH)^2 B - (BH)^3 B summed over a timeslice and colour.
// With B = b0 + b5 g5 (b5 = -i a / (1 + a^2)) and H = -kappa D_hop: odd
// powers of H never return to a site of a lattice with even extents; the two
// ways of returning in two hops along +-mu give (1 -+ g_mu) B (1 +- g_mu)
// kappa^2 = 2 kappa^2 b5 g5 (1 +- g_mu), which sum over mu to 16 kappa^2 b5 g5,
// independent of the links.  So the block is diag_b(B_b + 16 kappa^2 b5 e_b
// B_b^2) times 3 V3, B_b = 1/(1 + i a e_b), e_b = g5's eigenvalue on spin b.
// ---------------------------------------------------------------------------
__global__ void k_hpe_exact(int lt, double v3, double kappa, double a, double *raw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over lt * 16 entries
    if (i >= lt * 16) return;
    const int ab = i & 15, al = ab >> 2, be = ab & 3;
    double re = 0.0, im = 0.0;
    if (al == be) {
        const double e = be < 2 ? 1.0 : -1.0, den = 1.0 / (1.0 + a * a);
        const double br = den, bi = -e * a * den;                       // B_b
        const double b2r = br * br - bi * bi, b2i = 2.0 * br * bi;      // B_b^2
        const double cr = 0.0, ci = -16.0 * kappa * kappa * a * den * e;  // 16 kappa^2 b5 e_b
        re = 3.0 * v3 * (br + cr * b2r - ci * b2i);
        im = 3.0 * v3 * (bi + cr * b2i + ci * b2r);
    }
    raw[2 * i] = re;
    raw[2 * i + 1] = im;
}

void launch_hpe_exact(const Geom &g, double kappa, double a, double *raw, hipStream_t s)
{
    const int lt = g.L[3];
    hipLaunchKernelGGL(k_hpe_exact, dim3((lt * 16 + 255) / 256), dim3(256), 0, s, lt,
                       (double)g.L[0] * g.L[1] * g.L[2], kappa, a, raw);
}

// ---------------------------------------------------------------------------
// Projection: ops[n][op][t][2] from raw[n][kind][t][16][2].
//   op g < 16:        sum_a phase(g,a) * P[a][col(g,a)]
//   op 16 + 4g + nu:  1/4 [F(t) + F(t-d) - B(t) - B(t-d)], d = (nu == 3)
//   op 80 + i:        (L^D_{g_m, n} + L^D_{g_n, m}) / 2 over m <= n
// ---------------------------------------------------------------------------
struct GammaTab {
    int e[16][4];
};

__device__ __forceinline__ cpx<double> gproj(const GammaTab &G, int gi, const double *m)
{
    // sum_a phase(a) * P[a][col(a)], phase = i^ph
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int e = G.e[gi][a];
        const int col = e & 3, ph = (e >> 2) & 3;
        const double vr = m[2 * (4 * a + col)], vi = m[2 * (4 * a + col) + 1];
        const double cr = ph == 0 ? 1.0 : ph == 2 ? -1.0 : 0.0;
        const double ci = ph == 1 ? 1.0 : ph == 3 ? -1.0 : 0.0;
        re += cr * vr - ci * vi;
        im += cr * vi + ci * vr;
    }
    return cpx<double>{re, im};
}

__device__ __forceinline__ cpx<double> deriv_op(const GammaTab &G, const double *raw, int lt, int gi, int nu,
                                                int t)
{
    const double *F = raw + ((size_t)(1 + nu) * lt) * 32;
    const double *B = raw + ((size_t)(5 + nu) * lt) * 32;
    const int tm = nu == 3 ? (t == 0 ? lt - 1 : t - 1) : t;
    cpx<double> f0 = gproj(G, gi, F + (size_t)t * 32), f1 = gproj(G, gi, F + (size_t)tm * 32);
    cpx<double> b0 = gproj(G, gi, B + (size_t)t * 32), b1 = gproj(G, gi, B + (size_t)tm * 32);
    cpx<double> s = (f0 + f1) - (b0 + b1);
    return cpx<double>{0.25 * s.re, 0.25 * s.im};
}

__global__ void k_project(int n, int lt, const double *raw, double *ops, GammaTab G)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)n * 90 * lt) return;
    const int t = (int)(i % lt);
    const int op = (int)((i / lt) % 90);
    const size_t src = i / ((size_t)lt * 90);
    const double *r = raw + src * 9 * lt * 32;
    cpx<double> v;
    if (op < 16) {
        v = gproj(G, op, r + (size_t)t * 32);
    } else if (op < 80) {
        const int k = op - 16;
        v = deriv_op(G, r, lt, k / 4, k % 4, t);
    } else {
        int idx = op - 80, m = 0, nn = 0;
        for (int a = 0, c = 0; a < 4; a++)
            for (int b = a; b < 4; b++, c++)
                if (c == idx) {
                    m = a;
                    nn = b;
                }
        cpx<double> x = deriv_op(G, r, lt, 1 + m, nn, t), y = deriv_op(G, r, lt, 1 + nn, m, t);
        v = cpx<double>{0.5 * (x.re + y.re), 0.5 * (x.im + y.im)};
    }
    ops[2 * i] = v.re;
    ops[2 * i + 1] = v.im;
}

void launch_project(int n, int lt, const double *raw, double *ops, const int *gtab_host, hipStream_t s)
{
    GammaTab G;
    for (int g = 0; g < 16; g++)
        for (int a = 0; a < 4; a++) G.e[g][a] = gtab_host[4 * g + a];
    const size_t total = (size_t)n * 90 * lt;
    if (total == 0) return;
    hipLaunchKernelGGL(k_project, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, lt, raw, ops, G);
}

// ---------------------------------------------------------------------------
// TSM: est = mean(hp - lp_corr) + mean(lp_bulk); var = s^2/N of each set
// (real and imaginary parts separately, n - 1; NaN for one member).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mean_var(int n, const double *a, const double *b, size_t stride, size_t off,
                                         double m[2], double v[2])
{
    m[0] = m[1] = v[0] = v[1] = 0.0;
    if (n == 0) return;
    for (int j = 0; j < n; j++) {
        double x0 = a[j * stride + off], x1 = a[j * stride + off + 1];
        if (b) {
            x0 -= b[j * stride + off];
            x1 -= b[j * stride + off + 1];
        }
        m[0] += x0;
        m[1] += x1;
    }
    m[0] /= n;
    m[1] /= n;
    if (n < 2) {
        v[0] = v[1] = __builtin_nan("");
        return;
    }
    double s0 = 0.0, s1 = 0.0;
    for (int j = 0; j < n; j++) {
        double x0 = a[j * stride + off], x1 = a[j * stride + off + 1];
        if (b) {
            x0 -= b[j * stride + off];
            x1 -= b[j * stride + off + 1];
        }
        s0 += (x0 - m[0]) * (x0 - m[0]);
        s1 += (x1 - m[1]) * (x1 - m[1]);
    }
    v[0] = s0 / (n - 1) / n;
    v[1] = s1 / (n - 1) / n;
}

__global__ void k_tsm(int n_hp, int n_lp, int lt, const double *hp, const double *lpc, const double *lpb,
                      double *est, double *vre, double *vim, const double *add, const unsigned char *valid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over 90 * lt
    if (i >= 90 * lt) return;
    if (valid && !valid[i]) {
        est[2 * i] = est[2 * i + 1] = vre[i] = vim[i] = __builtin_nan("");
        return;
    }
    const size_t stride = (size_t)90 * lt * 2, off = (size_t)2 * i;
    double m1[2], v1[2], m2[2], v2[2];
    mean_var(n_hp, hp, lpc, stride, off, m1, v1);
    mean_var(n_lp, lpb, nullptr, stride, off, m2, v2);
    est[2 * i] = m1[0] + m2[0] + (add ? add[2 * i] : 0.0);
    est[2 * i + 1] = m1[1] + m2[1] + (add ? add[2 * i + 1] : 0.0);
    vre[i] = v1[0] + v2[0];
    vim[i] = v1[1] + v2[1];
}

void launch_tsm_combine(int n_hp, int n_lp, int lt, const double *ops_hp, const double *ops_lp_corr,
                        const double *ops_lp_bulk, double *est, double *var_re, double *var_im, hipStream_t s,
                        const double *ops_add, const unsigned char *valid)
{
    const int n = 90 * lt;
    hipLaunchKernelGGL(k_tsm, dim3((n + 127) / 128), dim3(128), 0, s, n_hp, n_lp, lt, ops_hp, ops_lp_corr,
                       ops_lp_bulk, est, var_re, var_im, ops_add, valid);
}

// out[i] = sum over k < nph, in order, of in[i * nph + k] (per elements of per doubles)
__global__ void k_sum_phases(const double *in, double *out, int n, int nph, size_t per)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (e >= per || i >= n) return;
    const double *p = in + (size_t)i * nph * per + e;
    double v = 0.0;
    for (int k = 0; k < nph; k++) v += p[(size_t)k * per];
    out[(size_t)i * per + e] = v;
}

void launch_sum_phases(const double *in, double *out, int n, int nph, size_t per, hipStream_t s)
{
    // at most 65535 noise vectors per launch (grid y)
    for (int i0 = 0; i0 < n; i0 += 65535) {
        const int m = n - i0 < 65535 ? n - i0 : 65535;
        hipLaunchKernelGGL(k_sum_phases, dim3((unsigned)((per + 255) / 256), m), dim3(256), 0, s,
                           in + (size_t)i0 * nph * per, out + (size_t)i0 * per, m, nph, per);
    }
}

}  // namespace tmk
