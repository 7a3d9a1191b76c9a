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

namespace tmk {

// Half-spinor projection for (1 + S g_mu) in the chiral basis.
// psi[3*spin + colour]; h[0..2] = row 0, h[3..5] = row 1.
template <class T, int MU, int S>
__device__ __forceinline__ void project(const cpx<T> psi[12], cpx<T> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cpx<T> p0 = psi[c], p1 = psi[3 + c], p2 = psi[6 + c], p3 = psi[9 + c];
        if (MU == 0) {  // rows: p0 - iS p3, p1 - iS p2
            h[c] = S > 0 ? p0 - ti(p3) : p0 + ti(p3);
            h[3 + c] = S > 0 ? p1 - ti(p2) : p1 + ti(p2);
        } else if (MU == 1) {  // p0 - S p3, p1 + S p2
            h[c] = S > 0 ? p0 - p3 : p0 + p3;
            h[3 + c] = S > 0 ? p1 + p2 : p1 - p2;
        } else if (MU == 2) {  // p0 - iS p2, p1 + iS p3
            h[c] = S > 0 ? p0 - ti(p2) : p0 + ti(p2);
            h[3 + c] = S > 0 ? p1 + ti(p3) : p1 - ti(p3);
        } else {  // p0 + S p2, p1 + S p3
            h[c] = S > 0 ? p0 + p2 : p0 - p2;
            h[3 + c] = S > 0 ? p1 + p3 : p1 - p3;
        }
    }
}

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

template <class T, int SP, int MU, bool DAG>
__device__ __forceinline__ void hop_mu(const DslashArgs &A, const Site &s, const char *in, cpx<T> acc[12])
{
    const int vh = A.g.vh;
    {  // forward neighbour, projector (1 - g_mu) [ (1 + g_mu) for DAG ]
        constexpr int S = DAG ? 1 : -1;
        const int nf = nbr<MU, 1>(A.g, s);
        cpx<T> psi[12], h[6], w[6];
        SpinorIO<SP>::load(in, vh, nf, psi);
        project<T, MU, S>(psi, h);
        Link<T> L;
        LinkIO<SP>::load(A.gauge, vh, A.out_par, MU, s.cb, L);
        umul(L, h, w);
        umul(L, h + 3, w + 3);
        if (MU == 3 && A.g.tbc < 0 && s.t == A.g.L[3] - 1) {
#pragma unroll
            for (int k = 0; k < 6; k++) w[k] = cpx<T>{-w[k].re, -w[k].im};
        }
        accum<T, MU, S>(acc, w);
    }
    {  // backward neighbour, projector (1 + g_mu) [ (1 - g_mu) for DAG ]
        constexpr int S = DAG ? -1 : 1;
        const int nb = nbr<MU, -1>(A.g, s);
        cpx<T> psi[12], h[6], w[6];
        SpinorIO<SP>::load(in, vh, nb, psi);
        project<T, MU, S>(psi, h);
        Link<T> L;
        LinkIO<SP>::load(A.gauge, vh, 1 - A.out_par, MU, nb, L);
        udagmul(L, h, w);
        udagmul(L, h + 3, w + 3);
        if (MU == 3 && A.g.tbc < 0 && s.t == 0) {
#pragma unroll
            for (int k = 0; k < 6; k++) w[k] = cpx<T>{-w[k].re, -w[k].im};
        }
        accum<T, MU, S>(acc, w);
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
        default: break;
        }
        P[c] = cpx<T>{(T)pr, (T)pi};
        Q[c] = cpx<T>{(T)qr, (T)qi};
    }
}

// SLOT: per-slot solver state (CG chunks) or uniform parameters (operator calls)
template <int SP, bool DAG, int EPI, bool IN2, bool SLOT>
__global__ __launch_bounds__(BLOCK) void k_dslash(const DslashArgs A)
{
    using T = typename Real<SP>::T;
    constexpr int XR = SP == P64 ? P64 : P32;
    __shared__ double red[BLOCK / 64];
    int sblk, slot;
    if (!map_block(A.nblk_site, A.nslot, A.swz, sblk, slot)) return;
    double kappa = A.kappa_u, a = A.a_u, alpha = 0;
    if constexpr (SLOT) {
        const SlotState &st = A.st[slot];
        if (st.status != ST_RUNNING) return;
        kappa = st.kappa;
        a = st.a;
        alpha = st.alpha;
    }
    const int vh = A.g.vh;
    const int cb = sblk * BLOCK + threadIdx.x;
    double part = 0.0;
    if (cb < vh) {
        const Site s = site_of(A.g, cb, A.out_par);
        const char *in = A.in + (size_t)slot * A.in_slot;
        cpx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = cpx<T>{(T)0, (T)0};
        hop_mu<T, SP, 0, DAG>(A, s, in, acc);
        hop_mu<T, SP, 1, DAG>(A, s, in, acc);
        hop_mu<T, SP, 2, DAG>(A, s, in, acc);
        hop_mu<T, SP, 3, DAG>(A, s, in, acc);
        cpx<T> P[2], Q[2];
        coefs<T>(A.coef, kappa, a, P, Q);
        cpx<T> v[12];
        if (IN2) {
            cpx<T> y[12];
            SpinorIO<SP>::load(A.in2 + (size_t)slot * A.in2_slot, vh, cb, y);
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = cmul(P[k / 6], y[k]) + cmul(Q[k / 6], acc[k]);
        } else {
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = cmul(Q[k / 6], acc[k]);
        }
        if (EPI == EPI_PLAIN || EPI == EPI_NORM) {
            SpinorIO<SP>::store(A.out + (size_t)slot * A.out_slot, vh, cb, v);
            if (EPI == EPI_NORM) {
#pragma unroll
                for (int k = 0; k < 12; k++) part += (double)norm2(v[k]);
            }
        } else if (EPI == EPI_CGUPD) {
            cpx<T> p[12], x[12], r[12];
            SpinorIO<SP>::load(A.p + (size_t)slot * A.p_slot, vh, cb, p);
            char *xs = A.x + (size_t)slot * A.xr_slot;
            char *rs = A.r + (size_t)slot * A.xr_slot;
            SpinorIO<XR>::load(xs, vh, cb, x);
            SpinorIO<XR>::load(rs, vh, cb, r);
            const T al = (T)alpha;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                x[k] = x[k] + cscale(al, p[k]);
                r[k] = r[k] - cscale(al, v[k]);
                part += (double)norm2(r[k]);
            }
            SpinorIO<XR>::store(xs, vh, cb, x);
            SpinorIO<XR>::store(rs, vh, cb, r);
        } else {  // EPI_RESID (FP64 only)
            cpx<T> b[12];
            SpinorIO<P64>::load(A.b + (size_t)slot * A.b_slot, vh, cb, b);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                v[k] = b[k] - v[k];
                part += (double)norm2(v[k]);
            }
            SpinorIO<SP>::store(A.out + (size_t)slot * A.out_slot, vh, cb, v);
        }
    }
    if (EPI != EPI_PLAIN) {
        part = block_sum<BLOCK>(part, red);
        if (threadIdx.x == 0) A.partial[(size_t)slot * A.nblk_site + sblk] = part;
    }
}

template <int SP, bool DAG, int EPI, bool IN2>
static void launch_t(const DslashArgs &A, hipStream_t s)
{
    const int total = A.nblk_site * A.nslot;
    const int grid = A.swz ? 8 * ((total + 7) / 8) : total;
    if (A.st)
        hipLaunchKernelGGL((k_dslash<SP, DAG, EPI, IN2, true>), dim3(grid), dim3(BLOCK), 0, s, A);
    else
        hipLaunchKernelGGL((k_dslash<SP, DAG, EPI, IN2, false>), dim3(grid), dim3(BLOCK), 0, s, A);
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

int launch_dslash(int sp, bool dag, int epi, bool in2, const DslashArgs &A, hipStream_t s)
{
    if (A.nslot < 1 || A.nblk_site < 1) return 0;
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
