/*
 * Plain FP64 CPU oracle for the twisted-mass disconnected-loop hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * Style: textbook loops over lexicographic sites, full 3x3 links,
 * full 4x4 gamma matrices, C99 double complex, no even-odd storage (the
 * even-odd Schur system is expressed with parity masks on full-lattice
 * arrays).  Written to be checked against the paper by eye, not to be fast.
 *
 * Conventions (the paper is silent on all of them; readings listed in the
 * design notes):
 *   site index  lex = x + Lx*(y + Ly*(z + Lz*t)), directions mu = 0..3 = x,y,z,t
 *   spinor      [lex][spin 4][colour 3] complex
 *   gauge       [lex][mu 4][row 3][col 3] complex, U_mu(x) links x -> x+mu
 *   time BC     hops across t = Lt-1 <-> 0 carry the factor tbc (-1 antiperiodic)
 *   gammas      chiral Euclidean basis, gamma5 = g1 g2 g3 g4 = diag(1,1,-1,-1)
 *   operator    M = 1 - kappa*D_hop + i*a*gamma5 with a = 2*kappa*mu; this is
 *               the B^-1 + H split of the hopping-parameter expansion
 *               (Sec. 2.4, Eq. HPE) with B = (1 + i a gamma5)^-1, H = -kappa D_hop.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* ------------------------------------------------------------------ */
/* Gamma matrices (chiral basis).                                      */
/* ------------------------------------------------------------------ */
static cplx GAM[5][4][4]; /* 0..3 = gamma_1..gamma_4, 4 = gamma_5 */
static int gam_ready = 0;

static void init_gamma(void)
{
    if (gam_ready) return;
    memset(GAM, 0, sizeof(GAM));
    const cplx J = _Complex_I;
    /* gamma_1 */
    GAM[0][0][3] = -J; GAM[0][1][2] = -J; GAM[0][2][1] = J; GAM[0][3][0] = J;
    /* gamma_2 */
    GAM[1][0][3] = -1; GAM[1][1][2] = 1; GAM[1][2][1] = 1; GAM[1][3][0] = -1;
    /* gamma_3 */
    GAM[2][0][2] = -J; GAM[2][1][3] = J; GAM[2][2][0] = J; GAM[2][3][1] = -J;
    /* gamma_4 */
    GAM[3][0][2] = 1; GAM[3][1][3] = 1; GAM[3][2][0] = 1; GAM[3][3][1] = 1;
    /* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 (computed, not typed) */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += GAM[0][i][k] * GAM[1][k][j];
            t1[i][j] = s;
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += t1[i][k] * GAM[2][k][j];
            t2[i][j] = s;
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += t2[i][k] * GAM[3][k][j];
            GAM[4][i][j] = s;
        }
    gam_ready = 1;
}

/* Export gamma_{mu+1} (mu = 0..3) or gamma_5 (mu = 4) as [4][4][re,im]. */
void orc_gamma(int mu, double *out)
{
    init_gamma();
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            out[2 * (4 * i + j)] = creal(GAM[mu][i][j]);
            out[2 * (4 * i + j) + 1] = cimag(GAM[mu][i][j]);
        }
}

/* ------------------------------------------------------------------ */
/* Geometry.                                                           */
/* ------------------------------------------------------------------ */
static long volume(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int *L, long s, int c[4])
{
    c[0] = (int)(s % L[0]); s /= L[0];
    c[1] = (int)(s % L[1]); s /= L[1];
    c[2] = (int)(s % L[2]); s /= L[2];
    c[3] = (int)s;
}

static long index_of(const int *L, const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static int parity_of(const int *L, long s)
{
    int c[4];
    coords(L, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Neighbour of s one step in direction mu (dir = +1 or -1).  *sign is the
 * boundary factor picked up by the hop: tbc when the hop wraps in time. */
static long hop(const int *L, long s, int mu, int dir, int tbc, double *sign)
{
    int c[4];
    coords(L, s, c);
    *sign = 1.0;
    c[mu] += dir;
    if (c[mu] >= L[mu]) { c[mu] -= L[mu]; if (mu == 3) *sign = tbc; }
    if (c[mu] < 0) { c[mu] += L[mu]; if (mu == 3) *sign = tbc; }
    return index_of(L, c);
}

#define SP(f, s) ((f) + 12 * (s))          /* spinor at site s */
#define LK(U, s, mu) ((U) + 36 * (s) + 9 * (mu)) /* 3x3 link */

/* ------------------------------------------------------------------ */
/* Hopping term D_hop (Sec. 2.4: H is proportional to the hopping term). */
/* D psi(x) = sum_mu (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) */
/* ------------------------------------------------------------------ */
void orc_dhop(const int *L, int tbc, const double *Ud, const double *ind, double *outd)
{
    init_gamma();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            double sg;
            /* forward: (1 - gamma_mu) U_mu(x) psi(x+mu) */
            long sf = hop(L, s, mu, +1, tbc, &sg);
            const cplx *u = LK(U, s, mu);
            const cplx *pf = SP(in, sf);
            cplx v[4][3];
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int b = 0; b < 3; b++) t += u[3 * a + b] * pf[3 * sp + b];
                    v[sp][a] = sg * t;
                }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx g = 0;
                    for (int sq = 0; sq < 4; sq++) g += GAM[mu][sp][sq] * v[sq][a];
                    acc[sp][a] += v[sp][a] - g;
                }
            /* backward: (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) */
            long sb = hop(L, s, mu, -1, tbc, &sg);
            const cplx *ub = LK(U, sb, mu);
            const cplx *pb = SP(in, sb);
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int b = 0; b < 3; b++) t += conj(ub[3 * b + a]) * pb[3 * sp + b];
                    v[sp][a] = sg * t;
                }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx g = 0;
                    for (int sq = 0; sq < 4; sq++) g += GAM[mu][sp][sq] * v[sq][a];
                    acc[sp][a] += v[sp][a] + g;
                }
        }
        cplx *o = SP(out, s);
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) o[3 * sp + a] = acc[sp][a];
    }
}

/* (c0 + c5*gamma5) applied site-locally, optionally only on one parity
 * (par = 0 even, 1 odd, -1 all; other sites are zeroed). */
static void apply_diag(const int *L, cplx c0, cplx c5, const cplx *in, cplx *out, int par)
{
    const long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        const cplx *p = SP(in, s);
        cplx *o = SP(out, s);
        if (par >= 0 && parity_of(L, s) != par) {
            for (int k = 0; k < 12; k++) o[k] = 0;
            continue;
        }
        cplx tmp[12];
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx g = 0;
                for (int sq = 0; sq < 4; sq++) g += GAM[4][sp][sq] * p[3 * sq + a];
                tmp[3 * sp + a] = c0 * p[3 * sp + a] + c5 * g;
            }
        for (int k = 0; k < 12; k++) o[k] = tmp[k];
    }
}

static void mask_parity(const int *L, cplx *f, int par)
{
    const long V = volume(L);
    for (long s = 0; s < V; s++)
        if (parity_of(L, s) != par)
            for (int k = 0; k < 12; k++) SP(f, s)[k] = 0;
}

/* M psi = psi - kappa D psi + i a gamma5 psi  (dag = 0)
 * M^dag psi = psi - kappa D^dag psi - i a gamma5 psi, with D^dag = g5 D g5 (dag = 1).
 * The second form is the gamma5-hermiticity reading M(mu)^dag = g5 M(-mu) g5. */
void orc_apply_M(const int *L, int tbc, const double *U, double kappa, double a, int dag,
                 const double *ind, double *outd)
{
    init_gamma();
    const long V = volume(L);
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    cplx *t = malloc(sizeof(cplx) * 12 * V);
    cplx *d = malloc(sizeof(cplx) * 12 * V);
    if (!dag) {
        orc_dhop(L, tbc, U, (const double *)in, (double *)d);
        apply_diag(L, 1.0, _Complex_I * a, in, t, -1);
        for (long k = 0; k < 12 * V; k++) out[k] = t[k] - kappa * d[k];
    } else {
        /* g5 M(-a) g5 */
        cplx *g = malloc(sizeof(cplx) * 12 * V);
        apply_diag(L, 0.0, 1.0, in, g, -1);
        orc_dhop(L, tbc, U, (const double *)g, (double *)d);
        apply_diag(L, 1.0, -_Complex_I * a, g, t, -1);
        for (long k = 0; k < 12 * V; k++) t[k] = t[k] - kappa * d[k];
        apply_diag(L, 0.0, 1.0, t, out, -1);
        free(g);
    }
    free(t);
    free(d);
}

/* ------------------------------------------------------------------ */
/* Even-odd Schur complement on the even sublattice.                    */
/*   M = [[A, -k D_eo], [-k D_oe, A]],  A = 1 + i a g5,                 */
/*   Mhat = A - k^2 D_eo A^-1 D_oe,  A^-1 = (1 - i a g5)/(1 + a^2).     */
/*   Mhat^dag = g5 Mhat(-a) g5.                                         */
/* Fields are full-lattice arrays whose odd sites are zero.             */
/* ------------------------------------------------------------------ */
static void mhat_plain(const int *L, int tbc, const double *U, double kappa, double a,
                       const cplx *in, cplx *out, cplx *w1, cplx *w2)
{
    const double den = 1.0 + a * a;
    /* w1 = D (in restricted to even) -> odd part */
    memcpy(w2, in, sizeof(cplx) * 12 * volume(L));
    mask_parity(L, w2, 0);
    orc_dhop(L, tbc, U, (const double *)w2, (double *)w1);
    /* w2 = A^-1 w1 on odd sites */
    apply_diag(L, 1.0 / den, -_Complex_I * a / den, w1, w2, 1);
    /* w1 = D w2 -> even part */
    orc_dhop(L, tbc, U, (const double *)w2, (double *)w1);
    /* out_e = A in_e - k^2 w1_e */
    apply_diag(L, 1.0, _Complex_I * a, in, w2, 0);
    const long V = volume(L);
    for (long s = 0; s < V; s++) {
        int ev = parity_of(L, s) == 0;
        for (int k = 0; k < 12; k++)
            SP(out, s)[k] = ev ? SP(w2, s)[k] - kappa * kappa * SP(w1, s)[k] : 0;
    }
}

void orc_apply_mhat(const int *L, int tbc, const double *U, double kappa, double a, int dag,
                    const double *ind, double *outd)
{
    init_gamma();
    const long V = volume(L);
    cplx *w1 = malloc(sizeof(cplx) * 12 * V);
    cplx *w2 = malloc(sizeof(cplx) * 12 * V);
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    if (!dag) {
        mhat_plain(L, tbc, (const double *)U, kappa, a, in, out, w1, w2);
    } else {
        cplx *g = malloc(sizeof(cplx) * 12 * V);
        cplx *h = malloc(sizeof(cplx) * 12 * V);
        apply_diag(L, 0.0, 1.0, in, g, 0);
        mhat_plain(L, tbc, U, kappa, -a, g, h, w1, w2);
        apply_diag(L, 0.0, 1.0, h, out, 0);
        free(g);
        free(h);
    }
    free(w1);
    free(w2);
}

static double dot_re(long n, const cplx *a, const cplx *b) /* Re <a,b> */
{
    double s = 0;
    for (long k = 0; k < n; k++) s += creal(conj(a[k]) * b[k]);
    return s;
}

/* Conjugate gradient on Mhat^dag Mhat x = Mhat^dag bhat (CG normal equations).
 * Zero initial guess.  Stops when |r_k| <= tol*|Mhat^dag bhat| or after
 * max_iter iterations; with fixed_iters > 0 it runs exactly that many
 * iterations instead (tol and max_iter ignored).  The residual r is the one
 * carried by the CG recursion.  Returns the iteration count. */
int orc_cg_eo(const int *L, int tbc, const double *U, double kappa, double a,
              const double *bhatd, double *xd, double tol, int max_iter, int fixed_iters,
              double *relres_out)
{
    init_gamma();
    const long V = volume(L), n = 12 * V;
    cplx *rhs = malloc(sizeof(cplx) * n), *r = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *u = malloc(sizeof(cplx) * n);
    cplx *ap = malloc(sizeof(cplx) * n);
    cplx *x = (cplx *)xd;
    orc_apply_mhat(L, tbc, U, kappa, a, 1, bhatd, (double *)rhs);
    for (long k = 0; k < n; k++) { x[k] = 0; r[k] = rhs[k]; p[k] = rhs[k]; }
    double rr = dot_re(n, r, r);
    const double rr0 = rr;
    int it = 0;
    if (rr0 > 0) {
        for (;;) {
            if (fixed_iters > 0) {
                if (it >= fixed_iters) break;
            } else {
                if (it >= max_iter) break;
            }
            orc_apply_mhat(L, tbc, U, kappa, a, 0, (const double *)p, (double *)u);
            orc_apply_mhat(L, tbc, U, kappa, a, 1, (const double *)u, (double *)ap);
            double pap = dot_re(n, u, u);
            double alpha = rr / pap;
            for (long k = 0; k < n; k++) { x[k] += alpha * p[k]; r[k] -= alpha * ap[k]; }
            double rr_new = dot_re(n, r, r);
            it++;
            if (fixed_iters <= 0 && rr_new <= tol * tol * rr0) { rr = rr_new; break; }
            double beta = rr_new / rr;
            for (long k = 0; k < n; k++) p[k] = r[k] + beta * p[k];
            rr = rr_new;
        }
    }
    if (relres_out) *relres_out = rr0 > 0 ? sqrt(rr / rr0) : 0.0;
    free(rhs); free(r); free(p); free(u); free(ap);
    return it;
}

/* Full solve M s = eta through the even-odd Schur system:
 *   bhat_e = eta_e + k D_eo A^-1 eta_o;  CG for s_e;
 *   s_o = A^-1 (eta_o + k D_oe s_e).
 * true_rel_out gets |eta - M s| / |eta| in FP64. */
int orc_solve(const int *L, int tbc, const double *U, double kappa, double a,
              const double *etad, double *sd, double tol, int max_iter, int fixed_iters,
              double *relres_out, double *true_rel_out)
{
    init_gamma();
    const long V = volume(L), n = 12 * V;
    const double den = 1.0 + a * a;
    const cplx *eta = (const cplx *)etad;
    cplx *s = (cplx *)sd;
    cplx *w1 = malloc(sizeof(cplx) * n), *w2 = malloc(sizeof(cplx) * n);
    cplx *bh = malloc(sizeof(cplx) * n), *xe = malloc(sizeof(cplx) * n);
    /* bhat */
    apply_diag(L, 1.0 / den, -_Complex_I * a / den, eta, w1, 1);
    orc_dhop(L, tbc, U, (const double *)w1, (double *)w2);
    for (long q = 0; q < V; q++) {
        int ev = parity_of(L, q) == 0;
        for (int k = 0; k < 12; k++) SP(bh, q)[k] = ev ? SP(eta, q)[k] + kappa * SP(w2, q)[k] : 0;
    }
    int it = orc_cg_eo(L, tbc, U, kappa, a, (const double *)bh, (double *)xe, tol, max_iter,
                       fixed_iters, relres_out);
    /* reconstruct odd sites */
    orc_dhop(L, tbc, U, (const double *)xe, (double *)w1);
    for (long q = 0; q < V; q++)
        for (int k = 0; k < 12; k++) SP(w2, q)[k] = SP(eta, q)[k] + kappa * SP(w1, q)[k];
    apply_diag(L, 1.0 / den, -_Complex_I * a / den, w2, w1, 1);
    for (long q = 0; q < V; q++) {
        int ev = parity_of(L, q) == 0;
        for (int k = 0; k < 12; k++) SP(s, q)[k] = ev ? SP(xe, q)[k] : SP(w1, q)[k];
    }
    if (true_rel_out) {
        orc_apply_M(L, tbc, U, kappa, a, 0, (const double *)s, (double *)w2);
        double num = 0, nrm = 0;
        for (long k = 0; k < n; k++) {
            cplx d = eta[k] - w2[k];
            num += creal(d * conj(d));
            nrm += creal(eta[k] * conj(eta[k]));
        }
        *true_rel_out = sqrt(num / nrm);
    }
    free(w1); free(w2); free(bh); free(xe);
    return it;
}

/* ------------------------------------------------------------------ */
/* Z4 noise (Sec. 2, Eq. 1-2; Z4 sources) from Philox4x64-10            */
/* (Salmon, Moraes, Dror, Shaw, SC'11), written from its definition:    */
/* ten rounds of two 64x64->128 multiplies with the output halves       */
/* crossed and xored with the key, key bumped by the Weyl constants.    */
/* ------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* eta(x)_{3*spin+colour}: word 0 of Philox(counter = (lex, src, 0, 0),
 * key = (seed, 0)); component k uses bits 2k (real sign) and 2k+1
 * (imaginary sign): ((-1)^b0 + i (-1)^b1) / sqrt(2). */
void orc_z4_source(const int *L, uint64_t seed, uint64_t src, double *outd)
{
    const long V = volume(L);
    cplx *out = (cplx *)outd;
    const double h = 0.70710678118654752440;
    for (long s = 0; s < V; s++) {
        uint64_t ctr[4] = {(uint64_t)s, src, 0, 0}, key[2] = {seed, 0}, w[4];
        orc_philox4x64_10(ctr, key, w);
        for (int k = 0; k < 12; k++) {
            int b0 = (int)((w[0] >> (2 * k)) & 1), b1 = (int)((w[0] >> (2 * k + 1)) & 1);
            out[12 * s + k] = (b0 ? -h : h) + _Complex_I * (b1 ? -h : h);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Loop contractions at every timeslice (Sec. 2.2: full-volume sources   */
/* give the loop at all insertion times).  Output [9][Lt][4][4] complex: */
/*   kind 0     P_ab(t)   = sum_{x in t} sum_c eta*_{ac}(x) s_{bc}(x)     */
/*   kind 1+nu  F^nu_ab(t) = sum eta*_{ac}(x) [U_nu(x) s(x+nu)]_{bc}      */
/*   kind 5+nu  B^nu_ab(t) = sum [U_nu(x) eta(x+nu)]*_{ac} s_{bc}(x)      */
/* with the time-boundary factor on hops that wrap.                      */
/* ------------------------------------------------------------------ */
void orc_contract(const int *L, int tbc, const double *Ud, const double *etad,
                  const double *sd, double *outd)
{
    const cplx *U = (const cplx *)Ud, *eta = (const cplx *)etad, *s = (const cplx *)sd;
    cplx *out = (cplx *)outd;
    const int T = L[3];
    const long V3 = (long)L[0] * L[1] * L[2];
    memset(out, 0, sizeof(cplx) * 9 * T * 16);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < T; t++) {
        for (long q = 0; q < V3; q++) {
            long x = q + V3 * t;
            const cplx *e = SP(eta, x), *sx = SP(s, x);
            cplx *P = out + 16 * (0 * T + t);
            for (int al = 0; al < 4; al++)
                for (int be = 0; be < 4; be++) {
                    cplx acc = 0;
                    for (int c = 0; c < 3; c++) acc += conj(e[3 * al + c]) * sx[3 * be + c];
                    P[4 * al + be] += acc;
                }
            for (int nu = 0; nu < 4; nu++) {
                double sg;
                long xf = hop(L, x, nu, +1, tbc, &sg);
                const cplx *u = LK(U, x, nu), *sf = SP(s, xf), *ef = SP(eta, xf);
                cplx us[4][3], ue[4][3];
                for (int sp = 0; sp < 4; sp++)
                    for (int a = 0; a < 3; a++) {
                        cplx t1 = 0, t2 = 0;
                        for (int b = 0; b < 3; b++) {
                            t1 += u[3 * a + b] * sf[3 * sp + b];
                            t2 += u[3 * a + b] * ef[3 * sp + b];
                        }
                        us[sp][a] = sg * t1;
                        ue[sp][a] = sg * t2;
                    }
                cplx *F = out + 16 * ((1 + nu) * T + t);
                cplx *B = out + 16 * ((5 + nu) * T + t);
                for (int al = 0; al < 4; al++)
                    for (int be = 0; be < 4; be++) {
                        cplx f = 0, b = 0;
                        for (int c = 0; c < 3; c++) {
                            f += conj(e[3 * al + c]) * us[be][c];
                            b += conj(ue[al][c]) * sx[3 * be + c];
                        }
                        F[4 * al + be] += f;
                        B[4 * al + be] += b;
                    }
            }
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
