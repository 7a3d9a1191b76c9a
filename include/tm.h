/*
 * tm.h - C ABI of the MI355X twisted-mass disconnected-loop library (libtm).
 *
 * The library computes stochastic estimates of quark loops with the
 * truncated solver method of Alexandrou, Drach, Jansen, Koutsou, Vaquero,
 * "Computation of disconnected contributions to nucleon observables"
 * (LATTICE 2013):
 *   - Z4 noise sources eta_j                         (Sec. 2, Eq. 1-2; Z4 noise)
 *   - solves M s_j = eta_j, M_E^-1 = (1/N) sum s eta^dag  (Sec. 2, Eq. estiM)
 *   - CG inversions, truncated for low precision     (Sec. 2.1, LP residual ~1e-2)
 *   - the TSM estimator                              (Sec. 2.1, Eq. estiTSM)
 *   - loops at every insertion time                  (Sec. 2.2, last paragraph)
 * for the twisted-mass Wilson operator
 *   M = 1 - kappa*D_hop + i*a*gamma5,   a = 2*kappa*mu,
 * i.e. M = B^-1 + H with B = (1 + i a gamma5)^-1 and H = -kappa*D_hop, the
 * split used in the hopping-parameter expansion (Sec. 2.4, Eq. HPE), with
 *   D_hop psi(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                       + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu).
 *
 * Conventions (the paper fixes none of them):
 *   lattice dims  {Lx, Ly, Lz, Lt}, every extent even and >= 2
 *   site index    lex = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2
 *   time BC       hops across t = Lt-1 <-> 0 carry t_bc (-1 antiperiodic)
 *   gammas        chiral Euclidean basis, gamma5 = diag(1, 1, -1, -1)
 *   canonical spinor  double[V][4 spin][3 colour][2 re,im]
 *   canonical gauge   double[V][4 mu][3 row][3 col][2 re,im]
 *
 * Errors: every call returns a tm_status; no exception crosses the ABI.
 * tm_last_error() gives the message of the last failing call on a context.
 * Device pointers are HIP device addresses on the context's device; host
 * pointers are ordinary host memory.  The caller owns every buffer it
 * passes; the library owns contexts, gauge handles and serving engines
 * until the matching destroy/free call.
 * Threads: calls on one context must not overlap in time from several host
 * threads, except tm_serve_submit, tm_serve_poll, tm_serve_status_get,
 * tm_serve_clock, tm_serve_drain, tm_serve_footprint, tm_last_error and
 * tm_memory_usage, which may run while a serving engine's worker thread
 * uses the context.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tm_context tm_context;
typedef struct tm_gauge tm_gauge;
typedef struct tm_server tm_server;

typedef enum tm_status {
    TM_OK = 0,
    TM_ERR_ARG = -1,     /* invalid argument (shape, null pointer, alias, unloaded precision) */
    TM_ERR_NOMEM = -2,   /* device allocation failed or exceeds the context's HBM budget */
    TM_ERR_HIP = -3,     /* a HIP runtime call failed */
    TM_ERR_NOCONV = -4,  /* a solve hit max_iter before its tolerance (outputs still written) */
    TM_ERR_NUMERIC = -5, /* NaN/Inf or a non-positive <p, A p> met in a solve */
    TM_ERR_STATE = -6    /* call not valid in the object's current state */
} tm_status;

/* Storage precisions.  Spinors and links in F16/BF16 are used by the
 * low-precision solver only; their arithmetic is FP32. */
typedef enum tm_prec {
    TM_PREC_F64 = 1,
    TM_PREC_F32 = 2,
    TM_PREC_F16 = 4,
    TM_PREC_BF16 = 8
} tm_prec;

/* Operators for tm_dslash.  HOP, M, MDAG act on full-lattice fields; the
 * MHAT family acts on the even half (the even-odd Schur complement
 *   Mhat = A - kappa^2 D_eo A^-1 D_oe,  A = 1 + i a gamma5,
 * with D_eo the hop from odd to even sites). */
typedef enum tm_op {
    TM_OP_HOP = 0,          /* out = D_hop in */
    TM_OP_M = 1,            /* out = M in */
    TM_OP_MDAG = 2,         /* out = M^dagger in = gamma5 M(-mu) gamma5 in */
    TM_OP_MHAT = 3,         /* out_e = Mhat in_e */
    TM_OP_MHAT_DAG = 4,     /* out_e = Mhat^dagger in_e */
    TM_OP_MHAT_DAG_MHAT = 5, /* out_e = Mhat^dagger Mhat in_e */
    TM_OP_BH = 6             /* out = B H in, full lattice: M = B^-1 + H with
                                B = (1 + i a gamma5)^-1 and H = -kappa D_hop, the
                                factor of the hopping parameter expansion (Sec. 2.4,
                                Eq. HPE) */
} tm_op;

/* Solver modes (Sec. 2.1: low- and high-precision inversions by CG). */
typedef enum tm_solve_mode {
    TM_SOLVE_F64 = 0,   /* plain FP64 CG throughout */
    TM_SOLVE_MIXED = 1, /* FP32 CG with FP64 reliable updates of x and the true residual */
    TM_SOLVE_LP = 2     /* every CG vector (p, the Dslash intermediates, x and r) stored in F16 or
                           BF16 with an FP32 per-site scale; FP32 arithmetic, FP64 global sums */
} tm_solve_mode;

/* Device allocator used for every library allocation.  NULL means hipMalloc
 * and hipFree.  The Python binding passes torch's caching allocator. */
typedef void *(*tm_alloc_fn)(size_t bytes, int device, void *user);
typedef void (*tm_free_fn)(void *ptr, int device, void *user);

/* ------------------------------------------------------------------ */
/* Context                                                             */
/* ------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hbm_budget (bytes) bounds the
 * device memory the context may hold at once (0 = no bound).  Ownership of
 * *out passes to the caller until tm_destroy.  Errors: TM_ERR_ARG (null
 * out, bad device), TM_ERR_HIP. */
int tm_create(int device, size_t hbm_budget, tm_alloc_fn alloc, tm_free_fn free_fn, void *user,
              tm_context **out);

/* Release every gauge field and workspace of the context, then the context. */
int tm_destroy(tm_context *ctx);

/* Message of the last failing call on ctx ("" if none), copied for the calling
 * thread: valid until that thread's next tm_last_error call. */
const char *tm_last_error(const tm_context *ctx);

/* Bytes currently held on the device by ctx, and the peak since creation. */
int tm_memory_usage(const tm_context *ctx, size_t *in_use, size_t *peak);

/* ------------------------------------------------------------------ */
/* Gauge field (the configuration the loops are measured on, Sec. 3)   */
/* ------------------------------------------------------------------ */

/* Upload a gauge field and build the device layouts for each precision in
 * prec_mask (bitwise OR of tm_prec; F64 is always built: it serves the
 * reconstruction, the true residual and the contractions).
 *   dims        {Lx, Ly, Lz, Lt}, each even and >= 2
 *   links_host  host, canonical gauge layout, V*4*9 complex doubles
 *   t_bc        -1 antiperiodic or +1 periodic in time
 * Every link is checked for unitarity and det = 1 (|U^dag U - 1| and
 * |det U - 1| below 1e-10).  The kernels address a link array through
 * 32-bit buffer offsets, so the FP64 copy (384 bytes per site) must stay
 * below 4 GiB: at most 11184810 sites (48^3 x 96 fits, 64^4 does not).
 * The caller keeps links_host; the library owns the device copies until
 * tm_free_gauge.  Synchronous.  Errors: TM_ERR_ARG (dims, too many sites,
 * t_bc, non-SU(3) link, NaN), TM_ERR_NOMEM, TM_ERR_HIP. */
int tm_load_gauge(tm_context *ctx, const int dims[4], const double *links_host, int t_bc,
                  unsigned prec_mask, tm_gauge **out);

int tm_free_gauge(tm_context *ctx, tm_gauge *gauge);

/* Bytes of one field in the library's device layout for precision prec:
 * subset 0 = one parity (V/2 sites), 1 = full lattice.  0 on bad input.
 * Layout (site-major structure of arrays over the V/2 sites of a parity,
 * site cb = lex/2 within its parity, full field = even half then odd half):
 *   F64   12 complex components k = 3*spin+colour, component k at [k][V/2] (16 B each)
 *   F32   6 float4 groups (components 2g, 2g+1) at [g][V/2]
 *   F16/BF16  3 groups of 8 halves (components 4g..4g+3) at [g][V/2], then a
 *         float per-site scale [V/2]; value = half * scale. */
size_t tm_field_bytes(const tm_gauge *gauge, tm_prec prec, int subset);

/* Convert nrhs full-lattice fields between the canonical spinor layout
 * (device, FP64) and the device layout of prec.  Asynchronous on
 * hip_stream (a hipStream_t, NULL = default stream).  Errors: TM_ERR_ARG. */
int tm_field_import(tm_context *ctx, const tm_gauge *gauge, tm_prec prec, int nrhs,
                    const double *canonical_dev, void *field_dev, void *hip_stream);
int tm_field_export(tm_context *ctx, const tm_gauge *gauge, tm_prec prec, int nrhs,
                    const void *field_dev, double *canonical_dev, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Dirac operator (Sec. 2.2 twisted-mass operator; Sec. 2.4 H)          */
/* ------------------------------------------------------------------ */

/* Apply op to nrhs fields in the device layout of prec (full-lattice
 * fields for HOP/M/MDAG, even-half fields for the MHAT family), fields
 * contiguous one after another.  kappa and two_kappa_mu = a as in M above.
 * in and out must not overlap.  Asynchronous on hip_stream; no host sync,
 * except that the MHAT family takes its temporaries (one even-odd half
 * field per rhs, two for MHAT_DAG_MHAT) from the context, grown on demand
 * with a device synchronisation; MHAT-family calls on one context that
 * overlap on different streams race on them.
 * Errors: TM_ERR_ARG (nrhs < 1 or > 16, aliasing, prec not loaded). */
int tm_dslash(tm_context *ctx, const tm_gauge *gauge, tm_op op, double kappa, double two_kappa_mu,
              tm_prec prec, int nrhs, const void *in, void *out, void *hip_stream);

/* As tm_dslash with explicit byte strides between consecutive fields of in
 * and of out (multiples of 16, at least one field); same semantics and
 * errors otherwise.  Lets callers lay batches out with padding. */
int tm_dslash_ex(tm_context *ctx, const tm_gauge *gauge, tm_op op, double kappa, double two_kappa_mu,
                 tm_prec prec, int nrhs, const void *in, size_t in_stride, void *out, size_t out_stride,
                 void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operators, arguments, layouts and results as tm_dslash_ex (bit for bit),
 * without any device allocation.  The temporaries of the MHAT family (one
 * even-odd half field per right-hand side, two for MHAT_DAG_MHAT; none for
 * HOP, M, MDAG and BH) come from a fixed array of TM_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on until the process ends.
 * All calls on one device share that array: calls that overlap in time on
 * one device (other streams, other host threads) race and must be ordered by
 * the caller.  Asynchronous on hip_stream.  Errors: as tm_dslash_ex, and
 * TM_ERR_ARG when the temporaries exceed the array (MHAT, MHAT_DAG: nrhs
 * half fields of prec; MHAT_DAG_MHAT: twice that). */
#define TM_NOALLOC_SCRATCH_BYTES (64u << 20)
int tm_dslash_noalloc(tm_context *ctx, const tm_gauge *gauge, tm_op op, double kappa, double two_kappa_mu,
                      tm_prec prec, int nrhs, const void *in, size_t in_stride, void *out, size_t out_stride,
                      void *hip_stream);

/* ------------------------------------------------------------------ */
/* Solver (Sec. 2.1: "the inverter, a CG solver")                       */
/* ------------------------------------------------------------------ */

typedef struct tm_solver_params {
    int mode;              /* tm_solve_mode */
    int half_prec;         /* TM_PREC_F16 or TM_PREC_BF16 for TM_SOLVE_LP */
    double tol;            /* stop at |r_k| <= tol*|r_0| on Mhat^dag Mhat x = Mhat^dag bhat */
    int max_iter;          /* iteration cap (TM_ERR_NOCONV when reached) */
    int fixed_iters;       /* > 0: run exactly this many iterations, ignore tol */
    double delta;          /* MIXED: reliable update when |r| < delta*|r at last update| (0 -> 0.001); convergence is always confirmed on the FP64 true residual */
    int chunk;             /* iterations per device launch chunk between host checks (0 -> auto) */
} tm_solver_params;

typedef struct tm_solve_stats {
    int iters;             /* CG iterations */
    int reliable_updates;  /* MIXED: number of FP64 reliable updates */
    double cg_rel_resid;   /* |r_k| / |r_0| of the iterated residual at exit */
    double true_rel_resid; /* |eta - M s| / |eta| recomputed in FP64 at exit */
    double seconds;        /* wall time of the whole call */
} tm_solve_stats;

/* Solve M x_i = b_i for nrhs full-lattice right-hand sides through
 * even-odd CG on Mhat^dag Mhat with zero initial guess:
 *   bhat_e = b_e + kappa D_eo A^-1 b_o,  CG for x_e,
 *   x_o = A^-1 (b_o + kappa D_oe x_e).
 * b, x: device, canonical spinor layout, nrhs fields each.  stats: host
 * array [nrhs] or NULL.  Runs on hip_stream and synchronises at exit.
 * Errors: TM_ERR_ARG, TM_ERR_NOMEM, TM_ERR_NOCONV (x and stats still
 * written), TM_ERR_NUMERIC. */
int tm_cg_solve(tm_context *ctx, const tm_gauge *gauge, double kappa, double two_kappa_mu,
                const tm_solver_params *params, int nrhs, const double *b, double *x,
                tm_solve_stats *stats, void *hip_stream);

/* The direction update that ends every CG iteration (Sec. 2.1, the CG
 * solver), as tm_cg_solve and tm_loops_tsm apply it, on nrhs caller fields:
 *   x_i += alpha_i p_i   (skipped when x is NULL), then
 *   p_i  = r_i + beta_i p_i,
 * both from the old p_i, with the solver's kernel: arithmetic in FP64 for
 * TM_PREC_F64, in FP32 for the other precisions, each result rounded to
 * the storage format of prec.
 *   p, r, x      device, nrhs even-half fields in the layout of prec
 *                (tm_field_bytes(gauge, prec, 1) bytes each), field i at
 *                base + i * stride; 16-byte aligned; p overlaps neither
 *                r nor x, r and x do not overlap
 *   stride       bytes between consecutive fields: a multiple of 16, at
 *                least one field
 *   alpha, beta  host, nrhs finite doubles each (copied at the call)
 *   nrhs         1..16
 * The gauge field only fixes the lattice; its links are not read.
 * Asynchronous on hip_stream; allocates nothing.  Errors: TM_ERR_ARG,
 * TM_ERR_HIP. */
int tm_cg_update(tm_context *ctx, const tm_gauge *gauge, tm_prec prec, int nrhs, void *p, const void *r, void *x,
                 size_t stride, const double *alpha, const double *beta, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Noise (Sec. 2: Z_N noise with Eq. 1-2; Z4 here)                      */
/* ------------------------------------------------------------------ */

/* Write the Z4 source eta(seed, src_id) in the canonical spinor layout to
 * the device buffer out: eta(x)_{3*spin+colour} = ((-1)^b0 + i (-1)^b1)/sqrt(2)
 * with b0, b1 bits 2k, 2k+1 of word 0 of Philox4x64-10(counter = (lex,
 * src_id, 0, 0), key = (seed, 0)).  Asynchronous on hip_stream. */
int tm_z4_source(tm_context *ctx, const int dims[4], uint64_t seed, uint64_t src_id, double *out,
                 void *hip_stream);

/* ------------------------------------------------------------------ */
/* Loops with the truncated solver method (Sec. 2.1 Eq. estiTSM, 2.2)   */
/* ------------------------------------------------------------------ */

#define TM_N_LOCAL 16 /* 1, g1..g4, g5, g1g5..g4g5, s12, s13, s14, s23, s24, s34 */
#define TM_N_DERIV 64 /* L^D_{G,nu}: index 16 + 4*G + nu, nu = x, y, z, t */
#define TM_N_SYM 10   /* (L^D_{g_m,n} + L^D_{g_n,m})/2, m <= n: index 80.. */
#define TM_N_OPS 90

typedef struct tm_tsm_params {
    double kappa;
    double two_kappa_mu;
    uint64_t noise_seed;
    int n_hp;                  /* correction set: source ids 0..n_hp-1, HP and LP solves */
    int n_lp;                  /* bulk set: ids n_hp..n_hp+n_lp-1, LP solves only */
    tm_solver_params hp;       /* high-precision solver (usually MIXED or F64 to 1e-10) */
    tm_solver_params lp;       /* low-precision solver (usually LP truncated at 1e-2) */
    int batch;                 /* right-hand sides per multi-RHS launch (1..16, 0 -> 12) */
    int want_true_resid;       /* 1: compute |eta - M s|/|eta| for every solve */
    int ops;                   /* 0: local and one-derivative loops; 1: the 16 local loops only
                                  (ops 16..89 NaN, raw kinds 1..8 zero; one contraction pass).
                                  Serving requests take 0 only. */
} tm_tsm_params;

typedef struct tm_tsm_stats {
    int hp_solves, lp_solves;
    long long hp_iters, lp_iters;        /* summed over solves */
    int hp_max_iters, lp_max_iters;
    int reliable_updates;
    double max_hp_true_resid;            /* over HP solves, if want_true_resid */
    double max_lp_true_resid;
    double seconds, hp_seconds, lp_seconds;
} tm_tsm_stats;

/* The whole path for one gauge field: Z4 sources, HP and LP solves,
 * contractions at all timeslices, projection onto the 90 operators and the
 * TSM combination
 *   est = (1/N_HP) sum_{j<N_HP} (L_j^HP - L_j^LP) + (1/N_LP) sum_{j>=N_HP} L_j^LP
 *   var = s^2(L^HP - L^LP)/N_HP + s^2(L^LP)/N_LP   (re and im separately, n-1),
 * a set with no members contributing 0 and a set with one member making
 * var NaN.  n_hp = 0 gives the plain estimator (Sec. 2, Eq. estiM).
 * Loops are the raw traces eta^dag G s (local) and the symmetric covariant
 * derivative L^D_{G,nu}(t) = 1/4 [F(t) + F(t - d) - B(t) - B(t - d)],
 *   F(t) = sum_{x in t} eta(x)^dag G U_nu(x) s(x+nu),
 *   B(t) = sum_{x in t} eta(x+nu)^dag G U_nu(x)^dagger s(x),
 * d = 1 for nu = t else 0; no factor 2 kappa, i or fermion-loop sign.
 * Outputs (host): est [TM_N_OPS][Lt][2], var_re and var_im [TM_N_OPS][Lt];
 * raw (optional, NULL to skip) [n_hp + (n_hp + n_lp)][9][Lt][4][4][2]: HP
 * spin matrices of ids 0..n_hp-1, then LP ones of ids 0..n_hp+n_lp-1, kinds
 * 0 local, 1..4 F^nu, 5..8 B^nu, entry [a][b] = sum eta*_a (...) s_b.
 * Synchronous.  Errors: TM_ERR_ARG, TM_ERR_NOMEM, TM_ERR_NOCONV (outputs
 * still written), TM_ERR_NUMERIC. */
int tm_loops_tsm(tm_context *ctx, const tm_gauge *gauge, const tm_tsm_params *params, double *est,
                 double *var_re, double *var_im, double *raw, tm_tsm_stats *stats);

/* The same sources, solves and TSM combination with the one-end trick
 * estimators of the twisted-mass formulation (Sec. 2.2, Eq. loopVv and
 * Eq. loopStD), for the same 90 operators X.  With s = M_u^-1 eta
 * (M_u = D_W + i a g5 the operator of this library, M_d the same with -a,
 * D_W = M at a = 0):
 *   flavour 0 (isovector)  -2 i a s^dag g5 X s       -> Tr(M_u^-1 X) - Tr(M_d^-1 X)
 *   flavour 1 (isoscalar)   2 s^dag g5 X g5 D_W s    -> Tr(M_u^-1 X) + Tr(M_d^-1 X)
 * (the isovector sign follows from M_u^-1 - M_d^-1 = -2ia M_u^-1 g5 M_d^-1
 * in this normalisation).  Outputs as tm_loops_tsm with a leading flavour
 * index: est [2][TM_N_OPS][Lt][2], var_re/var_im [2][TM_N_OPS][Lt], raw
 * (optional) [2][n_hp + n_hp + n_lp][9][Lt][4][4][2] holding the spin
 * matrices with the factor (-2ia or 2) applied, to be projected with the
 * insertions g5 G (flavour 0) and g5 G g5 (flavour 1).  Each source costs
 * one more Dslash application (D_W s) and one more contraction than
 * tm_loops_tsm.  Errors as tm_loops_tsm. */
int tm_loops_oet(tm_context *ctx, const tm_gauge *gauge, const tm_tsm_params *params, double *est,
                 double *var_re, double *var_im, double *raw, tm_tsm_stats *stats);

/* The same sources, solves and TSM combination with the hopping parameter
 * expansion (Sec. 2.4, Eq. HPE and Eq. loopHPE1) of the 16 local loops.
 * With M = B^-1 + H, B = (1 + i a g5)^-1 and H = -kappa D_hop,
 *   M^-1 = B - BHB + (BH)^2 B - (BH)^3 B + (BH)^4 M^-1;
 * the first four terms are traced exactly (for local G their site-diagonal
 * blocks do not depend on the links: 3 V3 diag_b(B_b + 16 kappa^2 b5 e_b
 * B_b^2), b5 = -i a/(1 + a^2), e_b = g5's eigenvalue on spin b) and the last
 * stochastically as eta^dag G (BH)^4 s with s = M^-1 eta.
 *   flavour 0: the standard estimator, identical to tm_loops_tsm;
 *   flavour 1: the expansion: ops 0..15 = exact part + TSM combination of
 *              eta^dag G (BH)^4 s, variances those of the stochastic term;
 *              ops 16..89 (operators with a link, whose exact part depends
 *              on the links) are NaN.
 * Outputs as tm_loops_oet: est [2][TM_N_OPS][Lt][2], var_re/var_im
 * [2][TM_N_OPS][Lt], raw (optional) [2][n_hp + n_hp + n_lp][9][Lt][4][4][2]
 * where flavour 1 holds eta^dag (BH)^4 s in kind 0 and zeros in kinds 1..8.
 * Each source costs four more full-lattice B H applications and one local
 * contraction.  Every extent must be >= 4 (TM_ERR_ARG otherwise: smaller
 * tori close two- and three-hop paths through the links).  Errors as
 * tm_loops_tsm. */
int tm_loops_hpe(tm_context *ctx, const tm_gauge *gauge, const tm_tsm_params *params, double *est,
                 double *var_re, double *var_im, double *raw, tm_tsm_stats *stats);

/* Time dilution and coherent sources (Sec. 2.3), optionally with the
 * hopping parameter expansion.  Noise vector r (ids and TSM sets as in
 * tm_loops_tsm) is split into one source per phase p: eta_r on the
 * timeslices t with t mod spacing == p (spacing = Lt: full time dilution;
 * smaller spacing: coherent sources with Lt/spacing timeslices, spacing
 * apart).  Every such source is solved (HP and LP in the correction set, LP
 * in the bulk), contracted, and the spin matrices of noise vector r are the
 * sums over its phases in phase order; the TSM combination then runs over
 * noise vectors.
 *   spacing:  divides Lt;
 *   phases:   n_phases distinct values in [0, spacing) (host), or NULL for
 *             all spacing phases; the cost is n_phases solves per noise
 *             vector and solver;
 *   hpe:      0: one estimator (flavour 0, as tm_loops_tsm); 1: also the
 *             expansion (flavour 1, as tm_loops_hpe, every extent >= 4).
 * Covered entries: a loop at t needs the noise on t (local and
 * spatial-derivative operators) or on t - 1, t and t + 1 (the time
 * derivative and the symmetrised operators containing it); est and the
 * variances are NaN elsewhere, and for ops 16..89 of flavour 1.
 * Outputs: est [1 + hpe][TM_N_OPS][Lt][2], var_re/var_im [1 + hpe][TM_N_OPS][Lt],
 * raw (optional) [1 + hpe][n_hp + n_hp + n_lp][9][Lt][4][4][2] per noise
 * vector (summed over its phases).  Device memory grows with
 * n_phases x (2 n_hp + n_lp) spin-matrix sets of 9 Lt 32 doubles each.
 * Errors: TM_ERR_ARG (spacing, phases, extents), then as tm_loops_tsm. */
int tm_loops_tdil(tm_context *ctx, const tm_gauge *gauge, const tm_tsm_params *params, int spacing,
                  const int *phases, int n_phases, int hpe, double *est, double *var_re, double *var_im, double *raw,
                  tm_tsm_stats *stats);

/* The contraction step of tm_loops_tsm alone, for given solutions: loops
 * at every insertion time (Sec. 2.2, last paragraph) of the local and
 * one-derivative operators (abstract) as spin matrices
 *   raw[i][9][Lt][4][4][2], kinds 0 local, 1..4 F^nu, 5..8 B^nu as in
 *   tm_loops_tsm, of eta_i = eta(noise_seed, src_ids[i]) (as tm_z4_source)
 *   and the solution s_i (any field; normally s_i = M^-1 eta_i).
 *   prec     TM_PREC_F64 or TM_PREC_F32: s and the links in that precision;
 *            FP32 products are summed in FP64
 *   s        device, n full-lattice fields in the layout of prec (see
 *            tm_field_bytes), field i at s + i * s_stride; s_stride a
 *            multiple of 256 and at least one field
 *   src_ids  host, n source ids;  raw  device, n * 9 * Lt * 32 doubles
 *   n        1..16
 * Asynchronous on hip_stream.  Its scratch (Z4 codes, partial sums) is the
 * context's, grown on demand (with a device synchronisation): calls on one
 * context that overlap on different streams race on it.  Errors:
 * TM_ERR_ARG, TM_ERR_NOMEM, TM_ERR_HIP. */
int tm_contract(tm_context *ctx, const tm_gauge *gauge, tm_prec prec, int n, const void *s, size_t s_stride,
                uint64_t noise_seed, const uint64_t *src_ids, double *raw, void *hip_stream);

/* Project spin matrices [n][9][Lt][4][4][2] (host) onto the 90 operator
 * loops [n][TM_N_OPS][Lt][2] (host), as in tm_loops_tsm. */
int tm_project_loops(int n, int lt, const double *raw, double *ops);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of loop requests                        */
/* ------------------------------------------------------------------ */

typedef struct tm_request {
    const tm_gauge *gauge;     /* resident gauge field (any loaded lattice) */
    tm_tsm_params params;      /* kappa, mu, seeds, N_HP, N_LP, solvers */
    uint64_t tag;              /* caller's identifier, returned with the result */
} tm_request;

typedef struct tm_result {
    uint64_t tag;
    int status;                /* tm_status of the request */
    int lt;
    double *est;               /* [TM_N_OPS][lt][2], owned by the server until tm_result_free */
    double *var_re, *var_im;   /* [TM_N_OPS][lt] */
    tm_tsm_stats stats;
    double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
} tm_result;

/* Start a serving engine on ctx.  slots = right-hand sides per multi-RHS
 * batch (1..16); workspace_budget = device bytes the engine may hold for
 * solver workspaces (requests wait until their footprint fits).  A worker
 * thread runs the loop: admission by footprint, packing of sources that
 * share a gauge field and precision into batches, refill of finished slots
 * between chunks, contraction and TSM combination per request. */
int tm_serve_create(tm_context *ctx, int slots, size_t workspace_budget, tm_server **out);
/* Queue a request (copied).  Errors: TM_ERR_ARG, TM_ERR_NOMEM (the
 * request's footprint can never fit the workspace budget). */
int tm_serve_submit(tm_server *srv, const tm_request *req);
/* Workspace bytes *bytes that req needs from the budget when none of its
 * batches is resident yet (its output buffers plus fresh batches for its
 * HP and LP precisions).  Capacity planning only; queues nothing.
 * Errors: TM_ERR_ARG. */
int tm_serve_footprint(const tm_server *srv, const tm_request *req, size_t *bytes);
/* Pop up to max finished results into out[] (returns the count, or < 0). */
int tm_serve_poll(tm_server *srv, tm_result *out, int max);
/* Block until every submitted request is finished. */
int tm_serve_drain(tm_server *srv);
void tm_result_free(tm_result *res);
/* Seconds on the server clock (same clock as tm_result times). */
double tm_serve_clock(tm_server *srv);

/* Snapshot of the serving loop, published by the worker once per pass. */
typedef struct tm_serve_status {
    int queued;               /* submitted, not admitted */
    int active;               /* admitted, not finished */
    int finished;             /* finished, not yet polled */
    int batches;              /* resident multi-RHS batches */
    int in_flight;            /* batches with a chunk on the GPU */
    int pending_jobs;         /* solves waiting for a slot */
    int running_slots;        /* occupied slots over all batches */
    int worker_error;         /* first error met by the worker (TM_OK if none) */
    size_t arena_used, arena_size, arena_largest_free;
    double t_snapshot;        /* server clock of the snapshot */
    double stall_s;           /* seconds since the worker last changed a request or batch
                                 while work was outstanding (0 when idle) */
    double busy_s;            /* server seconds so far with at least one chunk on the GPU */
    double slot_s;            /* slot-seconds so far: occupied slots integrated over time */
} tm_serve_status;
/* Copy the latest snapshot into *out.  Errors: TM_ERR_ARG. */
int tm_serve_status_get(tm_server *srv, tm_serve_status *out);
int tm_serve_destroy(tm_server *srv);

/* ------------------------------------------------------------------ */
/* Measurement helpers                                                 */
/* ------------------------------------------------------------------ */

/* Copy `bytes` from src to dst (device) with the library's streaming copy
 * kernel, the measured HBM ceiling for the roofline.  Asynchronous. */
int tm_stream_copy(tm_context *ctx, const void *src, void *dst, size_t bytes, void *hip_stream);

/* Host-side self checks of the library's index arithmetic (no GPU needed):
 * returns 0 when they pass. */
int tm_selftest(void);

#ifdef __cplusplus
}
#endif
#endif /* TM_H */
