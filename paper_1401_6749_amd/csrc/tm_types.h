// Types shared by the host driver code and the kernels of libtm.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace tmk {

// Half-precision links: all nine entries (36 B: [uint4 entries 0..3][uint4
// entries 4..7][uint entry 8], each [Vh]) or, with TM_HALF_LINK12, the first
// two rows (24 B: [uint4 entries 0..3][uint2 entries 4..5]) with the third
// rebuilt in FP32 at every load.
#ifndef TM_HALF_LINK12
#define TM_HALF_LINK12 0
#endif
constexpr int HALF_LINK_BYTES = TM_HALF_LINK12 ? 24 : 36;

// storage precision index (kernel templates); tm_prec bit = 1 << index
enum : int { P64 = 0, P32 = 1, P16 = 2, PBF = 3 };

// q = floor(n / d) for 32-bit n as (umulhi(n, m) + n) >> l with
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1
// (Granlund & Montgomery, "Division by invariant integers using multiplication").
struct FastDiv {
    uint32_t m;
    uint32_t l;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) l++;
    uint64_t m = ((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d) + 1;
    return FastDiv{(uint32_t)m, l};
}

inline uint32_t fastdiv_host(uint32_t n, FastDiv d)
{
    uint32_t hi = (uint32_t)(((uint64_t)n * d.m) >> 32);
    return (uint32_t)(((uint64_t)hi + n) >> d.l);
}

// Geometry of the even-odd site-major layout.
struct Geom {
    int L[4];    // Lx, Ly, Lz, Lt
    int lxh;     // Lx / 2
    int vh;      // V / 2 sites per parity
    int v3h;     // Lx*Ly*Lz / 2 sites per parity and timeslice
    int sy, sz, st;  // cb strides of a step in y, z, t
    int tbc;     // +1 periodic, -1 antiperiodic time boundary
    FastDiv div_xh, div_y, div_z;
};

inline Geom make_geom(const int dims[4], int tbc)
{
    Geom g;
    for (int i = 0; i < 4; i++) g.L[i] = dims[i];
    g.lxh = dims[0] / 2;
    g.vh = g.lxh * dims[1] * dims[2] * dims[3];
    g.v3h = g.lxh * dims[1] * dims[2];
    g.sy = g.lxh;
    g.sz = g.lxh * dims[1];
    g.st = g.lxh * dims[1] * dims[2];
    g.tbc = tbc;
    g.div_xh = make_fastdiv((uint32_t)g.lxh);
    g.div_y = make_fastdiv((uint32_t)dims[1]);
    g.div_z = make_fastdiv((uint32_t)dims[2]);
    return g;
}

// Per right-hand-side ("slot") solver state, resident on the device.
enum : int {
    ST_EMPTY = 0,
    ST_RUNNING = 1,
    ST_CONVERGED = 2,
    ST_MAXITER = 3,
    ST_NEED_UPDATE = 4,  // mixed precision: waiting for an FP64 reliable update
    ST_NUMERIC = 5
};

struct alignas(128) SlotState {
    int status;
    int iter;
    int max_iter;
    int mixed;        // 1: reliable-update criterion active
    double kappa;
    double a;         // 2 kappa mu
    double rr;        // |r|^2 of the current iterate
    double rr0;       // |r_0|^2 = |Mhat^dag bhat|^2
    double tol2;      // tol^2 (0 with fixed iterations)
    double delta2;    // reliable-update threshold squared
    double rr_ref;    // |r|^2 at the last reliable update
    double alpha, beta, pap;
    double rr_new;    // last |r|^2 (sloppy) computed by the beta kernel
    int xpend;        // 1: this iteration's x += alpha p is owed (set by the alpha kernel,
                      // applied by the direction update at the end of the iteration)
};

// Site-local coefficient sets of the Dslash epilogue out = P*in2 + Q*hop(in),
// per chirality (spins 0,1 and spins 2,3), built from (kappa, a).
enum : int {
    CM_HOP = 0,       // P = 0, Q = 1
    CM_AINV = 1,      // P = 0, Q = A^-1        (A = 1 + i a g5)
    CM_AINV_DAG = 2,  // P = 0, Q = A^-dagger
    CM_MHAT = 3,      // P = A, Q = -kappa^2
    CM_MHAT_DAG = 4,  // P = A^dagger, Q = -kappa^2
    CM_PREP = 5,      // P = 1, Q = kappa
    CM_RECON = 6,     // P = A^-1, Q = kappa A^-1
    CM_M = 7,         // P = A, Q = -kappa
    CM_MDAG = 8,      // P = A^dagger, Q = -kappa
    CM_BH = 9         // P = 0, Q = -kappa A^-1   (B H of the hopping parameter expansion)
};

// Epilogues of the Dslash kernel
enum : int {
    EPI_PLAIN = 0,  // out = P in2 + Q hop
    EPI_NORM = 1,   // as PLAIN, plus per-block |out|^2
    EPI_CGUPD = 2,  // Ap = P in2 + Q hop; r -= alpha Ap; per-block |r|^2 (x += alpha p in the direction update)
    EPI_RESID = 3,  // out = b - (P in2 + Q hop); per-block |out|^2
    EPI_START = 4   // v = P in2 + Q hop; r = out = v and x = 0 in the CG storage precision; per-block |v|^2
};

constexpr int MAX_SLOTS = 16;
constexpr int BLOCK = 256;  // threads per block of the site kernels
constexpr int TILE = 64;    // sites per reduction tile (partials are per slot and tile)

struct DslashArgs {
    Geom g;
    const void *gauge;  // link array of the storage precision
    const char *in;     // hop input (parity 1 - out_par), slot 0
    const char *in2;    // site-local input (parity out_par), slot 0
    char *out;
    size_t in_slot, in2_slot, out_slot;  // bytes between consecutive slots
    int out_par;
    int coef;
    double kappa_u, a_u;  // used when st == nullptr
    SlotState *st;
    int nslot, nblk_site, swz;  // nblk_site: blocks over the sites (set by the launcher)
    int ntile;                  // 64-site reduction tiles per slot
    uint32_t in_span, gauge_span;  // bytes reachable through the buffer resources (set by the launcher)
    int twalk;                     // timeslices walked per block (set by the launcher)
    int gouter;                    // slot groups slowest in the block order (set by the launcher)
    int wcy, wcz;                  // timeslice-walk chunk: y rows x z planes of full x rows (set by the launcher)
    double *partial;            // [nslot][ntile]
    // EPI_CGUPD (r), EPI_START (x, r)
    char *x, *r;
    const char *p;
    size_t xr_slot, p_slot;
    // EPI_RESID
    const char *b;
    size_t b_slot;
    // Z4-code inputs: codes[par * V/2 + cb] per slot, slot stride in bytes
    const uint32_t *codes;
    size_t codes_slot;
};

}  // namespace tmk
