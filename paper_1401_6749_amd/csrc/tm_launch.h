// Host-side launchers of the libtm kernels (all asynchronous on a stream).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tm_types.h"

namespace tmk {

// Dslash with epilogue; sp = storage precision of in/in2/out/p and of x, r
// in the CG update (links of the same precision).  Returns -1 on an
// unsupported combination.
int launch_dslash(int sp, bool dag, int epi, bool in2, const DslashArgs &A, hipStream_t s);
// the last preparation Dslash of a noise run with EPI_START: v = Mhat^dag bhat
// (A.in = A^-dag D'_oe bhat, A.in2 = bhat, both in precision sp: P32, or the
// half precision po itself) written as r (A.r), p (A.out) and x = 0 (A.x) in
// half precision po (P16 or PBF), with |v|^2 partials; -1 when no
// timeslice-walk chunk fits the lattice or the pair is not built (nothing
// launched)
int launch_dslash_start(int sp, int po, const DslashArgs &A, hipStream_t s);
// plain-epilogue Dslash with Z4-code inputs, uniform (kappa, a):
//   src 3: hop input A^-1 eta (parity 1 - out_par) and site input eta (prep:
//          bhat = eta + k D A^-1 eta); output in any storage precision
//   src 2: hop input a field, site input eta (reconstruction: A^-1 (eta + k D s)); P64 or P32
int launch_dslash_codes(int sp, int src, const DslashArgs &A, hipStream_t s);

// ---- CG scalars (one block per slot, fixed summation order) ----
void launch_cg_alpha(SlotState *st, const double *partial, int nslot, int nblk, hipStream_t s);
void launch_cg_beta(SlotState *st, const double *partial, int nslot, int nblk, hipStream_t s);
// end of a CG iteration: x += alpha p for slots whose iteration took a step
// (skipped when x is null: after reliable updates), then p = r + beta p for
// running slots (sp = p precision, xr = x and r precision)
void launch_p_update(int sp, int xr, const Geom &g, char *p, size_t p_slot, const char *r, size_t r_slot, char *x,
                     size_t x_slot, SlotState *st, int nslot, int swz, hipStream_t s);
// the same update with per-slot coefficients given by value (every slot
// steps x if x is not null and updates p); fields of one precision sp,
// slot i at base + i * slot_bytes
struct UpdateCoefs {
    double alpha[MAX_SLOTS], beta[MAX_SLOTS];
};
void launch_p_update_coefs(int sp, const Geom &g, char *p, const char *r, char *x, size_t slot_bytes,
                           const UpdateCoefs &c, int nslot, int swz, hipStream_t s);
// start n consecutive slots: rr0 = sum of the slot's nblk partials, status
// RUNNING (or CONVERGED if rr0 == 0); parameters per slot
struct SlotStartParams {
    double kappa[MAX_SLOTS], a[MAX_SLOTS], tol2[MAX_SLOTS], delta2[MAX_SLOTS];
    int max_iter[MAX_SLOTS];
    int mixed;
};
void launch_slot_start(SlotState *st, const double *partial, int nblk, const SlotStartParams &P, int n,
                       hipStream_t s);
void launch_slot_start(SlotState *st, const double *partial, int nblk, double kappa, double a, double tol2,
                       int max_iter, double delta2, int mixed, hipStream_t s);
// after FP64 reliable updates of n consecutive slots: rr_true = sum(partial);
// decide convergence, set beta
void launch_reliable_finish(SlotState *st, const double *partial, int nblk, int n, hipStream_t s);
// out[k] = sum(partial[k*nblk .. (k+1)*nblk)) for k < n (fixed order)
void launch_reduce(const double *partial, int nblk, int n, double *out, hipStream_t s);

// ---- site-local vector kernels on nslot consecutive half fields ----
void launch_convert(int pin, int pout, const Geom &g, const char *in, size_t in_slot, char *out, size_t out_slot,
                    int nslot, hipStream_t s);
void launch_zero(int p, const Geom &g, char *f, size_t slot, int nslot, hipStream_t s);
// r = p = in (rounded to pout), x = 0 for nslot slots; r, p and x share the pitch out_slot; pin P32 or P64
void launch_cg_start(int pin, int pout, const Geom &g, const char *in, size_t in_slot, char *r, char *p, char *x,
                     size_t out_slot, int nslot, hipStream_t s);
// x64 += x32; x32 = 0 (if x32_zero), n consecutive slots with strides s64, s32
void launch_accum_x(const Geom &g, char *x64, size_t s64, const char *x32_in, char *x32_zero, size_t s32, int n,
                    hipStream_t s);
// per-tile (64 sites) |f|^2 partials of one FP64 half field
void launch_norm_partial(const Geom &g, const char *f, double *partial, hipStream_t s);
// out = c * in with c per chirality: A^-1 (mode 1) or identity (mode 0), FP64
void launch_site_diag(const Geom &g, int mode, double a, const char *in, char *out, hipStream_t s);

// ---- noise ----
// Z4 codes of both parities: codes[par*vh + cb]
void launch_z4_codes(const Geom &g, uint64_t seed, uint64_t src, uint32_t *codes, hipStream_t s);
// the same for n sources (n <= MAX_SLOTS) into codes + i * 2 * vh; source i
// is zero outside the timeslices t = tph[i] mod tmod[i] when tmod[i] > 0
struct Z4Sources {
    uint64_t seed[MAX_SLOTS], src[MAX_SLOTS];
    int tmod[MAX_SLOTS], tph[MAX_SLOTS];
};
void launch_z4_codes(const Geom &g, const Z4Sources &Z, int n, uint32_t *codes, hipStream_t s);
// eta of one parity as an FP64 half field (times A^-1 when ainv != 0)
void launch_z4_field(const Geom &g, const uint32_t *codes_par, int ainv, double a, char *out, hipStream_t s);
// canonical FP64 layout [V][4][3][2]
void launch_z4_canonical(const Geom &g, uint64_t seed, uint64_t src, double *out, hipStream_t s);

// ---- contractions ----
int contract_nchunk(const Geom &g);
// spin matrices of one source into raw_out [9][T][16][2]: s and links in FP64
// or FP32 (sps; gauge must be that precision's link array), accumulation FP64
void launch_contract(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                     const uint32_t *codes, double *cpart, double *raw_out, hipStream_t s);
// n sources at once (n <= MAX_SLOTS): source i has s_even + i * s_stride,
// s_odd + i * s_stride, codes + i * 2 * vh, partials cpart + i * contract_part_doubles
// and output raw_out[i]
struct RawOuts {
    double *p[MAX_SLOTS];
};
size_t contract_part_doubles(const Geom &g);
void launch_contract(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                     size_t s_stride, const uint32_t *codes, double *cpart, const RawOuts &raw, int n, hipStream_t s);
// the same with a field as the left vector (the one-end trick): left fields
// l_even/l_odd + i * l_stride, right fields s_even/s_odd + i * s_stride, all
// in precision sps; raw = (sr + i si) * the spin-matrix sums
void launch_contract_lr(int sps, const Geom &g, const void *gauge, const char *s_even, const char *s_odd,
                        size_t s_stride, const char *l_even, const char *l_odd, size_t l_stride, double *cpart,
                        const RawOuts &raw, int n, double sr, double si, hipStream_t s, bool local_only = false);
// local spin matrices only (kind 0 of raw[i]; other kinds untouched) of n
// sources with Z4-code left vectors, as launch_contract
void launch_contract_local(int sps, const Geom &g, const char *s_even, const char *s_odd, size_t s_stride,
                           const uint32_t *codes, double *cpart, const RawOuts &raw, int n, hipStream_t s);
// exact part of the hopping parameter expansion as local spin matrices
// raw[0][T][16][2] (kinds 1..8 untouched); even extents >= 4
void launch_hpe_exact(const Geom &g, double kappa, double a, double *raw, hipStream_t s);
// raw [n][9][T][16][2] -> ops [n][90][T][2]; gtab: [16][4] (col | phase << 2)
void launch_project(int n, int lt, const double *raw, double *ops, const int *gtab_host, hipStream_t s);
// TSM combination over per-source ops; est += ops_add when given; entries
// (op, t) with valid[op * T + t] == 0 are NaN (estimate and variances)
void launch_tsm_combine(int n_hp, int n_lp, int lt, const double *ops_hp, const double *ops_lp_corr,
                        const double *ops_lp_bulk, double *est, double *var_re, double *var_im, hipStream_t s,
                        const double *ops_add = nullptr, const unsigned char *valid = nullptr);
// out[i] = sum_k in[i * nph + k] in order k = 0..nph-1, i < n, per doubles each
void launch_sum_phases(const double *in, double *out, int n, int nph, size_t per, hipStream_t s);

// ---- layout ----
// canonical FP64 gauge (device) -> per-precision link arrays
void launch_gauge_pack(int p, const Geom &g, const double *canon, void *out, hipStream_t s);
// canonical full-lattice spinors <-> layout (full field = even half, then odd half)
void launch_field_import(int p, const Geom &g, int nrhs, const double *canon, char *field, hipStream_t s);
void launch_field_export(int p, const Geom &g, int nrhs, const char *field, double *canon, hipStream_t s);

// streaming copy probe
void launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// gamma table for the projection: [16][4] entries (column | phase << 2),
// phase 0..3 = 1, i, -1, -i; built from the four basis matrices.
const int *gamma_table();

__host__ __device__ inline size_t half_bytes(int p, const Geom &g)
{
    return (size_t)g.vh * (p == P64 ? 192 : p == P32 ? 96 : 52);
}
inline size_t link_array_bytes(int p, const Geom &g)
{
    return (size_t)2 * 4 * g.vh * (p == P64 ? 96 : p == P32 ? 48 : HALF_LINK_BYTES);
}
__host__ __device__ inline int nblk_of(const Geom &g) { return (g.vh + BLOCK - 1) / BLOCK; }
// per-slot partial sums: one per 64-site tile
__host__ __device__ inline int ntile_of(const Geom &g) { return (g.vh + TILE - 1) / TILE; }

}  // namespace tmk
