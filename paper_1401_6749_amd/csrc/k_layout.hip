// Layout conversion: canonical lexicographic FP64 arrays <-> the even-odd
// site-major structure-of-arrays layouts of every storage precision.
#include "tm_dev.h"
#include "tm_launch.h"

namespace tmk {

// canonical gauge [V][4][3][3][2] (device, FP64) -> [par][mu][group][Vh]
template <int P>
__global__ __launch_bounds__(BLOCK) void k_gauge_pack(Geom g, const double *canon, void *out)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    const int par = blockIdx.y;
    if (cb >= g.vh) return;
    const Site s = site_of(g, cb, par);
    const size_t lex = (size_t)lex_of(g, s);
    for (int mu = 0; mu < 4; mu++) {
        const double2 *u = (const double2 *)canon + (lex * 4 + mu) * 9;  // rows 0,1 = entries 0..5
        const size_t base = (size_t)(par * 4 + mu);
        if constexpr (P == P64) {
            double2 *o = (double2 *)out + base * 6 * g.vh;
            for (int k = 0; k < 6; k++) o[(size_t)k * g.vh + cb] = u[k];
        } else if constexpr (P == P32) {
            float4 *o = (float4 *)out + base * 3 * g.vh;
            for (int q = 0; q < 3; q++)
                o[(size_t)q * g.vh + cb] = make_float4((float)u[2 * q].x, (float)u[2 * q].y, (float)u[2 * q + 1].x,
                                                       (float)u[2 * q + 1].y);
        } else {
            // packed complex halves in the layout LinkHalfIO reads (nine
            // entries, or the first two rows with TM_HALF_LINK12)
            char *o = (char *)out + base * HALF_LINK_BYTES * g.vh;
            uint32_t w[9];
            for (int k = 0; k < 9; k++) {
                const uint32_t lo = HalfCodec<P>::enc((float)u[k].x), hi = HalfCodec<P>::enc((float)u[k].y);
                w[k] = lo | (hi << 16);
            }
            ((uint4 *)o)[cb] = make_uint4(w[0], w[1], w[2], w[3]);
            if constexpr (TM_HALF_LINK12 != 0) {
                ((uint2 *)(o + (size_t)16 * g.vh))[cb] = make_uint2(w[4], w[5]);
            } else {
                ((uint4 *)o)[(size_t)g.vh + cb] = make_uint4(w[4], w[5], w[6], w[7]);
                ((uint32_t *)(o + (size_t)32 * g.vh))[cb] = w[8];
            }
        }
    }
}

void launch_gauge_pack(int p, const Geom &g, const double *canon, void *out, hipStream_t s)
{
    dim3 grid(nblk_of(g), 2);
    switch (p) {
    case P64: hipLaunchKernelGGL((k_gauge_pack<P64>), grid, dim3(BLOCK), 0, s, g, canon, out); break;
    case P32: hipLaunchKernelGGL((k_gauge_pack<P32>), grid, dim3(BLOCK), 0, s, g, canon, out); break;
    case P16: hipLaunchKernelGGL((k_gauge_pack<P16>), grid, dim3(BLOCK), 0, s, g, canon, out); break;
    case PBF: hipLaunchKernelGGL((k_gauge_pack<PBF>), grid, dim3(BLOCK), 0, s, g, canon, out); break;
    }
}

// canonical spinor [V][4][3][2] <-> layout; full field = even half, odd half
template <int P, bool IMPORT>
__global__ __launch_bounds__(BLOCK) void k_field_conv(Geom g, const double *canon_in, double *canon_out,
                                                      const char *fin, char *fout, size_t fbytes)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    const int par = blockIdx.y & 1, rhs = blockIdx.y >> 1;
    if (cb >= g.vh) return;
    const Site s = site_of(g, cb, par);
    const size_t lex = (size_t)lex_of(g, s);
    const size_t V = (size_t)2 * g.vh;
    const size_t hb = half_bytes(P, g);
    if (IMPORT) {
        const double2 *c = (const double2 *)canon_in + ((size_t)rhs * V + lex) * 12;
        cpx<double> v[12];
        for (int k = 0; k < 12; k++) v[k] = cpx<double>{c[k].x, c[k].y};
        SpinorIO<P>::store(fout + (size_t)rhs * fbytes + par * hb, g.vh, cb, v);
    } else {
        cpx<double> v[12];
        SpinorIO<P>::load(fin + (size_t)rhs * fbytes + par * hb, g.vh, cb, v);
        double2 *c = (double2 *)canon_out + ((size_t)rhs * V + lex) * 12;
        for (int k = 0; k < 12; k++) c[k] = make_double2(v[k].re, v[k].im);
    }
}

template <bool IMPORT>
static void field_conv(int p, const Geom &g, int nrhs, const double *ci, double *co, const char *fi, char *fo,
                       hipStream_t s)
{
    dim3 grid(nblk_of(g), 2 * nrhs);
    const size_t fb = 2 * half_bytes(p, g);
    switch (p) {
    case P64: hipLaunchKernelGGL((k_field_conv<P64, IMPORT>), grid, dim3(BLOCK), 0, s, g, ci, co, fi, fo, fb); break;
    case P32: hipLaunchKernelGGL((k_field_conv<P32, IMPORT>), grid, dim3(BLOCK), 0, s, g, ci, co, fi, fo, fb); break;
    case P16: hipLaunchKernelGGL((k_field_conv<P16, IMPORT>), grid, dim3(BLOCK), 0, s, g, ci, co, fi, fo, fb); break;
    case PBF: hipLaunchKernelGGL((k_field_conv<PBF, IMPORT>), grid, dim3(BLOCK), 0, s, g, ci, co, fi, fo, fb); break;
    }
}

void launch_field_import(int p, const Geom &g, int nrhs, const double *canon, char *field, hipStream_t s)
{
    field_conv<true>(p, g, nrhs, canon, nullptr, nullptr, field, s);
}
void launch_field_export(int p, const Geom &g, int nrhs, const char *field, double *canon, hipStream_t s)
{
    field_conv<false>(p, g, nrhs, nullptr, canon, field, nullptr, s);
}

}  // namespace tmk
