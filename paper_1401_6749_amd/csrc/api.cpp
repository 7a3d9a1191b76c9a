// C ABI of libtm: contexts, gauge fields, the Dirac operator, the solver,
// noise and the truncated-solver loop estimator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "tm_arena.h"
#include "tm_internal.h"

using namespace tmk;

namespace tmi {

int set_err(tm_context *c, int code, const char *fmt, ...)
{
    if (!c) return code;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(c->mu);
    c->err = buf;
    return code;
}

void *dalloc(tm_context *c, size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->budget && c->in_use + bytes > c->budget) return nullptr;
    }
    void *p = nullptr;
    if (c->alloc) {
        p = c->alloc(bytes, c->device, c->user);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (!p) return nullptr;
    std::lock_guard<std::mutex> lk(c->mu);
    c->allocs[p] = bytes;
    c->in_use += bytes;
    c->peak = std::max(c->peak, c->in_use);
    return p;
}

void dfree(tm_context *c, void *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->allocs.find(p);
        if (it == c->allocs.end()) return;
        c->in_use -= it->second;
        c->allocs.erase(it);
    }
    if (c->free_fn)
        c->free_fn(p, c->device, c->user);
    else
        (void)hipFree(p);
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace tmi

using namespace tmi;

// ---------------------------------------------------------------------------
// Fixed device scratch of tm_dslash_noalloc: one array per device, allocated
// with the library's code object when it is loaded on that device and held
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it only stands in for the symbol): tm_create looks up
// its device address once per device, with that device current, and the
// entry point uses that address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[TM_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex scratch_mu;
std::unordered_map<int, void *> scratch_addr;  // device -> address of its scratch

// address of the device's scratch, looked up on first use (device current)
int scratch_setup(int device, void **out)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    auto it = scratch_addr.find(device);
    if (it != scratch_addr.end()) {
        *out = it->second;
        return TM_OK;
    }
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TM_ERR_HIP;
    scratch_addr[device] = p;
    *out = p;
    return TM_OK;
}

void *scratch_of(int device)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    auto it = scratch_addr.find(device);
    return it == scratch_addr.end() ? nullptr : it->second;
}
}  // namespace

// ---------------------------------------------------------------------------
// gamma table for the projection (chiral basis; each of the 16 insertions has
// exactly one non-zero entry per row, valued 1, i, -1 or -i)
// ---------------------------------------------------------------------------
namespace tmk {
namespace {
typedef std::complex<double> C;
struct M4 {
    C m[4][4];
};
M4 mmul(const M4 &a, const M4 &b)
{
    M4 r{};
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            C s = 0;
            for (int k = 0; k < 4; k++) s += a.m[i][k] * b.m[k][j];
            r.m[i][j] = s;
        }
    return r;
}
M4 basis(int mu)
{
    const C I(0, 1);
    M4 g{};
    switch (mu) {
    case 0: g.m[0][3] = -I; g.m[1][2] = -I; g.m[2][1] = I; g.m[3][0] = I; break;
    case 1: g.m[0][3] = -1.0; g.m[1][2] = 1.0; g.m[2][1] = 1.0; g.m[3][0] = -1.0; break;
    case 2: g.m[0][2] = -I; g.m[1][3] = I; g.m[2][0] = I; g.m[3][1] = -I; break;
    default: g.m[0][2] = 1.0; g.m[1][3] = 1.0; g.m[2][0] = 1.0; g.m[3][1] = 1.0; break;
    }
    return g;
}
struct Tab {
    int e[64];
    bool ok;
    Tab()
    {
        ok = true;
        M4 one{};
        for (int i = 0; i < 4; i++) one.m[i][i] = 1.0;
        M4 g[4] = {basis(0), basis(1), basis(2), basis(3)};
        M4 g5 = mmul(mmul(g[0], g[1]), mmul(g[2], g[3]));
        std::vector<M4> G;
        G.push_back(one);
        for (int m = 0; m < 4; m++) G.push_back(g[m]);
        G.push_back(g5);
        for (int m = 0; m < 4; m++) G.push_back(mmul(g[m], g5));
        for (int m = 0; m < 4; m++)
            for (int n = m + 1; n < 4; n++) {
                M4 a = mmul(g[m], g[n]), b = mmul(g[n], g[m]), s{};
                for (int i = 0; i < 4; i++)
                    for (int j = 0; j < 4; j++) s.m[i][j] = C(0, 0.5) * (a.m[i][j] - b.m[i][j]);
                G.push_back(s);
            }
        for (int gi = 0; gi < 16; gi++)
            for (int a = 0; a < 4; a++) {
                int col = -1, ph = 0, nnz = 0;
                for (int b = 0; b < 4; b++) {
                    C v = G[gi].m[a][b];
                    if (std::abs(v) < 1e-12) continue;
                    nnz++;
                    col = b;
                    if (std::abs(v - C(1, 0)) < 1e-12) ph = 0;
                    else if (std::abs(v - C(0, 1)) < 1e-12) ph = 1;
                    else if (std::abs(v - C(-1, 0)) < 1e-12) ph = 2;
                    else if (std::abs(v - C(0, -1)) < 1e-12) ph = 3;
                    else ok = false;
                }
                if (nnz != 1) ok = false;
                e[4 * gi + a] = (col & 3) | (ph << 2);
            }
    }
};
const Tab &tab()
{
    static Tab t;
    return t;
}
}  // namespace
const int *gamma_table() { return tab().e; }
}  // namespace tmk

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int tm_create(int device, size_t hbm_budget, tm_alloc_fn alloc, tm_free_fn free_fn, void *user,
                         tm_context **out)
{
    if (!out) return TM_ERR_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TM_ERR_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr)) return TM_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return TM_ERR_HIP;
    void *scr = nullptr;
    if (scratch_setup(device, &scr) != TM_OK) return TM_ERR_HIP;
    tm_context *c = new tm_context();
    c->device = device;
    c->budget = hbm_budget;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    if (const char *e = getenv("TM_XCD_SWIZZLE")) c->swz = atoi(e);
    if (const char *e = getenv("TM_GRAPHS")) c->use_graphs = atoi(e);
    *out = c;
    return TM_OK;
}

extern "C" int tm_destroy(tm_context *ctx)
{
    if (!ctx) return TM_ERR_ARG;
    (void)hipDeviceSynchronize();
    std::vector<void *> ps;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : ctx->allocs) ps.push_back(kv.first);
    }
    for (void *p : ps) dfree(ctx, p);
    delete ctx;
    return TM_OK;
}

// The message is copied under the context lock into a per-thread buffer: a
// serving worker may set a new message on the context at any time.
extern "C" const char *tm_last_error(const tm_context *ctx)
{
    if (!ctx) return "null context";
    thread_local std::string copy;
    std::lock_guard<std::mutex> lk(ctx->mu);
    copy = ctx->err;
    return copy.c_str();
}

extern "C" int tm_memory_usage(const tm_context *ctx, size_t *in_use, size_t *peak)
{
    if (!ctx) return TM_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (in_use) *in_use = ctx->in_use;
    if (peak) *peak = ctx->peak;
    return TM_OK;
}

// ---------------------------------------------------------------------------
// gauge
// ---------------------------------------------------------------------------
static bool dims_ok(const int *d)
{
    if (!d) return false;
    long long v = 1;
    for (int i = 0; i < 4; i++) {
        if (d[i] < 2 || d[i] % 2) return false;
        v *= d[i];
    }
    return v <= (1ll << 30);
}

// The kernels reach a link array and a spinor field through buffer resources
// with 32-bit byte offsets.  The largest array is the FP64 link copy, 2
// parities x 4 directions x 96 bytes per even-odd site = 384 bytes per site,
// so a lattice fits when 384 V stays below 4 GiB (every spinor field, at most
// 192 bytes per site of a parity, then fits too).
static bool lattice_fits(const int *d)
{
    const unsigned long long v = (unsigned long long)d[0] * d[1] * d[2] * d[3];
    return v * 384ull <= 0xFFFFFFFFull;
}

// max over links of |U^dag U - 1| and |det U - 1|; NaN-aware
static double su3_violation(const double *links, size_t nlinks)
{
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<double> worst(nt, 0.0);
    std::vector<std::thread> th;
    for (unsigned k = 0; k < nt; k++)
        th.emplace_back([&, k] {
            double w = 0;
            for (size_t l = k; l < nlinks; l += nt) {
                const std::complex<double> *u = (const std::complex<double> *)(links + 18 * l);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        std::complex<double> s = 0;
                        for (int r = 0; r < 3; r++) s += std::conj(u[3 * r + i]) * u[3 * r + j];
                        double d = std::abs(s - (i == j ? 1.0 : 0.0));
                        if (!(d <= w)) w = std::isnan(d) ? INFINITY : std::max(w, d);
                    }
                std::complex<double> det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                                           u[2] * (u[3] * u[7] - u[4] * u[6]);
                double d = std::abs(det - 1.0);
                if (!(d <= w)) w = std::isnan(d) ? INFINITY : std::max(w, d);
            }
            worst[k] = w;
        });
    for (auto &t : th) t.join();
    double w = 0;
    for (double x : worst) w = std::max(w, x);
    return w;
}

extern "C" int tm_load_gauge(tm_context *ctx, const int dims[4], const double *links_host, int t_bc,
                             unsigned prec_mask, tm_gauge **out)
{
    if (!ctx) return TM_ERR_ARG;
    if (!out || !links_host) return set_err(ctx, TM_ERR_ARG, "null argument");
    *out = nullptr;
    if (!dims_ok(dims)) return set_err(ctx, TM_ERR_ARG, "lattice extents must be even and >= 2");
    if (!lattice_fits(dims))
        return set_err(ctx, TM_ERR_ARG,
                       "lattice too large: its FP64 link array would exceed the 4 GiB that 32-bit buffer offsets "
                       "address (at most %llu sites)", 0xFFFFFFFFull / 384ull);
    if (t_bc != 1 && t_bc != -1) return set_err(ctx, TM_ERR_ARG, "t_bc must be +1 or -1");
    if (prec_mask & ~15u) return set_err(ctx, TM_ERR_ARG, "unknown precision bits 0x%x", prec_mask);
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    const double viol = su3_violation(links_host, 4 * V);
    if (!(viol < 1e-10)) return set_err(ctx, TM_ERR_ARG, "gauge links are not SU(3) (max violation %.3e)", viol);
    TM_HIP(ctx, hipSetDevice(ctx->device));
    tm_gauge *G = new tm_gauge();
    G->ctx = ctx;
    for (int i = 0; i < 4; i++) G->dims[i] = dims[i];
    G->tbc = t_bc;
    G->g = make_geom(dims, t_bc);
    const size_t canon_bytes = V * 4 * 18 * sizeof(double);
    double *canon = (double *)dalloc(ctx, canon_bytes);
    if (!canon) {
        delete G;
        return set_err(ctx, TM_ERR_NOMEM, "cannot allocate %zu bytes for the gauge upload", canon_bytes);
    }
    unsigned mask = prec_mask | TM_PREC_F64;
    int rc = TM_OK;
    hipError_t e = hipMemcpy(canon, links_host, canon_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = set_err(ctx, TM_ERR_HIP, "gauge upload: %s", hipGetErrorString(e));
    for (int p = 0; p < 4 && rc == TM_OK; p++) {
        if (!(mask & (1u << p))) continue;
        G->links[p] = dalloc(ctx, link_array_bytes(p, G->g));
        if (!G->links[p]) {
            rc = set_err(ctx, TM_ERR_NOMEM, "cannot allocate the gauge copy of precision %d", p);
            break;
        }
        launch_gauge_pack(p, G->g, canon, G->links[p], nullptr);
        G->precs |= 1u << p;
    }
    e = hipDeviceSynchronize();
    if (rc == TM_OK && e != hipSuccess) rc = set_err(ctx, TM_ERR_HIP, "gauge pack: %s", hipGetErrorString(e));
    dfree(ctx, canon);
    if (rc != TM_OK) {
        for (int p = 0; p < 4; p++) dfree(ctx, G->links[p]);
        delete G;
        return rc;
    }
    *out = G;
    return TM_OK;
}

extern "C" int tm_free_gauge(tm_context *ctx, tm_gauge *G)
{
    if (!ctx || !G || G->ctx != ctx) return TM_ERR_ARG;
    (void)hipDeviceSynchronize();
    for (int p = 0; p < 4; p++) dfree(ctx, G->links[p]);
    delete G;
    return TM_OK;
}

static int prec_index(int prec)
{
    switch (prec) {
    case TM_PREC_F64: return P64;
    case TM_PREC_F32: return P32;
    case TM_PREC_F16: return P16;
    case TM_PREC_BF16: return PBF;
    }
    return -1;
}

extern "C" size_t tm_field_bytes(const tm_gauge *G, tm_prec prec, int subset)
{
    const int p = prec_index(prec);
    if (!G || p < 0 || (subset != 0 && subset != 1)) return 0;
    return half_bytes(p, G->g) * (subset ? 2 : 1);
}

extern "C" int tm_field_import(tm_context *ctx, const tm_gauge *G, tm_prec prec, int nrhs,
                               const double *canonical_dev, void *field_dev, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    const int p = prec_index(prec);
    if (!G || p < 0 || nrhs < 1 || nrhs > 32768 || !canonical_dev || !field_dev)
        return set_err(ctx, TM_ERR_ARG, "tm_field_import: bad argument");
    launch_field_import(p, G->g, nrhs, canonical_dev, (char *)field_dev, (hipStream_t)hip_stream);
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

extern "C" int tm_field_export(tm_context *ctx, const tm_gauge *G, tm_prec prec, int nrhs, const void *field_dev,
                               double *canonical_dev, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    const int p = prec_index(prec);
    if (!G || p < 0 || nrhs < 1 || nrhs > 32768 || !canonical_dev || !field_dev)
        return set_err(ctx, TM_ERR_ARG, "tm_field_export: bad argument");
    launch_field_export(p, G->g, nrhs, (const char *)field_dev, canonical_dev, (hipStream_t)hip_stream);
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

// ---------------------------------------------------------------------------
// Dirac operator
// ---------------------------------------------------------------------------
static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

extern "C" int tm_dslash_ex(tm_context *ctx, const tm_gauge *G, tm_op op, double kappa, double a, tm_prec prec,
                            int nrhs, const void *in, size_t in_stride, void *out, size_t out_stride,
                            void *hip_stream);

extern "C" int tm_dslash(tm_context *ctx, const tm_gauge *G, tm_op op, double kappa, double a, tm_prec prec,
                         int nrhs, const void *in, void *out, void *hip_stream)
{
    const int p = prec_index(prec);
    if (!ctx) return TM_ERR_ARG;
    if (!G || p < 0) return set_err(ctx, TM_ERR_ARG, "tm_dslash: bad gauge or precision");
    const bool full = op == TM_OP_HOP || op == TM_OP_M || op == TM_OP_MDAG || op == TM_OP_BH;
    const size_t fb = half_bytes(p, G->g) * (full ? 2 : 1);
    return tm_dslash_ex(ctx, G, op, kappa, a, prec, nrhs, in, fb, out, fb, hip_stream);
}

// Temporaries of the MHAT family: bytes needed (0 for full-lattice operators).
static size_t dslash_tmp_bytes(const tm_gauge *G, int p, tm_op op, int nrhs)
{
    const size_t hb = half_bytes(p, G->g);
    if (op == TM_OP_MHAT || op == TM_OP_MHAT_DAG) return hb * nrhs;
    if (op == TM_OP_MHAT_DAG_MHAT) return 2 * hb * nrhs;
    return 0;
}

// tm_dslash_ex with its temporaries given: tmp (device) of at least
// dslash_tmp_bytes(), or nullptr to take them from the context's scratch,
// grown on demand.
static int dslash_impl(tm_context *ctx, const tm_gauge *G, tm_op op, double kappa, double a, tm_prec prec, int nrhs,
                       const void *in, size_t in_stride, void *out, size_t out_stride, void *hip_stream, char *tmp,
                       size_t tmp_cap);

extern "C" int tm_dslash_ex(tm_context *ctx, const tm_gauge *G, tm_op op, double kappa, double a, tm_prec prec,
                            int nrhs, const void *in, size_t in_stride, void *out, size_t out_stride,
                            void *hip_stream)
{
    return dslash_impl(ctx, G, op, kappa, a, prec, nrhs, in, in_stride, out, out_stride, hip_stream, nullptr, 0);
}

extern "C" int tm_dslash_noalloc(tm_context *ctx, const tm_gauge *G, tm_op op, double kappa, double a,
                                 tm_prec prec, int nrhs, const void *in, size_t in_stride, void *out,
                                 size_t out_stride, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    char *tmp = (char *)scratch_of(ctx->device);
    if (!tmp) return set_err(ctx, TM_ERR_HIP, "tm_dslash_noalloc: no scratch address for device %d", ctx->device);
    return dslash_impl(ctx, G, op, kappa, a, prec, nrhs, in, in_stride, out, out_stride, hip_stream, tmp,
                       TM_NOALLOC_SCRATCH_BYTES);
}

static int dslash_impl(tm_context *ctx, const tm_gauge *G, tm_op op, double kappa, double a, tm_prec prec, int nrhs,
                       const void *in, size_t in_stride, void *out, size_t out_stride, void *hip_stream, char *tmp,
                       size_t tmp_cap)
{
    if (!ctx) return TM_ERR_ARG;
    const int p = prec_index(prec);
    if (!G || p < 0) return set_err(ctx, TM_ERR_ARG, "tm_dslash: bad gauge or precision");
    if (!(G->precs & (1u << p))) return set_err(ctx, TM_ERR_ARG, "tm_dslash: gauge not loaded in this precision");
    if (nrhs < 1 || nrhs > MAX_SLOTS) return set_err(ctx, TM_ERR_ARG, "tm_dslash: nrhs must be 1..%d", MAX_SLOTS);
    if (!in || !out) return set_err(ctx, TM_ERR_ARG, "tm_dslash: null field");
    if (op < TM_OP_HOP || op > TM_OP_BH) return set_err(ctx, TM_ERR_ARG, "tm_dslash: unknown op");
    const Geom &g = G->g;
    const size_t hb = half_bytes(p, g);
    const bool full = op == TM_OP_HOP || op == TM_OP_M || op == TM_OP_MDAG || op == TM_OP_BH;
    const size_t fb = full ? 2 * hb : hb;
    if (in_stride < fb || out_stride < fb || in_stride % 16 || out_stride % 16)
        return set_err(ctx, TM_ERR_ARG, "tm_dslash: strides must be multiples of 16 and at least one field");
    if (overlap(in, in_stride * (nrhs - 1) + fb, out, out_stride * (nrhs - 1) + fb))
        return set_err(ctx, TM_ERR_ARG, "tm_dslash: in and out overlap");
    hipStream_t s = (hipStream_t)hip_stream;
    DslashArgs A;
    std::memset(&A, 0, sizeof(A));
    A.g = g;
    A.gauge = G->links[p];
    A.nslot = nrhs;
    A.swz = ctx->swz;
    A.kappa_u = kappa;
    A.a_u = a;
    A.in_slot = A.in2_slot = in_stride;
    A.out_slot = out_stride;
    const char *ic = (const char *)in;
    char *oc = (char *)out;
    if (full) {
        const int coef = op == TM_OP_HOP ? CM_HOP : op == TM_OP_M ? CM_M : op == TM_OP_BH ? CM_BH : CM_MDAG;
        const bool dag = op == TM_OP_MDAG;
        const bool in2 = op == TM_OP_M || op == TM_OP_MDAG;
        for (int par = 0; par < 2; par++) {
            A.in = ic + (1 - par) * hb;
            A.in2_slot = in_stride;
            A.in2 = in2 ? ic + par * hb : nullptr;
            A.out = oc + par * hb;
            A.out_par = par;
            A.coef = coef;
            launch_dslash(p, dag, EPI_PLAIN, in2, A, s);
        }
    } else {
        // temporaries: odd half per rhs, plus an even half per rhs for MHAT_DAG_MHAT
        const size_t need = dslash_tmp_bytes(G, p, op, nrhs);
        if (tmp) {
            if (need > tmp_cap)
                return set_err(ctx, TM_ERR_ARG,
                               "tm_dslash_noalloc: the operator needs %zu bytes of temporaries, the fixed scratch "
                               "holds %zu", need, tmp_cap);
        } else {
            const size_t grow = 2 * hb * nrhs;
            if (ctx->op_tmp_bytes < grow) {
                (void)hipDeviceSynchronize();
                dfree(ctx, ctx->op_tmp);
                ctx->op_tmp = dalloc(ctx, grow);
                ctx->op_tmp_bytes = ctx->op_tmp ? grow : 0;
                if (!ctx->op_tmp) return set_err(ctx, TM_ERR_NOMEM, "tm_dslash: no memory for temporaries");
            }
            tmp = (char *)ctx->op_tmp;
        }
        char *t = tmp, *u = t + hb * nrhs;
        auto mhat = [&](const char *src, size_t src_stride, char *dst, size_t dst_stride, bool dag) {
            A.in_slot = src_stride;
            A.out_slot = hb;
            A.in = src;
            A.in2 = nullptr;
            A.out = t;
            A.out_par = 1;
            A.coef = dag ? CM_AINV_DAG : CM_AINV;
            launch_dslash(p, dag, EPI_PLAIN, false, A, s);
            A.in_slot = hb;
            A.in2_slot = src_stride;
            A.out_slot = dst_stride;
            A.in = t;
            A.in2 = src;
            A.out = dst;
            A.out_par = 0;
            A.coef = dag ? CM_MHAT_DAG : CM_MHAT;
            launch_dslash(p, dag, EPI_PLAIN, true, A, s);
        };
        if (op == TM_OP_MHAT) mhat(ic, in_stride, oc, out_stride, false);
        else if (op == TM_OP_MHAT_DAG) mhat(ic, in_stride, oc, out_stride, true);
        else {
            mhat(ic, in_stride, u, hb, false);
            mhat(u, hb, oc, out_stride, true);
        }
    }
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
static int check_solver(tm_context *ctx, const tm_gauge *G, const tm_solver_params *p)
{
    if (!p) return set_err(ctx, TM_ERR_ARG, "null solver params");
    if (p->mode < TM_SOLVE_F64 || p->mode > TM_SOLVE_LP) return set_err(ctx, TM_ERR_ARG, "unknown solver mode");
    if (p->mode == TM_SOLVE_LP && p->half_prec != TM_PREC_F16 && p->half_prec != TM_PREC_BF16)
        return set_err(ctx, TM_ERR_ARG, "LP solver needs half_prec F16 or BF16");
    if (p->fixed_iters <= 0 && !(p->tol > 0 && p->tol < 1)) return set_err(ctx, TM_ERR_ARG, "tol must be in (0, 1)");
    if (p->fixed_iters <= 0 && p->max_iter < 1) return set_err(ctx, TM_ERR_ARG, "max_iter must be >= 1");
    const int sp = kind_prec(kind_of(*p));
    if (!(G->precs & (1u << sp))) return set_err(ctx, TM_ERR_ARG, "gauge field not loaded in the solver's precision");
    if (p->mode == TM_SOLVE_LP && !(G->precs & (1u << P32)))
        return set_err(ctx, TM_ERR_ARG, "LP solves also need the FP32 links");
    return TM_OK;
}

static void job_from(Job &j, const tm_solver_params &p, double kappa, double a)
{
    j.kappa = kappa;
    j.a = a;
    j.tol = p.tol;
    j.max_iter = p.max_iter;
    j.fixed = p.fixed_iters;
    j.delta = p.delta > 0 ? p.delta : TM_DEFAULT_DELTA;
}

extern "C" int tm_cg_update(tm_context *ctx, const tm_gauge *G, tm_prec prec, int nrhs, void *p, const void *r,
                            void *x, size_t stride, const double *alpha, const double *beta, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    const int pi = prec_index(prec);
    if (!G || pi < 0) return set_err(ctx, TM_ERR_ARG, "tm_cg_update: bad gauge or precision");
    if (nrhs < 1 || nrhs > MAX_SLOTS) return set_err(ctx, TM_ERR_ARG, "tm_cg_update: nrhs must be 1..%d", MAX_SLOTS);
    if (!p || !r || !alpha || !beta) return set_err(ctx, TM_ERR_ARG, "tm_cg_update: null argument");
    const size_t hb = half_bytes(pi, G->g);
    const bool aligned = (uintptr_t)p % 16 == 0 && (uintptr_t)r % 16 == 0 && (uintptr_t)x % 16 == 0;
    if (stride < hb || stride % 16 || !aligned)
        return set_err(ctx, TM_ERR_ARG, "tm_cg_update: fields must be 16-byte aligned, the stride a multiple of 16 "
                                        "and at least one field");
    const size_t span = stride * (size_t)(nrhs - 1) + hb;
    if (overlap(p, span, r, span) || (x && (overlap(p, span, x, span) || overlap(r, span, x, span))))
        return set_err(ctx, TM_ERR_ARG, "tm_cg_update: p, r and x must not overlap");
    UpdateCoefs c;
    std::memset(&c, 0, sizeof(c));
    for (int i = 0; i < nrhs; i++) {
        if (!std::isfinite(alpha[i]) || !std::isfinite(beta[i]))
            return set_err(ctx, TM_ERR_ARG, "tm_cg_update: alpha and beta must be finite");
        c.alpha[i] = alpha[i];
        c.beta[i] = beta[i];
    }
    launch_p_update_coefs(pi, G->g, (char *)p, (const char *)r, (char *)x, stride, c, nrhs, ctx->swz,
                          (hipStream_t)hip_stream);
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

extern "C" int tm_cg_solve(tm_context *ctx, const tm_gauge *G, double kappa, double a, const tm_solver_params *params,
                           int nrhs, const double *b, double *x, tm_solve_stats *stats, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    if (!G || !b || !x || nrhs < 1) return set_err(ctx, TM_ERR_ARG, "tm_cg_solve: bad argument");
    int rc = check_solver(ctx, G, params);
    if (rc) return rc;
    const double t0 = now_s();
    TM_HIP(ctx, hipSetDevice(ctx->device));
    const size_t V = (size_t)2 * G->g.vh;
    std::vector<Job> jobs(nrhs);
    std::vector<Job *> q;
    for (int i = 0; i < nrhs; i++) {
        Job &j = jobs[i];
        j.noise = false;
        j.b_canon = b + (size_t)i * V * 24;
        j.x_canon = x + (size_t)i * V * 24;
        job_from(j, *params, kappa, a);
        j.want_true = 1;
        q.push_back(&j);
    }
    // own non-blocking stream (capturable), ordered after the caller's stream
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    TM_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    TM_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    TM_HIP(ctx, hipEventRecord(ev, (hipStream_t)hip_stream));
    TM_HIP(ctx, hipStreamWaitEvent(st, ev, 0));
    Batch *B = nullptr;
    const Kind k = kind_of(*params);
    rc = batch_create(ctx, G, k, std::min(nrhs, MAX_SLOTS), params->chunk, st, &B);
    if (!rc) {
        std::vector<Batch *> bs{B};
        std::vector<std::vector<Job *>> qs{q};
        rc = run_jobs(bs, qs);
        batch_destroy(B);
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    (void)hipEventDestroy(ev);
    if (rc) return rc;
    const double t1 = now_s();
    int worst = TM_OK;
    for (int i = 0; i < nrhs; i++) {
        if (stats) {
            stats[i].iters = jobs[i].iters;
            stats[i].reliable_updates = jobs[i].updates;
            stats[i].cg_rel_resid = jobs[i].cg_rel;
            stats[i].true_rel_resid = jobs[i].true_rel;
            stats[i].seconds = t1 - t0;
        }
        if (jobs[i].status == TM_ERR_NUMERIC) worst = TM_ERR_NUMERIC;
        else if (jobs[i].status == TM_ERR_NOCONV && worst == TM_OK) worst = TM_ERR_NOCONV;
    }
    if (rc) return rc;
    if (worst == TM_ERR_NUMERIC) return set_err(ctx, worst, "tm_cg_solve: non-finite or non-positive curvature");
    if (worst == TM_ERR_NOCONV) return set_err(ctx, worst, "tm_cg_solve: max_iter reached before tol");
    return TM_OK;
}

// ---------------------------------------------------------------------------
// noise
// ---------------------------------------------------------------------------
extern "C" int tm_z4_source(tm_context *ctx, const int dims[4], uint64_t seed, uint64_t src, double *out,
                            void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    if (!dims_ok(dims) || !out) return set_err(ctx, TM_ERR_ARG, "tm_z4_source: bad argument");
    Geom g = make_geom(dims, -1);
    launch_z4_canonical(g, seed, src, out, (hipStream_t)hip_stream);
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

// ---------------------------------------------------------------------------
// contractions of given solutions with their Z4 sources
// ---------------------------------------------------------------------------
extern "C" int tm_contract(tm_context *ctx, const tm_gauge *G, tm_prec prec, int n, const void *s, size_t s_stride,
                           uint64_t noise_seed, const uint64_t *src_ids, double *raw, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    const int p = prec_index(prec);
    if (!G || (p != P64 && p != P32)) return set_err(ctx, TM_ERR_ARG, "tm_contract: gauge, or precision not F64/F32");
    if (!(G->precs & (1u << p))) return set_err(ctx, TM_ERR_ARG, "tm_contract: gauge not loaded in this precision");
    if (n < 1 || n > MAX_SLOTS || !s || !src_ids || !raw)
        return set_err(ctx, TM_ERR_ARG, "tm_contract: n must be 1..%d and every pointer set", MAX_SLOTS);
    const Geom &g = G->g;
    const size_t hb = half_bytes(p, g);
    if (s_stride < 2 * hb || s_stride % 256)
        return set_err(ctx, TM_ERR_ARG, "tm_contract: s_stride must be a multiple of 256 and at least one field");
    const size_t codes_b = ((size_t)n * 2 * g.vh * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t need = codes_b + (size_t)n * contract_part_doubles(g) * sizeof(double);
    if (ctx->ct_tmp_bytes < need) {
        (void)hipDeviceSynchronize();
        dfree(ctx, ctx->ct_tmp);
        ctx->ct_tmp = dalloc(ctx, need);
        ctx->ct_tmp_bytes = ctx->ct_tmp ? need : 0;
        if (!ctx->ct_tmp) return set_err(ctx, TM_ERR_NOMEM, "tm_contract: no memory for its scratch");
    }
    uint32_t *codes = (uint32_t *)ctx->ct_tmp;
    double *cpart = (double *)((char *)ctx->ct_tmp + codes_b);
    hipStream_t st = (hipStream_t)hip_stream;
    Z4Sources Z{};
    RawOuts R{};
    const size_t per = (size_t)9 * g.L[3] * 32;
    for (int i = 0; i < n; i++) {
        Z.seed[i] = noise_seed;
        Z.src[i] = src_ids[i];
        R.p[i] = raw + i * per;
    }
    launch_z4_codes(g, Z, n, codes, st);
    const char *se = (const char *)s;
    launch_contract(p, g, G->links[p], se, se + hb, s_stride, codes, cpart, R, n, st);
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

// ---------------------------------------------------------------------------
// projection on the host (utility for raw spin matrices)
// ---------------------------------------------------------------------------
extern "C" int tm_project_loops(int n, int lt, const double *raw, double *ops)
{
    if (n < 0 || lt < 2 || !raw || !ops) return TM_ERR_ARG;
    const int *tb = gamma_table();
    typedef std::complex<double> Cd;
    auto gp = [&](int gi, const double *m) {
        Cd s = 0;
        for (int a = 0; a < 4; a++) {
            int col = tb[4 * gi + a] & 3, ph = tb[4 * gi + a] >> 2;
            Cd v(m[2 * (4 * a + col)], m[2 * (4 * a + col) + 1]);
            static const Cd P[4] = {Cd(1, 0), Cd(0, 1), Cd(-1, 0), Cd(0, -1)};
            s += P[ph] * v;
        }
        return s;
    };
    auto der = [&](const double *r, int gi, int nu, int t) {
        const double *F = r + (size_t)(1 + nu) * lt * 32, *B = r + (size_t)(5 + nu) * lt * 32;
        int tm = nu == 3 ? (t + lt - 1) % lt : t;
        return 0.25 * (gp(gi, F + t * 32) + gp(gi, F + tm * 32) - gp(gi, B + t * 32) - gp(gi, B + tm * 32));
    };
    for (int j = 0; j < n; j++) {
        const double *r = raw + (size_t)j * 9 * lt * 32;
        double *o = ops + (size_t)j * TM_N_OPS * lt * 2;
        for (int t = 0; t < lt; t++) {
            for (int gi = 0; gi < 16; gi++) {
                Cd v = gp(gi, r + t * 32);
                o[2 * (gi * lt + t)] = v.real();
                o[2 * (gi * lt + t) + 1] = v.imag();
                for (int nu = 0; nu < 4; nu++) {
                    Cd d = der(r, gi, nu, t);
                    int op = 16 + 4 * gi + nu;
                    o[2 * (op * lt + t)] = d.real();
                    o[2 * (op * lt + t) + 1] = d.imag();
                }
            }
            int i = 0;
            for (int m = 0; m < 4; m++)
                for (int nn = m; nn < 4; nn++, i++) {
                    Cd v = 0.5 * (der(r, 1 + m, nn, t) + der(r, 1 + nn, m, t));
                    o[2 * ((80 + i) * lt + t)] = v.real();
                    o[2 * ((80 + i) * lt + t) + 1] = v.imag();
                }
        }
    }
    return TM_OK;
}

// ---------------------------------------------------------------------------
// loops with the truncated solver method
// ---------------------------------------------------------------------------
// estimators of tsm_run: eta^dag G s; the one-end trick (isovector, isoscalar);
// eta^dag G s and the hopping parameter expansion from the same solves
enum Est { EST_STD = 0, EST_OET = 1, EST_HPE = 2 };
// time dilution (Sec. 2.3): noise vector r becomes one source per phase p,
// eta_r on the timeslices t = p mod spacing; spacing 0 = undiluted
struct Dil {
    int spacing = 0;
    std::vector<int> phases;
};
int tsm_run(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P, double *est, double *vre, double *vim,
            double *raw_host, tm_tsm_stats *stats, Est mode = EST_STD, const Dil &dil = Dil());

extern "C" int tm_loops_tsm(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P, double *est, double *var_re,
                            double *var_im, double *raw, tm_tsm_stats *stats)
{
    if (!ctx) return TM_ERR_ARG;
    return tsm_run(ctx, G, P, est, var_re, var_im, raw, stats);
}

extern "C" int tm_loops_oet(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P, double *est, double *var_re,
                            double *var_im, double *raw, tm_tsm_stats *stats)
{
    if (!ctx) return TM_ERR_ARG;
    return tsm_run(ctx, G, P, est, var_re, var_im, raw, stats, EST_OET);
}

extern "C" int tm_loops_hpe(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P, double *est, double *var_re,
                            double *var_im, double *raw, tm_tsm_stats *stats)
{
    if (!ctx) return TM_ERR_ARG;
    if (G && G->ctx == ctx)
        for (int d = 0; d < 4; d++)
            if (G->dims[d] < 4)
                return set_err(ctx, TM_ERR_ARG, "tm_loops_hpe: every extent must be >= 4 (got %d)", G->dims[d]);
    return tsm_run(ctx, G, P, est, var_re, var_im, raw, stats, EST_HPE);
}

extern "C" int tm_loops_tdil(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P, int spacing,
                             const int *phases, int n_phases, int hpe, double *est, double *var_re, double *var_im,
                             double *raw, tm_tsm_stats *stats)
{
    if (!ctx) return TM_ERR_ARG;
    if (!G || !P || G->ctx != ctx) return set_err(ctx, TM_ERR_ARG, "tm_loops_tdil: null gauge/parameters or another context's gauge");
    const int lt = G->dims[3];
    if (spacing < 1 || spacing > lt || lt % spacing)
        return set_err(ctx, TM_ERR_ARG, "tm_loops_tdil: spacing must divide the time extent %d (got %d)", lt, spacing);
    Dil dil;
    dil.spacing = spacing;
    if (!phases) {
        for (int p = 0; p < spacing; p++) dil.phases.push_back(p);
    } else {
        if (n_phases < 1 || n_phases > spacing) return set_err(ctx, TM_ERR_ARG, "tm_loops_tdil: need 1..spacing phases");
        std::vector<char> seen(spacing, 0);
        for (int k = 0; k < n_phases; k++) {
            const int p = phases[k];
            if (p < 0 || p >= spacing || seen[p])
                return set_err(ctx, TM_ERR_ARG, "tm_loops_tdil: phases must be distinct and in [0, spacing)");
            seen[p] = 1;
            dil.phases.push_back(p);
        }
    }
    if ((size_t)(2 * P->n_hp + P->n_lp) * dil.phases.size() > (size_t)1 << 26)
        return set_err(ctx, TM_ERR_ARG, "tm_loops_tdil: too many solves");
    if (hpe)
        for (int d = 0; d < 4; d++)
            if (G->dims[d] < 4)
                return set_err(ctx, TM_ERR_ARG, "tm_loops_tdil: the expansion needs every extent >= 4 (got %d)",
                               G->dims[d]);
    return tsm_run(ctx, G, P, est, var_re, var_im, raw, stats, hpe ? EST_HPE : EST_STD, dil);
}

// insertion tables of the one-end trick: g5 G (flavour 0) and g5 G g5 (flavour 1),
// from the table of G (entry = column | phase << 2, phase 0..3 = 1, i, -1, -i)
static void oet_gamma_tables(int vv[64], int ws[64])
{
    const int *g = gamma_table();
    for (int gi = 0; gi < 16; gi++)
        for (int a = 0; a < 4; a++) {
            const int e = g[4 * gi + a], col = e & 3, ph = e >> 2;
            const int fa = a >= 2 ? 2 : 0, fc = col >= 2 ? 2 : 0;
            vv[4 * gi + a] = col | (((ph + fa) & 3) << 2);
            ws[4 * gi + a] = col | (((ph + fa + fc) & 3) << 2);
        }
}

int tsm_check(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P)
{
    if (!G || !P) return set_err(ctx, TM_ERR_ARG, "null gauge or parameters");
    if (G->ctx != ctx) return set_err(ctx, TM_ERR_ARG, "gauge field belongs to another context");
    if (P->n_hp < 0 || P->n_lp < 0 || P->n_hp + P->n_lp < 1)
        return set_err(ctx, TM_ERR_ARG, "need n_hp >= 0, n_lp >= 0 and at least one source");
    if (P->n_hp + P->n_lp > (1 << 24)) return set_err(ctx, TM_ERR_ARG, "too many sources");
    if (P->batch < 0 || P->batch > MAX_SLOTS) return set_err(ctx, TM_ERR_ARG, "batch must be 0..%d", MAX_SLOTS);
    if (P->ops != 0 && P->ops != 1) return set_err(ctx, TM_ERR_ARG, "ops must be 0 (all) or 1 (local only)");
    int rc = TM_OK;
    if (P->n_hp > 0 && (rc = check_solver(ctx, G, &P->hp))) return rc;
    if ((rc = check_solver(ctx, G, &P->lp))) return rc;
    return TM_OK;
}

// (operator, t) entries an estimator covers: with time dilution, local and
// spatial-derivative loops need the noise on t, the time-derivative loops
// (and the symmetrised operators containing one) on t - 1, t and t + 1; the
// expansion covers the 16 local loops only
static void valid_mask(int lt, const Dil &dil, bool local_only, unsigned char *m)
{
    std::vector<unsigned char> cov(lt, 1), wide(lt, 1);
    if (dil.spacing > 0)
        for (int t = 0; t < lt; t++) {
            cov[t] = 0;
            for (int p : dil.phases) cov[t] |= (unsigned char)(t % dil.spacing == p);
        }
    for (int t = 0; t < lt; t++) wide[t] = cov[t] && cov[(t + 1) % lt] && cov[(t + lt - 1) % lt];
    for (int op = 0; op < TM_N_OPS; op++) {
        bool tder = false;
        if (op >= 16 && op < 80) tder = (op - 16) % 4 == 3;
        if (op >= 80) {
            int i = op - 80, m = 0;
            while (i >= 4 - m) i -= 4 - m++;
            tder = m == 3 || m + i == 3;
        }
        for (int t = 0; t < lt; t++)
            m[op * lt + t] = (local_only && op >= 16) ? 0 : tder ? wide[t] : cov[t];
    }
}

int tsm_run(tm_context *ctx, const tm_gauge *G, const tm_tsm_params *P, double *est, double *vre, double *vim,
            double *raw_host, tm_tsm_stats *stats, Est mode, const Dil &dil)
{
    const bool oet = mode == EST_OET, hpe = mode == EST_HPE;
    if (!est || !vre || !vim) return set_err(ctx, TM_ERR_ARG, "tm_loops: null output");
    int rc = tsm_check(ctx, G, P);
    if (rc) return rc;
    const int batch = P->batch > 0 ? std::min(P->batch, MAX_SLOTS) : 12;
    TM_HIP(ctx, hipSetDevice(ctx->device));
    const double t0 = now_s();
    const int lt = G->dims[3];
    const int n_hp = P->n_hp, n_lpt = P->n_hp + P->n_lp;
    // estimators: eta^dag G s; the isovector and isoscalar one-end trick; or
    // eta^dag G s and the expansion's stochastic term eta^dag G (BH)^4 s
    const int nf = mode == EST_STD ? 1 : 2;
    const size_t raw_per = (size_t)9 * lt * 32;  // doubles per source
    const size_t ops_per = (size_t)TM_N_OPS * lt * 2;
    const size_t n_ids = (size_t)(n_hp + n_lpt);
    const size_t src_raw = n_ids * raw_per, src_ops = n_ids * ops_per;
    // with more than one phase each solve has its own spin matrices, summed
    // per noise vector in phase order afterwards
    const int nph = dil.spacing > 0 ? (int)dil.phases.size() : 1;
    const size_t job_raw = nph > 1 ? n_ids * nph * raw_per : 0;  // per flavour
    const size_t mask_doubles = ((size_t)nf * TM_N_OPS * lt + 7) / 8;
    const size_t dev_doubles =
        nf * (src_raw + job_raw + src_ops + ops_per * 2) + (hpe ? raw_per + ops_per : 0) + mask_doubles;
    double *dbuf = (double *)dalloc(ctx, dev_doubles * sizeof(double));
    if (!dbuf) return set_err(ctx, TM_ERR_NOMEM, "tm_loops: no memory for per-source loops");
    // the expansion's (and a local-only run's) raw spin matrices carry the local kind only
    if (hpe || P->ops == 1) {
        hipError_t e = hipMemsetAsync(dbuf, 0, dev_doubles * sizeof(double), nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) {
            dfree(ctx, dbuf);
            return set_err(ctx, TM_ERR_HIP, "tm_loops_hpe: clearing the loop buffers: %s", hipGetErrorString(e));
        }
    }
    // flavour f: raw [n_hp | n_lpt] sources, ops likewise, then est and variances
    auto raw_hp = [&](int f) { return dbuf + f * src_raw; };
    auto raw_lp = [&](int f) { return raw_hp(f) + n_hp * raw_per; };
    double *jobb = dbuf + nf * src_raw;
    // spin matrices of the solve of noise vector i (HP, or LP), phase k
    auto job_out = [&](int f, bool is_hp, int i, int k) {
        if (nph == 1) return (is_hp ? raw_hp(f) : raw_lp(f)) + (size_t)i * raw_per;
        return jobb + f * job_raw + ((is_hp ? 0 : (size_t)n_hp) + i) * nph * raw_per + (size_t)k * raw_per;
    };
    double *opsb = jobb + nf * job_raw;
    auto ops_hp = [&](int f) { return opsb + f * src_ops; };
    auto ops_lp = [&](int f) { return ops_hp(f) + n_hp * ops_per; };
    double *estb = opsb + nf * src_ops;
    auto d_est = [&](int f) { return estb + f * 2 * ops_per; };
    double *raw_exact = estb + nf * 2 * ops_per, *ops_exact = raw_exact + raw_per;  // HPE only
    unsigned char *d_mask = (unsigned char *)(estb + nf * 2 * ops_per + (hpe ? raw_per + ops_per : 0));
    std::vector<Job> hp((size_t)n_hp * nph), lp((size_t)n_lpt * nph);
    std::vector<Job *> qh, ql;
    auto make = [&](Job &j, bool is_hp, int i, int k) {
        j.noise = true;
        j.seed = P->noise_seed;
        j.src = i;
        j.tmod = dil.spacing;
        j.tph = dil.spacing > 0 ? dil.phases[k] : 0;
        job_from(j, is_hp ? P->hp : P->lp, P->kappa, P->two_kappa_mu);
        j.raw_out = job_out(0, is_hp, i, k);
        j.oet = oet;
        j.hpe = hpe;
        j.local_only = P->ops == 1;
        j.raw_out2 = nf > 1 ? job_out(1, is_hp, i, k) : nullptr;
        j.want_true = P->want_true_resid;
        j.hp = is_hp;
    };
    for (int i = 0; i < n_hp; i++)
        for (int k = 0; k < nph; k++) {
            make(hp[(size_t)i * nph + k], true, i, k);
            qh.push_back(&hp[(size_t)i * nph + k]);
        }
    for (int i = 0; i < n_lpt; i++)
        for (int k = 0; k < nph; k++) {
            make(lp[(size_t)i * nph + k], false, i, k);
            ql.push_back(&lp[(size_t)i * nph + k]);
        }
    std::vector<Batch *> bs;
    std::vector<std::vector<Job *>> qs;
    std::vector<hipStream_t> streams;
    auto add = [&](Kind k, const tm_solver_params &sp, std::vector<Job *> &q) -> int {
        hipStream_t st;
        TM_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        streams.push_back(st);
        Batch *B = nullptr;
        int e = batch_create(ctx, G, k, std::min<int>(batch, (int)q.size()), sp.chunk, st, &B);
        if (e) return e;
        bs.push_back(B);
        qs.push_back(q);
        return TM_OK;
    };
    if (n_hp > 0) rc = add(kind_of(P->hp), P->hp, qh);
    // LP sources split over lp_batches batches on their own streams, so one
    // batch's host turnaround (harvest, refill) overlaps another's kernels
    static const int lp_batches = std::max(1, std::min(4, [] {
        const char *e = getenv("TM_LP_BATCHES");
        return e ? atoi(e) : 1;
    }()));
    const int nlb = std::max(1, std::min<int>(lp_batches, (int)(ql.size() + batch - 1) / batch));
    for (int k = 0; k < nlb && !rc; k++) {
        std::vector<Job *> part(ql.begin() + ql.size() * k / nlb, ql.begin() + ql.size() * (k + 1) / nlb);
        rc = add(kind_of(P->lp), P->lp, part);
    }
    if (!rc) rc = run_jobs(bs, qs);
    double hp_end = 0, lp_end = 0;
    for (Batch *B : bs) {
        if (B == bs.front() && n_hp > 0) hp_end = B->t_last;
        else lp_end = std::max(lp_end, B->t_last);
        batch_destroy(B);
    }
    hipStream_t s = streams.empty() ? nullptr : streams.back();
    std::vector<unsigned char> mask;  // host source of an async copy: outlives the stream syncs below
    if (!rc) {
        for (hipStream_t x : streams) hipStreamSynchronize(x);
        int tv[64], tw[64];
        if (oet) oet_gamma_tables(tv, tw);
        if (hpe) {
            launch_hpe_exact(G->g, P->kappa, P->two_kappa_mu, raw_exact, s);
            launch_project(1, lt, raw_exact, ops_exact, gamma_table(), s);
        }
        // covered entries per flavour (the rest NaN); masks only where some entry is not covered
        mask.assign((size_t)nf * TM_N_OPS * lt, 0);
        bool masked[2] = {false, false};
        for (int f = 0; f < nf; f++) {
            unsigned char *m = mask.data() + (size_t)f * TM_N_OPS * lt;
            valid_mask(lt, dil, (hpe && f == 1) || P->ops == 1, m);
            for (size_t q = 0; q < (size_t)TM_N_OPS * lt; q++) masked[f] |= m[q] == 0;
        }
        hipError_t e = hipMemcpyAsync(d_mask, mask.data(), mask.size(), hipMemcpyHostToDevice, s);
        for (int f = 0; f < nf && e == hipSuccess; f++) {
            if (nph > 1) {
                launch_sum_phases(job_out(f, true, 0, 0), raw_hp(f), n_hp, nph, raw_per, s);
                launch_sum_phases(job_out(f, false, 0, 0), raw_lp(f), n_lpt, nph, raw_per, s);
            }
            const int *gt = !oet ? gamma_table() : f == 0 ? tv : tw;
            double *de = d_est(f), *dvre = de + ops_per, *dvim = dvre + ops_per / 2;
            launch_project(n_hp, lt, raw_hp(f), ops_hp(f), gt, s);
            launch_project(n_lpt, lt, raw_lp(f), ops_lp(f), gt, s);
            // HPE flavour: exact part added to the 16 local loops, the others undefined
            const bool hf = hpe && f == 1;
            launch_tsm_combine(n_hp, P->n_lp, lt, ops_hp(f), ops_lp(f), ops_lp(f) + (size_t)n_hp * ops_per, de, dvre,
                               dvim, s, hf ? ops_exact : nullptr,
                               masked[f] ? d_mask + (size_t)f * TM_N_OPS * lt : nullptr);
            e = hipMemcpyAsync(est + f * ops_per, de, ops_per * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(vre + f * ops_per / 2, dvre, ops_per / 2 * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(vim + f * ops_per / 2, dvim, ops_per / 2 * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && raw_host)
                e = hipMemcpyAsync(raw_host + f * src_raw, raw_hp(f), src_raw * sizeof(double), hipMemcpyDeviceToHost,
                                   s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = set_err(ctx, TM_ERR_HIP, "tm_loops: %s", hipGetErrorString(e));
    }
    for (hipStream_t x : streams) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
    }
    dfree(ctx, dbuf);
    const double t1 = now_s();
    int worst = TM_OK;
    const Job *bad = nullptr;  // first solve that ended with non-finite values
    if (stats) std::memset(stats, 0, sizeof(*stats));
    for (auto *v : {&hp, &lp})
        for (Job &j : *v) {
            if (j.status == TM_ERR_NUMERIC && !bad) bad = &j;
            if (stats) {
                if (j.hp) {
                    stats->hp_solves++;
                    stats->hp_iters += j.iters;
                    stats->hp_max_iters = std::max(stats->hp_max_iters, j.iters);
                    stats->max_hp_true_resid = std::max(stats->max_hp_true_resid, j.true_rel);
                } else {
                    stats->lp_solves++;
                    stats->lp_iters += j.iters;
                    stats->lp_max_iters = std::max(stats->lp_max_iters, j.iters);
                    stats->max_lp_true_resid = std::max(stats->max_lp_true_resid, j.true_rel);
                }
                stats->reliable_updates += j.updates;
            }
            if (j.status == TM_ERR_NUMERIC) worst = TM_ERR_NUMERIC;
            else if (j.status == TM_ERR_NOCONV && worst == TM_OK) worst = TM_ERR_NOCONV;
        }
    if (stats) {
        stats->seconds = t1 - t0;
        stats->hp_seconds = hp_end > 0 ? hp_end - t0 : 0;
        stats->lp_seconds = lp_end > 0 ? lp_end - t0 : 0;
    }
    if (rc) return rc;
    if (worst == TM_ERR_NUMERIC)
        return set_err(ctx, worst,
                       "tm_loops: non-finite values in a solve (%s source %llu, phase %d: iteration %d, |r|^2 %.3e "
                       "-> %.3e, pAp %.3e, alpha %.3e, beta %.3e)",
                       bad->hp ? "HP" : "LP", (unsigned long long)bad->src, bad->tph, bad->end.iter, bad->end.rr,
                       bad->end.rr_new, bad->end.pap, bad->end.alpha, bad->end.beta);
    if (worst == TM_ERR_NOCONV) return set_err(ctx, worst, "tm_loops: a solve reached max_iter");
    return TM_OK;
}

// ---------------------------------------------------------------------------
// measurement helpers
// ---------------------------------------------------------------------------
extern "C" int tm_stream_copy(tm_context *ctx, const void *src, void *dst, size_t bytes, void *hip_stream)
{
    if (!ctx) return TM_ERR_ARG;
    if (!src || !dst || bytes % 16 || overlap(src, bytes, dst, bytes))
        return set_err(ctx, TM_ERR_ARG, "tm_stream_copy: bad arguments (bytes must be a multiple of 16)");
    launch_stream_copy(src, dst, bytes, (hipStream_t)hip_stream);
    TM_HIP(ctx, hipGetLastError());
    return TM_OK;
}

extern "C" int tm_selftest(void)
{
    // fast division against the hardware divide
    uint64_t x = 88172645463325252ull;
    for (uint32_t d = 1; d <= 4096; d++) {
        FastDiv f = make_fastdiv(d);
        for (int k = 0; k < 2000; k++) {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            uint32_t n = (uint32_t)(x & 0x7FFFFFFFu);
            if (k < 64) n = (uint32_t)k * d + (uint32_t)(k & 3) - 1u;
            if (fastdiv_host(n, f) != n / d) return 1;
        }
    }
    // gamma table: one entry per row, all 16 insertions built
    const int *t = gamma_table();
    for (int i = 0; i < 64; i++)
        if (t[i] < 0 || t[i] > 15) return 2;
    // geometry: strides and per-timeslice ranges
    int dims[4] = {6, 4, 2, 8};
    Geom g = make_geom(dims, -1);
    if (g.vh != 6 * 4 * 2 * 8 / 2 || g.v3h * dims[3] != g.vh || g.st != g.v3h) return 3;
    // lattice size limit of the 32-bit buffer offsets
    {
        const int fit[3][4] = {{32, 32, 32, 64}, {48, 48, 48, 96}, {2, 2, 2, 2}};
        const int big[3][4] = {{64, 64, 64, 64}, {56, 56, 56, 64}, {1024, 1024, 16, 2}};
        for (int k = 0; k < 3; k++)
            if (!lattice_fits(fit[k]) || lattice_fits(big[k])) return 9;
    }
    // arena: random allocations and releases keep blocks disjoint, in range,
    // aligned, and coalesce back to one free block
    {
        tmi::Arena A;
        char *base = (char *)(uintptr_t)0x10000000;
        const size_t size = 1 << 24;
        A.init(base, size);
        std::vector<std::pair<char *, size_t>> live;
        uint64_t z = 12345;
        for (int it = 0; it < 20000; it++) {
            z = z * 6364136223846793005ull + 1442695040888963407ull;
            if ((z >> 33) % 3 && live.size() < 200) {
                size_t n = 1 + (z >> 40) % 300000;
                char *p = (char *)A.alloc(n);
                if (!p) continue;
                if ((size_t)(p - base) % 256 || p < base || p + n > base + size) return 4;
                for (auto &q : live)
                    if (p < q.first + q.second && q.first < p + n) return 5;
                live.push_back({p, n});
            } else if (!live.empty()) {
                size_t k = (z >> 20) % live.size();
                A.release(live[k].first);
                live.erase(live.begin() + k);
            }
        }
        for (auto &q : live) A.release(q.first);
        if (A.used != 0 || A.largest_free() != size || A.free_.size() != 1) return 6;
    }
    return 0;
}
