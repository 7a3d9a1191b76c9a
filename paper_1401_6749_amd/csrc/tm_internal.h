// Host-side internals of libtm: context, gauge handles and the slot engine
// that runs many independent CG solves ("slots") in multi-RHS launches.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "tm.h"
#include "tm_launch.h"
#include "tm_types.h"
#include "tm_jobs.h"


struct tm_context {
    int device = 0;
    size_t budget = 0;
    size_t in_use = 0, peak = 0;
    tm_alloc_fn alloc = nullptr;
    tm_free_fn free_fn = nullptr;
    void *user = nullptr;
    mutable std::mutex mu;  // allocation table and error string
    std::unordered_map<void *, size_t> allocs;
    std::string err;
    int swz = 1;         // XCD-aware block mapping
    std::atomic<int> use_graphs{1};  // capture CG chunks in hipGraphs (a serving worker may clear it)
    // scratch of tm_dslash (grown on demand)
    void *op_tmp = nullptr;
    size_t op_tmp_bytes = 0;
    // scratch of tm_contract: Z4 codes and partial sums (grown on demand)
    void *ct_tmp = nullptr;
    size_t ct_tmp_bytes = 0;
};

struct tm_gauge {
    tm_context *ctx = nullptr;
    int dims[4] = {0, 0, 0, 0};
    int tbc = -1;
    tmk::Geom g;
    unsigned precs = 0;  // bit (1 << P) per built precision
    void *links[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace tmi {

int set_err(tm_context *c, int code, const char *fmt, ...);
void *dalloc(tm_context *c, size_t bytes);
void dfree(tm_context *c, void *p);
double now_s();

#define TM_HIP(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return tmi::set_err((ctx), TM_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Slot engine
// ---------------------------------------------------------------------------


struct Batch {
    tm_context *ctx = nullptr;
    Mem mem;
    const tm_gauge *G = nullptr;
    Kind kind = K_F64;
    int sp = tmk::P64, xr = tmk::P64;
    int S = 1;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    size_t hsp = 0, hxr = 0;  // slot pitches of the CG fields (padded)
    size_t h64 = 0;           // FP64 half field (unpadded: scratch halves are adjacent)
    char *p = nullptr, *u = nullptr, *t = nullptr, *x = nullptr, *r = nullptr;
    char *x64 = nullptr, *b64 = nullptr;
    uint32_t *codes = nullptr;
    char *FA = nullptr, *FB = nullptr, *FC = nullptr;  // scratch: FP64 full field [even | odd], or per-slot halves
    char *FD = nullptr;       // fourth per-slot scratch half (low-precision kinds: one-end trick)
    int wpp = tmk::P64;       // precision of the per-slot scratch halves
    size_t wpitch = 0;        // their slot pitch
    int wslots = 1;           // slots a run may span
    double *partial = nullptr;
    int nblk = 0;
    double *cpart = nullptr;
    double *dres = nullptr;     // small device results
    double *hres = nullptr;     // pinned mirror
    tmk::SlotState *st = nullptr;
    tmk::SlotState *st_h = nullptr;  // pinned
    std::vector<Job *> slot_job;
    std::vector<int> slot_updates;
    std::vector<int> slot_pending_update;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int g_iters = 0;
    bool in_flight = false;
    int chunk = 8;
    size_t bytes = 0;
    double t_first = 0, t_last = 0;
    long long iters_done = 0;
};

size_t batch_footprint(const tm_gauge *G, Kind kind, int S);
int batch_create(tm_context *ctx, const tm_gauge *G, Kind kind, int S, int chunk, hipStream_t stream, Batch **out,
                 const Mem *mem = nullptr);
void batch_destroy(Batch *b);
int batch_fill(Batch *b, int slot, Job *j);
// place up to n jobs into free slots (noise solves with equal kappa, a in
// consecutive slots are prepared together); returns the number placed
int batch_fill_many(Batch *b, Job *const *jobs, int n);
int batch_launch_chunk(Batch *b);
// after the chunk's event completed: reliable updates and harvests; fills
// *finished with the jobs that completed.  Returns tm_status.
int batch_process(Batch *b, std::vector<Job *> &finished);
int batch_active(const Batch *b);
int batch_free_slot(const Batch *b);

// Run queues of jobs on a set of batches until all are finished.
int run_jobs(std::vector<Batch *> &batches, std::vector<std::vector<Job *>> &queues);

Kind kind_of(const tm_solver_params &p);
int kind_prec(Kind k);  // storage precision of the Dslash operands
int auto_chunk(const tm_gauge *G, Kind k, int S);

}  // namespace tmi
