// Host-side description of one solve ("job") of the slot engine and of the
// solver kinds, shared by the engine, the C ABI and the serving scheduler.
// No HIP types: the serving scheduler is also built without the runtime.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "tm_types.h"

namespace tmi {

// Reliable-update threshold of the mixed solver when the caller passes 0:
// the FP32 recursion carries the residual down three orders of magnitude
// before the FP64 true residual replaces it, four orders above FP32 rounding.
constexpr double TM_DEFAULT_DELTA = 1e-3;

enum Kind { K_F64 = 0, K_MIXED = 1, K_LP16 = 2, K_LPBF = 3 };

// solver kind of a set of solver parameters (tm_solve_mode values; half
// precision 8 = BF16)
inline Kind kind_of_mode(int mode, int half_prec)
{
    if (mode == 1) return K_MIXED;
    if (mode == 2) return half_prec == 8 ? K_LPBF : K_LP16;
    return K_F64;
}

// Device memory source of a batch: the context allocator by default, or a
// serving engine's arena.
struct Mem {
    void *(*alloc)(void *self, size_t bytes) = nullptr;
    void (*free)(void *self, void *p) = nullptr;
    void *self = nullptr;
};

struct Job {
    // input
    bool noise = true;
    uint64_t seed = 0, src = 0;
    const double *b_canon = nullptr;  // explicit right-hand side (device, canonical)
    double *x_canon = nullptr;        // explicit solution output (device, canonical)
    double kappa = 0, a = 0;
    double tol = 1e-10;
    int max_iter = 100000;
    int fixed = 0;
    double delta = 0.1;
    double *raw_out = nullptr;  // noise: device [9][T][16][2] (one-end trick: the isovector part)
    bool oet = false;           // one-end trick estimators instead of eta^dag G s
    double *raw_out2 = nullptr; // one-end trick: the isoscalar part; HPE: eta^dag G (BH)^4 s (kind 0) [9][T][16][2]
    bool hpe = false;           // also the stochastic term of the hopping parameter expansion
    bool local_only = false;    // local spin matrices only (kind 0)
    int tmod = 0, tph = 0;      // time dilution: eta only on the timeslices t = tph mod tmod (tmod 0: all)
    int want_true = 0;
    // output
    int status = 0;  // tm_status
    int iters = 0, updates = 0;
    double cg_rel = 0, true_rel = -1;
    tmk::SlotState end{};  // slot state at the end of the solve (diagnostics)
    double t_fill = 0, t_done = 0;
    // owner bookkeeping
    void *owner = nullptr;
    int owner_idx = 0;
    bool hp = false;
};

}  // namespace tmi
