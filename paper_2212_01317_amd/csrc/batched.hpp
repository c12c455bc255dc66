// Device-side structures of the batched conditional simulation (batched.hip) and its launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mpr_internal.hpp"

namespace mpr {

// One scene, as the batched kernels read it.  Geometry is kept for both tile heights (index 0: 16, 1: 32).
struct BatchScene {
    const float* t;
    const uint8_t* mask;
    const TBand* tp;
    float* buf[2];        // state after an even / odd number of sweeps
    double* acc;
    long long* epart;     // [R][max tiles] energy partials (fixed point)
    double* e_real;       // [R]
    double* series;       // [cap + 1] realization-averaged energy per bond
    int H, W, lb_h, lb_w, nbx, ntx, Mw;
    int nty[2], ntiles[2], rchunk[2], nchunks[2];
    int64_t HW;
    uint32_t scene;
    double inv_norm;      // 1 / (J * number of bonds)
};

struct BatchRun {
    int phase;            // 0 equilibrating, 1 sampling, 2 done
    int k_star;           // equilibration sweeps
    int samp;             // sampling sweeps accumulated
    int converged;        // 0 when the cap ended equilibration
};

struct BatchCtl {
    int k;                        // sweeps done
    int n_active;                 // scenes not done
    unsigned long long queue;     // work-queue head of the current sweep
};

struct BatchCfg {
    int R;
    uint32_t real_offset, key0, key1;
    float q, J, delta_e;
    double two_pi_q, Jd;
    int energy;                   // record energies (AUTO mode, or requested)
    int stop_mode, n_fit, n_f, n_max, n_eq, n_samp;
};

struct BatchDev {
    BatchScene* scenes;
    BatchRun* runs;
    int* order;                   // scenes, largest work first
    int64_t* prefix;              // [n + 1] work-list prefix over `order` (scenes still running)
    BatchCtl* ctl;
    BatchCfg cfg;
    int n;
};

// ---- the batch on the realization-lane sweep (runs with 64 or more realizations) ----
// One scene as the lane batch reads it: the arguments of its lane sweep (the sweep index is set per launch), its
// window bits, temperature table, the two state buffers in the lane layout, and the per-scene reductions.
struct BatchLaneScene {
    RlArgs a;
    const uint2* cells;
    const TBand* tb;
    float* buf[2];        // [G][HW][64]: state after an even / odd number of sweeps
    double* acc;
    const uint8_t* mask;
    long long* epart;     // [R][nparts] energy partials (fixed point)
    double* e_real;       // [R]
    double* series;       // [cap + 1]
    int64_t HW;
    int64_t work;         // work items of one sweep (waves)
    int nparts;           // nbands * nseg
    double inv_norm;      // 1 / (J * number of bonds)
};

// Eight work queues, one per XCD: XCD x takes the items [bound[x], bound[x + 1]) of the work list in order, so
// adjacent bands of a scene run on one XCD (their shared columns come from its L2 cache); the bounds split the
// estimated time of the sweep (sites and gap sites of the running scenes) into eighths.
struct BatchLaneCtl {
    int k;
    int n_active;
    unsigned long long queue[8];
    int64_t bound[9];
};

struct BatchLaneDev {
    BatchLaneScene* scenes;
    BatchRun* runs;
    int* order;
    int64_t* prefix;
    BatchLaneCtl* ctl;
    BatchCfg cfg;
    int n;
    int tm;               // temperature lookup of every scene's sweep (TM_ALIGNED / TM_TWO / TM_ANY)
    const int64_t* gaps;  // [n] gap sites of each scene
};

// the persistent lane sweep of all running scenes (rl_sweep.hip)
hipError_t launch_batchl_sweep(const BatchLaneDev& b, int grid, hipStream_t s);
// one sweep of the lane batch: counter, sweep, energies, accumulation, phases and the next work list
hipError_t launch_batchl_step(const BatchLaneDev& b, int grid, int acc_blocks, hipStream_t s);
// the XCD bounds of the current work list (before the first sweep; the phase kernel renews them after each sweep)
hipError_t launch_batchl_bounds(const BatchLaneDev& b, hipStream_t s);
// *out += number of gap sites (mask 0) among mask[0 .. HW)
hipError_t launch_count_gaps(const uint8_t* mask, int64_t HW, int64_t* out, hipStream_t s);

hipError_t launch_batch_sweep(const BatchDev& b, int variant, int grid, hipStream_t s);
hipError_t launch_batch_step(const BatchDev& b, int variant, int next_variant, int grid, int acc_blocks,
                             hipStream_t s);

}  // namespace mpr
