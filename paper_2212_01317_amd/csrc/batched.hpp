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

hipError_t launch_batch_sweep(const BatchDev& b, int variant, int grid, hipStream_t s);
hipError_t launch_batch_step(const BatchDev& b, int variant, int next_variant, int grid, int acc_blocks,
                             hipStream_t s);

}  // namespace mpr
