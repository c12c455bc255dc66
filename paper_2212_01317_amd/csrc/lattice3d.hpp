// Declarations of the 3D lattice (lattice3d.hip), kept apart from mpr_internal.hpp so that the plane's kernels do
// not depend on them.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mpr_internal.hpp"

namespace mpr {

// ---- the 3D lattice (lattice3d.hip): grids D x H x W, site n = (z H + y) W + x, six neighbours, blocks
// lb_d x lb_h x lb_w ----
// The FP32 filter's bound on |dE_fp32 - dE_exact| / J with six neighbours: |(Cx, Sy)| <= 6 makes the terms of the
// plane's derivation 3/2 as large, about 2.3e-5 with every FP32 rounding; 2.75e-5 leaves margin.
constexpr float kDeltaE3 = 2.75e-5f;
constexpr int kB3 = 8;           // owned columns of a wave of the 3D sweep (16 would need more than 256 VGPRs)
constexpr int kZSeg3 = 64;       // planes of a wave's segment
constexpr int kNW3 = 4;          // waves (consecutive rows) of a workgroup of the 3D sweep
struct Lat3Args {
    int D, H, W, R, Rp, Mw, nbands, nzseg, zseg;
    int nrows;                   // row tiles of kNW3 rows
    int lb_d, lb_h, lb_w, nbx, nby;
    uint32_t lbw_inv;            // ceil(2^32 / lb_w) for lb_w > 1
    uint32_t sweep, real_offset, scene, key0, key1;
    int colour;
    float q, J, delta_e;
    double two_pi_q, Jd;
};
int64_t lat3_blocks(int64_t D, int64_t H, int64_t W, int lb_d, int lb_h, int lb_w);
// S[b], N[b], Tsum[b], Nobs[b] of Eq. (2) per 3D block (bonds to the +x, +y, +z neighbour)
hipError_t launch_block_stats3(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W, int lb_d,
                               int lb_h, int lb_w, double two_pi_q, double J, double* S, int* N, double* Ts, int* No,
                               hipStream_t s);
struct Init3Args {
    float* state;                // [R][n]
    const float* t;
    const uint8_t* mask;
    const double* Ts;
    const int* No;
    const float* gmean;
    int64_t D, H, W;
    int lb_d, lb_h, lb_w, nbx, nby;
    int R;
    uint32_t real_offset, scene, key0, key1;
    int mode;
};
hipError_t launch_init3(const Init3Args& a, hipStream_t s);
// fixed-point energy partials of every realization of a [R][n] state (bonds to +x, +y, +z), layout [R][nparts]
int energy3_parts(int64_t D, int64_t H, int64_t W);
hipError_t launch_energy3_full(const float* state, int64_t D, int64_t H, int64_t W, int R, float q, long long* partial,
                               int nparts, hipStream_t s);
// gap bits of each row's window columns: [(D H) nbands]
hipError_t launch_cells3(const uint8_t* mask, int64_t D, int64_t H, int64_t W, int nbands, uint32_t* cells,
                         hipStream_t s);
// one half-sweep (colour a.colour, all rows) of the lane-layout state [G][n][64], in place; with epart set, the
// fixed-point energy of each row's colour-1 sites goes to epart[r][(y * nbands + band) * nzseg + zseg]
hipError_t launch_sweep3(const Lat3Args& a, const uint32_t* cells, const TBand* tb, float* state, long long* epart,
                         hipStream_t s);
// the matching curve of the cubic lattice: periodic L^3, one chain per temperature
hipError_t launch_ref3_half(float* state, const float* Tgrid, int nT, int L, uint32_t sweep, int colour, float q,
                            float delta_e, uint32_t key0, uint32_t key1, double two_pi_q, hipStream_t s);
int ref3_energy_parts(int L);
hipError_t launch_ref3_energy(const float* state, int L, int nT, float q, double* partial, int nparts, hipStream_t s);

}  // namespace mpr
