// Internal declarations shared by the host API and the kernel launchers of libmpr (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mpr {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Absolute bound on |dE_fp32 - dE_exact| / J for the FP32 Metropolis filter of the sweep kernels.  Derivation:
// every stored cos/sin of an angle carries at most e = 3.2e-7 absolute error (the gfx950 v_sin/v_cos_f32 error
// measured exhaustively over [0, 1/2] revolution is 1.25e-7; rounding of q * t adds at most 2 pi * 2^-25);
// dE/J = -((c' - c) Cx + (s' - s) Sy) with |(c' - c, s' - s)| <= 2 and |(Cx, Sy)| <= 4 accumulates at most
// 22.6 e + 3.7e-6 including every FP32 rounding; 1.25e-5 leaves margin.
constexpr float kDeltaE = 1.25e-5f;

// Per-block temperature as the sweep keeps it in LDS, with the constants of its FP32 filter: kappa = J log2(e) / T
// (0 when T == 0), the band terms of the filter's error bound (band, and kb per unit |X|).
struct alignas(16) TBand {
    float T, kappa, band, kb;
};
// Directional coupling (one temperature per bond direction): the filter's y = log2 of the acceptance ratio is
// X_h kx + X_v ky with kx = J log2(e) / Tx, ky = J log2(e) / Ty; its error band is band + |X_h| kbx + |X_v| kby.
struct alignas(16) TBandDir {
    float Tx, Ty, kx, ky, kbx, kby, band, pad;
};
// The lowest directional temperature, in units of J.
constexpr double kTMinDirectional = 1e-3;
hipError_t launch_tpairs_directional(const float* T, int64_t B, float J, float delta, float floor_T, TBandDir* out,
                                     hipStream_t s);
hipError_t launch_floor(float* T, int64_t n, float floor_T, hipStream_t s);

// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Carve {
    char* base;
    size_t used;
    size_t cap;
    template <class T>
    T* take(size_t count)
    {
        size_t off = (used + 255) & ~(size_t)255;
        used = off + count * sizeof(T);
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

// ---- launchers (kernels.hip) ----
hipError_t launch_map_reduce(const float* z, const uint8_t* mask, int64_t n, float* pmin, float* pmax,
                             unsigned long long* pcnt, unsigned long long* pbad, int nblocks, hipStream_t s);
hipError_t launch_map_finalize(const float* pmin, const float* pmax, const unsigned long long* pcnt,
                               const unsigned long long* pbad, int nblocks, double* range, unsigned long long* counts,
                               hipStream_t s);
hipError_t launch_map_apply(const float* z, const uint8_t* mask, int64_t n, const double* range, float* t,
                            hipStream_t s);
int map_reduce_blocks(int64_t n);

struct StatsGeom {
    int64_t H, W;
    int lb_h, lb_w, nbx, nby, nchunk, G;
    int64_t B() const { return (int64_t)nbx * nby; }
};
StatsGeom stats_geom(int64_t H, int64_t W, int lb_h, int lb_w);
// bonds: 1 = horizontal bonds only, 2 = vertical only, 3 = both
hipError_t launch_block_stats(const float* t, const uint8_t* mask, const StatsGeom& g, double two_pi_q, double J,
                              double* pS, int* pN, double* pTs, int* pNo, double* S, int* N, double* Ts, int* No,
                              hipStream_t s, int bonds = 3);
hipError_t launch_calibrate(const double* S, const int* N, int64_t B, double J, const double* cT, const double* ce,
                            int nc, float* T_out, double* e_out, int* nb_out, unsigned* n_have, hipStream_t s);
hipError_t launch_global_mean(const double* Ts, const int* No, int64_t B, float* gmean, hipStream_t s);
hipError_t launch_tpairs(const float* T, int64_t B, float J, float delta, TBand* tp, hipStream_t s);

struct InitArgs {
    float* state;
    float* state2;       // optional second buffer that receives the same start
    const float* t;
    const uint8_t* mask;
    const double* Ts;
    const int* No;
    const float* gmean;
    int64_t H, W;
    int lb_h, lb_w, nbx;
    int R;
    uint32_t real_offset, scene, key0, key1;
    int mode;
};
hipError_t launch_init(const InitArgs& a, hipStream_t s);

struct SweepFusedArgs {
    const float* src;    // [R][H][W] state after sweep k-1
    float* dst;          // [R][H][W] state after sweep k (sample cells must already hold their angles)
    const uint8_t* mask;
    const TBand* Tb;
    int H, W, lb_h, lb_w, nbx, ntx, nty, ntiles, Mw, R, rchunk, nchunks;
    int tile_h;          // 16 or 32 (tile width is 64)
    int64_t HW;
    uint32_t sweep, real_offset, scene, key0, key1;
    float q, J, delta_e;
    double two_pi_q, Jd;
    long long* e_partial;  // [R][ntiles] energy of each tile's colour-1 bonds (fixed point, 2^-32), or null
};
void fused_geometry(int64_t H, int64_t W, int R, int tile_h, int* ntx, int* nty, int* rchunk, int* nchunks);
hipError_t launch_sweep_fused(const SweepFusedArgs& a, hipStream_t s);
// Energies are accumulated in fixed point: each site's bond energy divided by J (at most 4 in magnitude) is
// rounded to a multiple of 2^-24 (an int32), and the integers are summed exactly (int64 beyond a thread), so the
// sums do not depend on their order.  kFixUnit converts back.
constexpr double kFixUnit = 1.0 / 16777216.0;
hipError_t launch_energy_full(const float* state, int64_t H, int64_t W, int R, float q, float J, long long* partial,
                              int nparts, hipStream_t s);
int energy_full_parts(int64_t H, int64_t W);
// partial layout [R][nparts] (fixed point); e_real[R] scratch; e_out = mean over r of sum_p partial[r][p] * unit *
// inv_norm, with inv_norm = 1 / (number of bonds): the energy per bond in units of J
hipError_t launch_energy_reduce(const long long* partial, int nparts, int R, double inv_norm, double* e_real,
                                double* e_out, hipStream_t s);
hipError_t launch_accumulate(const float* state, const uint8_t* mask, int64_t HW, int R, int first, double* acc,
                             hipStream_t s);
hipError_t launch_predict(const double* acc, const float* z, const uint8_t* mask, int64_t n, int64_t n_samples,
                          const double* range, float* zhat, hipStream_t s);
hipError_t launch_validate(const float* zhat, const float* truth, const uint8_t* ev, int64_t n, double* part,
                           int nblocks, double* out, hipStream_t s);
int validate_blocks(int64_t n);

// Realization-lane sweep (rl_sweep.hip): single-checkerboard order, state layout [H W][Rp] with the realization
// innermost (Rp = R rounded up to 64); a wave owns kRlBand columns x kRlSegRows rows of 64 realizations.
constexpr int kRlBand = 12;
constexpr int kRlSegRows = 96;         // longest row segment (rows are halved for small grids, down to 32)
constexpr int64_t kRlTargetWaves = 8192; // segments are shortened until a sweep has this many waves
constexpr int64_t kRlMinWaves = 2048;    // fewer waves than this: the fused tile sweep is used instead
constexpr int kRlWaves = 2;      // waves per SIMD the kernel is compiled for
struct RlGeom {
    int Rp, nbands, nseg, seg_rows;
    int64_t n_items;     // waves per sweep: nbands * nseg * Rp / 64
};
RlGeom rl_geometry(int64_t H, int64_t W, int R);
// the same with full-length row segments (kRlSegRows rows): the geometry of the batched form, whose scenes together
// fill the device
RlGeom rl_geometry_full(int64_t H, int64_t W, int R);
// how the lane sweep finds a column's temperature for temperature blocks tb_w wide: 1 aligned with the bands, 2 at
// most two temperature columns per window, 0 any (a division per column)
int rl_tm(int tb_w);
struct RlArgs {
    int H, W, R, Rp, Mw;
    int nbands, nseg, seg_rows;
    int64_t n_items;
    int tb_h, tb_w, nbx_t, nby_t;   // temperature layout (blocks, or 1 x 1 per site)
    uint32_t tb_w_inv;       // ceil(2^32 / tb_w) for tb_w > 1
    uint32_t sweep, real_offset, scene, key0, key1;
    float q, J, delta_e;
    double two_pi_q, Jd;
};
// cells: [(H + 4) * nbands] uint2 (gap bits, sample bits of each wave's window columns, rows -2 .. H + 1)
hipError_t launch_rl_cells(const uint8_t* mask, int64_t H, int64_t W, uint2* cells, hipStream_t s);
// [R][HW] -> [HW][Rp] into out (and out2 if not null); pad realizations get 0
hipError_t launch_rl_to_lanes(const float* in, int64_t HW, int R, float* out, float* out2, hipStream_t s);
// [HW][Rp] -> [R][HW]
hipError_t launch_rl_from_lanes(const float* in, int64_t HW, int R, float* out, hipStream_t s);
hipError_t launch_rl_accumulate(const float* S, const uint8_t* mask, int64_t HW, int R, int first, double* acc,
                                hipStream_t s);
// one sweep src -> dst; with epart set, the fixed-point energy of each wave's colour-1 sites goes to
// epart[r][seg * nbands + band] (layout [R][nbands * nseg])
// tbd != nullptr: directional coupling with the per-block table tbd (tb is then unused)
hipError_t launch_sweep_rl(const RlArgs& a, const uint2* cells, const TBand* tb, const TBandDir* tbd, const float* src,
                           float* dst, long long* epart, hipStream_t s);

// Sec. 2.2.2 double-checkerboard sweep (dc.hip): four in-place phases per sweep over all realizations.
struct DcArgs {
    float* state;        // [R][H][W], updated in place
    const uint8_t* mask;
    const TBand* tb;     // temperatures with the tb_h x tb_w layout (blocks, or 1 x 1 per site)
    int64_t H, W;
    int lb_h, lb_w;      // the blocks of the checkerboard
    int tb_h, tb_w, nbx_t;
    int Mw, R;
    uint32_t real_offset, scene, key0, key1;
    float q, J, delta_e;
    double two_pi_q, Jd;
};
hipError_t launch_dc_sweep(const DcArgs& a, uint32_t sweep, hipStream_t s);

// Sec. 2.2.3: site temperatures from the block map by n_s passes of the radius-r_s window mean (FP64 planes a, b).
hipError_t launch_sst(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t r_s,
                      int32_t n_s, double* a, double* b, float* out, hipStream_t s);

// ---- instruction-rate probe (rates.hip) ----
// Probes, in order: v_add_u32, v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32, v_bitop3_b32, v_sin_f32, v_cos_f32,
// v_exp_f32, v_cvt_f32_u32, v_xor_b32, and two pairs: v_mad_u64_u32 with an independent v_add_u32, and
// v_mad_u64_u32 feeding a v_bitop3_b32.  ns[i] = kernel time of probe i per wave-instruction of the probe, times the
// number of wave-instructions of the v_add_u32 probe (so that ns[i] / ns[0] is the issue cost relative to the add).
constexpr int kProbeCount = 12;
int probe_grid();
size_t probe_out_bytes();
double probe_wave_instructions();
hipError_t time_probes(uint32_t* out, hipStream_t s, double* ns);

// ---- temperature gradient (grad.hip) ----
hipError_t launch_block_energy(const float* state, const uint8_t* mask, const StatsGeom& g, double two_pi_q,
                               double J, int R, double* part, double* Hrb, hipStream_t s);
int grad_parts(int64_t HW);
hipError_t launch_temperature_grad(const float* state, const double* Hrb, const float* gz, const uint8_t* mask,
                                   int64_t HW, int R, int64_t B, const double* range, const float* T_blocks,
                                   double* part, double* g, double* dT, hipStream_t s);

struct RefArgs {
    float* state;          // [nT][L][L]
    const float* Tgrid;
    int L, Mw, colour;
    uint32_t sweep, key0, key1;
    float q, delta_e;
    double two_pi_q;
};
hipError_t launch_ref_fill(float* state, int64_t n, float v, hipStream_t s);
hipError_t launch_ref_half(const RefArgs& a, int nT, hipStream_t s);
hipError_t launch_ref_energy(const float* state, int L, int nT, float q, double* partial, int nparts,
                             hipStream_t s);
int ref_energy_parts(int L);
hipError_t launch_ref_accumulate(const double* partial, int nparts, int nT, double inv_norm, double* e_sum,
                                 int first, hipStream_t s);
hipError_t launch_ref_finish(const double* e_sum, int nT, double inv_meas, double* e_out, hipStream_t s);

}  // namespace mpr
