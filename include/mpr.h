/*
 * mpr.h — C ABI of the MI355X (gfx950) implementation of the SV-MPR gap-filling method:
 * conditional Monte Carlo simulation of the modified planar rotator (MPR) model with per-block temperatures
 * (Lach & Zukovic, arXiv 2212.01317, Sec. 2).
 *
 * The problem (Sec. 2.1): an H x W grid whose sites are either samples (G_S, value known) or gaps (G_P, value to
 * predict).  The data are mapped linearly onto spin angles, a temperature is calibrated per block of lb_h x lb_w
 * sites by energy matching (Sec. 2.2.2), the gap spins are relaxed by checkerboard Metropolis sweeps with the
 * samples held fixed until the energy series stops drifting (Sec. 3.4), and the prediction at each gap is the
 * mean of the conditional distribution, estimated over realizations and sampling sweeps (Sec. 2.1).
 *
 * Conventions (every entry point):
 *   - Pointers are DEVICE pointers owned by the caller unless marked "host".  Arrays are row-major and contiguous:
 *     site n = y * W + x.  mask: 1 = sample (observed), 0 = gap.  z at a gap is ignored (it may be NaN).
 *   - Spin angles are stored in turns t in [0, 1] (phi = 2 pi t).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is enqueued on it; a call returns
 *     without waiting unless its comment says it synchronises the stream.
 *   - Nothing is allocated on the device by the library: scratch memory is the caller's `workspace`, whose size is
 *     given by the matching *_workspace_bytes query.  The workspace must stay valid until the enqueued work ends.
 *   - The return value is an mpr_status; nothing throws across the ABI.  On any non-OK status mpr_last_error()
 *     returns a message (thread-local).  Argument checks happen before any work is enqueued.  A device error is
 *     reported as MPR_ERR_HIP by the call that observes it.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = (seed low 32 bits, seed high 32 bits) and
 *     counter = (pair, sweep, realization, scene << 4 | tag << 1 | colour), where the same-colour sites of a row are
 *     paired four columns apart (pair = y * ceil(W/4) + x/4; the site with ((x >> 1) & 1) == 0 takes words 0 and 1,
 *     the other words 2 and 3); a word w becomes the uniform (w >> 8) * 2^-24.  Tags: 0 sweep, 1 random start,
 *     2 reference lattice.  Realizations are keyed by their global index (real_offset + r), so any subset of the
 *     realizations reproduces the same chains.
 */
#ifndef MPR_H
#define MPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPR_OK = 0,
    MPR_ERR_INVALID_ARG = 1,        /* a pointer, size or parameter is invalid */
    MPR_ERR_SHAPE = 2,              /* grid or block shape out of the supported range */
    MPR_ERR_NO_SAMPLES = 3,         /* the mask has no observed site */
    MPR_ERR_NO_SAMPLE_BONDS = 4,    /* no pair of neighbouring samples anywhere: T cannot be estimated */
    MPR_ERR_NONFINITE_INPUT = 5,    /* an observed value is NaN or infinite */
    MPR_ERR_WORKSPACE_TOO_SMALL = 6,
    MPR_ERR_HIP = 7,                /* a HIP runtime call failed */
    MPR_WARN_NOT_CONVERGED = 8      /* AUTO stopping reached n_max without declaring equilibrium (results valid) */
} mpr_status;

enum { MPR_INIT_RANDOM = 0, MPR_INIT_BLOCK_MEAN = 1 };
enum { MPR_STOP_FIXED = 0, MPR_STOP_AUTO = 1, MPR_STOP_AUTO_CHAIN = 2 };
enum { MPR_T_BLOCK = 0, MPR_T_SITE = 1 };
enum { MPR_ORDER_SC = 0, MPR_ORDER_DC = 1 };
enum { MPR_SWEEP_AUTO = 0, MPR_SWEEP_TILES = 1, MPR_SWEEP_LANES = 2 };
enum { MPR_COUPLING_ISOTROPIC = 0, MPR_COUPLING_DIRECTIONAL = 1 };

/* Parameters of one conditional simulation (host struct). */
typedef struct {
    float q;              /* modification parameter of Eq. (1), 0 < q <= 1/2 */
    float J;              /* coupling of Eq. (1), J > 0 */
    int32_t n_real;       /* number of realizations R (independent chains), 1 .. 65535 */
    int32_t real_offset;  /* global index of realization 0 (for splitting the realizations over calls) */
    int32_t init_mode;    /* MPR_INIT_BLOCK_MEAN (SV-MPR, Sec. 3.3) or MPR_INIT_RANDOM (MPR) */
    int32_t stop_mode;    /* MPR_STOP_AUTO (Sec. 3.4 equilibrium test on the realization-averaged energy),
                             MPR_STOP_AUTO_CHAIN (the same test on every realization's own energy; the scene stops
                             once every chain has passed once), or MPR_STOP_FIXED (n_eq sweeps) */
    int32_t n_eq;         /* FIXED: number of equilibration sweeps */
    int32_t n_samp;       /* sampling sweeps S after equilibrium, each accumulated into the mean */
    int32_t n_fit;        /* AUTO: memory length of the energy series (paper default 20) */
    int32_t n_f;          /* AUTO: check every n_f sweeps (paper default 5); first check at n_fit + n_f */
    int32_t n_max;        /* AUTO: cap on the equilibration sweeps */
    uint64_t seed;
    uint32_t scene_id;    /* 0 .. 2^28 - 1, separates the random streams of different scenes */
    int32_t t_mode;       /* MPR_T_BLOCK (0): T_blocks has one temperature per lb_h x lb_w block (BST);
                             MPR_T_SITE (1): T_blocks has one temperature per site, [H*W] (SST, Sec. 2.2.3), while
                             lb_h x lb_w still give the blocks of the block-mean start.  Zero-initialised configs are
                             MPR_T_BLOCK. */
    int32_t order;        /* MPR_ORDER_SC (0): single checkerboard, all gap sites of colour 0 then of colour 1;
                             MPR_ORDER_DC (1): double checkerboard of Sec. 2.2.2 over the lb_h x lb_w blocks coloured
                             by (block row + block column) % 2: colour 0 then 1 in the even blocks, then in the odd
                             blocks (a different chain; mpr_simulate only). */
    int32_t sweep_kernel; /* which kernel mpr_simulate sweeps the single-checkerboard order with; every choice gives
                             the same chains bit for bit.  MPR_SWEEP_TILES (1): tiles of sites in LDS, lanes =
                             sites; MPR_SWEEP_LANES (2): state with the realization innermost, lanes = 64
                             realizations of one site (sides below 65536); MPR_SWEEP_AUTO (0, zero-initialised):
                             LANES when R >= 64 and the grid gives at least 2048 waves, else TILES.  mpr_sweep uses
                             TILES; the batched form uses LANES for every scene when R >= 64 (or LANES is asked
                             for) and its scenes share one temperature-lookup form, else TILES. */
    int32_t coupling;     /* MPR_COUPLING_ISOTROPIC (0, zero-initialised): one temperature per block.
                             MPR_COUPLING_DIRECTIONAL (1): the directional exchange interaction suggested in Sec. 4,
                             kept local to blocks: T_blocks[2*B] holds Tx of every block (its horizontal bonds) and
                             then Ty (its vertical bonds); an update is accepted iff
                             u2 < exp(J ah / Tx + J av / Ty), ah and av the sums of cos 2 pi q (t' - t_j) -
                             cos 2 pi q (t - t_j) over the left/right and up/down neighbours (couplings J and J Tx/Ty
                             at temperature Tx); temperatures below 1e-3 J are raised to fl32(1e-3 J).  Runs in the
                             single-checkerboard order with block temperatures on the realization-lane kernel (AUTO
                             selects it; TILES is refused); the energy series stays the unweighted Eq. (1) energy per
                             bond.  mpr_simulate only; sides below 65536 (MPR_ERR_SHAPE otherwise). */
} mpr_sim_config;

/* Sec. 2.1, first step: linear map of the samples onto spin angles.  zmin and zmax are taken over the samples;
 * t = fl32((z - zmin) / (zmax - zmin)) at samples (so the extremes map to exactly 0 and 1 turn), t = 0 at gaps and
 * everywhere when zmax == zmin.  Writes t_out[H*W] and range_out[2] = {zmin, zmax} (double).
 * Synchronises the stream (it must know whether there is a sample and whether all samples are finite).
 * Errors: MPR_ERR_NO_SAMPLES, MPR_ERR_NONFINITE_INPUT, MPR_ERR_SHAPE (H, W < 1).
 * Workspace: mpr_map_workspace_bytes. */
size_t mpr_map_workspace_bytes(int64_t H, int64_t W);
mpr_status mpr_map_angles(const float* z, const uint8_t* mask, int64_t H, int64_t W, float* t_out,
                          double* range_out, void* workspace, size_t ws_bytes, void* stream);

/* Eq. (2) per block (Sec. 2.2.2): for each T-block b of lb_h x lb_w sites (ceil division; blocks are numbered
 * row-major, nbx = ceil(W / lb_w)), S_out[b] = sum over bonds between two samples owned by b of -J cos(2 pi q dt),
 * where every site owns the bonds to its right and lower neighbour; N_out[b] = number of such bonds;
 * Tsum_out[b] / Nobs_out[b] = sum / count of the sample angles in b.  FP64 sums.  Any output may be NULL.
 * Asynchronous.  Workspace: mpr_block_stats_workspace_bytes. */
size_t mpr_block_stats_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w);
mpr_status mpr_block_stats(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w,
                           float q, float J, double* S_out, int32_t* N_out, double* Tsum_out, int32_t* Nobs_out,
                           void* workspace, size_t ws_bytes, void* stream);

/* Energy-matching curve (Sec. 2.1, a reading of the matching step): the equilibrium energy per bond of the
 * unconditional MPR model at J = 1 on a periodic L x L lattice, for each temperature T_grid[i] (device, float,
 * increasing).  Chain i starts from t = 1/2, runs n_therm sweeps, then averages the per-bond energy over n_meas
 * sweeps; the chains use the reference-lattice stream (tag 2, realization i, scene 0).  e_out[nT] (device, double).
 * L even, 2 .. 4096.  Asynchronous.  Workspace: mpr_reference_curve_workspace_bytes. */
size_t mpr_reference_curve_workspace_bytes(int32_t nT, int32_t L);
mpr_status mpr_reference_curve(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm,
                               int32_t n_meas, uint64_t seed, double* e_out, void* workspace, size_t ws_bytes,
                               void* stream);

/* Block-specific temperatures (Sec. 2.2.2): e_b = S_b / (J N_b) from mpr_block_stats, T_b = J g(e_b) where g
 * inverts the matching curve (curve_T[n_curve] increasing, curve_e[n_curve]; device, double): the curve is made
 * non-decreasing by a running maximum, g is piecewise linear in (e, log T) between points, linear in T between
 * (e = -1, T = 0) and the first point, 0 for e <= -1 and curve_T[n_curve - 1] beyond the last point.  A block
 * without sample bonds gets the median of the other blocks' T (even count: mean of the two middle values).
 * lb_h >= H and lb_w >= W gives the single global temperature of the plain MPR method.  T_out[B] (float);
 * e_blocks_out[B] and nbonds_out[B] are optional (NULL).  Synchronises the stream (to report
 * MPR_ERR_NO_SAMPLE_BONDS).  Workspace: mpr_calibrate_workspace_bytes. */
size_t mpr_calibrate_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w);
mpr_status mpr_calibrate_temperature(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h,
                                     int32_t lb_w, float q, float J, const double* curve_T, const double* curve_e,
                                     int32_t n_curve, float* T_out, double* e_blocks_out, int32_t* nbonds_out,
                                     void* workspace, size_t ws_bytes, void* stream);

/* Size in bytes of the static device scratch of the entry points that allocate nothing (one copy per device). */
#define MPR_NOALLOC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid hipMalloc): the
 * calibration of mpr_calibrate_temperature, with the same arguments, results and errors, but no workspace argument:
 * its scratch is a static device array of MPR_NOALLOC_SCRATCH_BYTES (16 MiB) per device, which the library holds on
 * every device it runs on until the process ends.  Grids and block sizes whose mpr_calibrate_workspace_bytes exceed
 * that size return MPR_ERR_WORKSPACE_TOO_SMALL before any device work (4096 x 4096 with 32 x 32 blocks needs
 * 0.56 MiB, 16384 x 16384 with 32 x 32 blocks 9 MiB).  Allocates nothing and calls no allocating routine.  The
 * pointers and the stream belong to the current device, whose array is used (its address is looked up on the first
 * call on that device).  Every call on a device shares that device's array, which keeps the last call's contents
 * (nothing in it has to start at zero: the calibration writes every entry before reading it); calls that overlap on
 * one device (other streams or host threads) race.  Synchronises the stream, like mpr_calibrate_temperature. */
mpr_status mpr_calibrate_temperature_noalloc(const float* t, const uint8_t* mask, int64_t H, int64_t W,
                                             int32_t lb_h, int32_t lb_w, float q, float J, const double* curve_T,
                                             const double* curve_e, int32_t n_curve, float* T_out,
                                             double* e_blocks_out, int32_t* nbonds_out, void* stream);

/* Directional-coupling extension (Sec. 4 suggests an exchange interaction that depends on the direction, with the
 * parameters kept local to blocks): per block, Tx by the energy matching of mpr_calibrate_temperature applied to its
 * horizontal sample bonds only (a sample and its right neighbour) and Ty to its vertical ones (a sample and its
 * lower neighbour), each with its own median fill, then both raised to at least fl32(1e-3 J).  The same matching
 * curve is used for both directions (exact when Tx = Ty).  Tx_out[B], Ty_out[B] (float).  Synchronises the stream;
 * MPR_ERR_NO_SAMPLE_BONDS when a direction has no sample bond at all.  Workspace: mpr_calibrate_workspace_bytes. */
mpr_status mpr_calibrate_directional(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h,
                                     int32_t lb_w, float q, float J, const double* curve_T, const double* curve_e,
                                     int32_t n_curve, float* Tx_out, float* Ty_out, void* workspace, size_t ws_bytes,
                                     void* stream);

/* Conditional simulation (Sec. 2.1, Sec. 2.2.2, Sec. 3.3, Sec. 3.4).
 *   t[H*W]: mapped angles (samples used); T_blocks[B]: block temperatures (float) with the same lb_h x lb_w layout,
 *   or, with cfg->t_mode == MPR_T_SITE, T_blocks[H*W]: one temperature per site (the sweeps use T of the site).
 *   Start: gaps take the block mean of the sample angles (a block without samples: the global sample mean), or a
 *   uniform draw (tag 1).  Then sweeps k = 1, 2, ...: all gap sites of colour (x + y) % 2 == 0, then of colour 1,
 *   each an independent-uniform Metropolis proposal t' = u1 accepted iff u2 < exp(-dE / T_b) (T_b = 0, and any
 *   T_b that is not > 0, NaN included: iff dE <= 0), dE from Eq. (1) over the in-grid nearest neighbours (open
 *   boundaries).  After each sweep the
 *   realization-averaged whole-grid energy per bond e(k) is recorded (e(0) before the first sweep).
 *   FIXED: k* = n_eq.  AUTO: at k = n_fit + j n_f the ordinary least-squares slope beta of the last n_fit energies
 *   is taken; equilibrium when beta * sign(e(k) - e(0)) <= 0; the cap n_max gives MPR_WARN_NOT_CONVERGED.
 *   AUTO_CHAIN (a reading of Sec. 3.3 / 3.4 in which the energy series is that of one simulation): the same test on
 *   each realization's own series e_r(k) at the same check points; a chain that passes stays passed, and k* is the
 *   first check at which every chain has passed.
 *   Then n_samp sampling sweeps (k* + 1 ...), after each of which every realization's gap angles are added to
 *   acc_out in realization order (FP64; samples' entries are 0).
 * The workspace holds a second state buffer of n_real*H*W floats (the sweep reads one buffer and writes the other).
 * Outputs: state[n_real*H*W] (float; in: ignored, out: final states), acc_out[H*W] (double), energy_out[k* + 1]
 * (double, optional NULL; size n_max + 1 for AUTO, n_eq + 1 for FIXED), *sweeps_done_out = k* (host, optional).
 * FIXED mode is asynchronous; AUTO and AUTO_CHAIN synchronise the stream at every check.  Workspace:
 * mpr_simulate_workspace_bytes.  Calls with the same arguments give bit-identical results. */
size_t mpr_simulate_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg);
mpr_status mpr_simulate(const float* t, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks,
                        int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, float* state, double* acc_out,
                        double* energy_out, int32_t* sweeps_done_out, void* workspace, size_t ws_bytes,
                        void* stream);

/* Sec. 2.2.3 (SST, site-specific temperatures): from the block temperatures T_blocks[ceil(H/lb_h)*ceil(W/lb_w)]
 * (every site starts with its block's value), n_s successive passes replace the temperature of every site by the
 * mean over the (2 r_s + 1) x (2 r_s + 1) square of sites around it, cut at the grid edges (mean over the in-grid
 * sites; the paper leaves the shape of the area and r_s open).  FP64, each window summed row by row from the top
 * left, one rounding to FP32: T_site_out[H*W] (float).  0 <= r_s <= 64, 0 <= n_s <= 1000.  Asynchronous.
 * Workspace: mpr_sst_temperatures_workspace_bytes (two FP64 planes). */
size_t mpr_sst_temperatures_workspace_bytes(int64_t H, int64_t W);
mpr_status mpr_sst_temperatures(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t r_s,
                                int32_t n_s, float* T_site_out, void* workspace, size_t ws_bytes, void* stream);

/* Continuation of chains: sweeps k_first .. k_first + n_sweeps - 1 (the sweep counter keys the random stream) with
 * exactly the per-sweep arithmetic of mpr_simulate (no start, no stopping rule, no accumulation).  The sweeps
 * alternate between two buffers [n_real*H*W]: sweep k_first reads `state` and writes `state_alt`, the next one reads
 * `state_alt` and writes `state`, and so on, so the result is in `state` when n_sweeps is even and in `state_alt`
 * when it is odd.  Both buffers must hold the same sample angles (e.g. state_alt a copy of state); only gap cells
 * are written.  Uses cfg->q, J, n_real, real_offset, seed, scene_id, t_mode.  Resuming a saved state with the next sweep
 * counter reproduces an uninterrupted run bit for bit.  energy_out[n_sweeps] (optional): the realization-averaged
 * energy per bond after each sweep.  Asynchronous.  Workspace: mpr_sweep_workspace_bytes. */
size_t mpr_sweep_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg);
mpr_status mpr_sweep(float* state, float* state_alt, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks,
                     int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, int32_t k_first, int32_t n_sweeps,
                     double* energy_out, void* workspace, size_t ws_bytes, void* stream);

/* Prediction (Sec. 2.1, last step): at gaps zhat = fl32(zmin + (zmax - zmin) * acc / n_samples) with
 * range = {zmin, zmax} from mpr_map_angles; at samples zhat = z.  Asynchronous. */
mpr_status mpr_predict(const double* acc, const float* z, const uint8_t* mask, int64_t H, int64_t W,
                       int64_t n_samples, const double* range, float* zhat_out, void* stream);

/* Eq. (3) and Eq. (4): out[0] = AAE = mean |truth - zhat|, out[1] = RASE = sqrt(mean (truth - zhat)^2) over the
 * n sites with eval_mask != 0 (0 when there is none).  FP64, device out[2].  Asynchronous.
 * Workspace: mpr_validate_workspace_bytes. */
size_t mpr_validate_workspace_bytes(int64_t n);
mpr_status mpr_validate(const float* zhat, const float* truth, const uint8_t* eval_mask, int64_t n, double* out,
                        void* workspace, size_t ws_bytes, void* stream);

/* Batched simulation (a project addition): many scenes of different sizes and gap fractions, each with n_real
 * realizations.  Each scene follows exactly the arithmetic of mpr_simulate with cfg->scene_id replaced by its own
 * scene_id (its own stopping test and sampling sweeps), so its results are bit-identical to a single-scene call.
 * All scenes are advanced together by one persistent sweep kernel per sweep that takes work items from device work
 * queues, largest scenes first: with n_real >= 64 (cfg->sweep_kernel AUTO or LANES; or any n_real with LANES), the
 * realization-lane sweep over (scene, realization group, band, row segment) items from eight queues, one per XCD,
 * provided every scene's sides are below 65536 and all scenes share one temperature-lookup form (their lb_w all
 * multiples of the 12-column band, all at least 15 wide, or all otherwise); else (or with TILES) the tile sweep over
 * (scene, tile, realization chunk) items.  The sweeps, energies, stopping tests and sampling are replayed from a HIP
 * graph captured once per call (n_f sweeps per graph); the stream is synchronised once per graph replay.  On the
 * lane sweep the scenes' starts are spread over the caller's stream and three private streams of the library
 * (created once per host thread and device, default priority), forked from the caller's stream and joined back into
 * it by events, so that the call still begins after and ends before the caller's other work on `stream`.  The
 * per-chain stopping test (MPR_STOP_AUTO_CHAIN) is refused (MPR_ERR_INVALID_ARG).  tile_h: 16 or 32 (tile height of
 * the tile sweep; results do not depend on it), or 0 to time one sweep with each and keep the faster
 * (*tile_h_used_out reports the choice, 0 when the lane sweep ran).
 * sweeps_done_out[n_scenes] (host, optional): k* per scene; converged_out[n_scenes] (host, optional): 1 where the scene
 * met the equilibrium test (or ran FIXED), 0 where AUTO reached n_max without it (the call then returns
 * MPR_WARN_NOT_CONVERGED).  Workspace: mpr_simulate_batched_workspace_bytes (lane sweep: two lane buffers per
 * scene plus small per-scene arrays; tile sweep: a second state buffer per scene plus small per-scene arrays). */
typedef struct {
    int64_t H, W;             /* grid of this scene */
    int32_t lb_h, lb_w;       /* its temperature blocks */
    uint32_t scene_id;        /* its random stream, 0 .. 2^28 - 1 */
    const float* t;           /* [H*W] mapped angles (samples used) */
    const uint8_t* mask;      /* [H*W] 1 = sample */
    const float* T_blocks;    /* [ceil(H/lb_h) * ceil(W/lb_w)] */
    float* state;             /* [n_real*H*W] out: final states */
    double* acc;              /* [H*W] out: accumulated gap angles */
    double* energy;           /* [cap + 1] out, optional (NULL) */
} mpr_scene;
size_t mpr_simulate_batched_workspace_bytes(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg);
mpr_status mpr_simulate_batched(const mpr_scene* scenes /* host array */, int32_t n_scenes,
                                const mpr_sim_config* cfg, int32_t tile_h, int32_t* sweeps_done_out,
                                int32_t* converged_out, int32_t* tile_h_used_out, void* workspace, size_t ws_bytes,
                                void* stream);

/* Temperature gradient (a project addition on Sec. 2.2.2: tuning the block temperatures by gradient).
 * For a density proportional to exp(-sum_b H_b / T_b), d<f>/dT_b = Cov(f, H_b) / T_b^2.
 *
 * mpr_block_energy: H_out[r * B + b] (double) = H_b of realization r of `state` [n_real*H*W]: the sum of Eq. (1) over
 * every bond with at least one gap end, counted in the block of its gap end; a bond between two gaps of different
 * blocks counts one half in each; bonds between samples are left out.  FP64 (published formula).  Asynchronous.
 * Workspace: mpr_block_energy_workspace_bytes. */
size_t mpr_block_energy_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t n_real);
mpr_status mpr_block_energy(const float* state, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w,
                            float q, float J, int32_t n_real, double* H_out, void* workspace, size_t ws_bytes,
                            void* stream);

/* mpr_temperature_grad: score-function estimate of dL/dT_b for a loss L of the prediction of a run with one sampling
 * sweep (E[zhat] = zmin + (zmax - zmin) E[t]).  state [n_real*H*W]: the final states of that run; H_blocks
 * [n_real*n_blocks] from mpr_block_energy; grad_zhat [H*W] (float) = dL/dzhat; range = {zmin, zmax} (device).
 * g_r = sum over gaps of grad_zhat * (zmax - zmin) * t_r; dT_out[b] (double) = Cov_r(g, H_b) / T_b^2 with the
 * unbiased (R - 1) covariance, 0 where T_b = 0.  n_real >= 2.  FP64, fixed reduction order.  Asynchronous.
 * Workspace: mpr_temperature_grad_workspace_bytes. */
size_t mpr_temperature_grad_workspace_bytes(int64_t H, int64_t W, int32_t n_real);
mpr_status mpr_temperature_grad(const float* state, const double* H_blocks, const float* grad_zhat,
                                const uint8_t* mask, int64_t H, int64_t W, int32_t n_real, int64_t n_blocks,
                                const double* range, const float* T_blocks, double* dT_out, void* workspace,
                                size_t ws_bytes, void* stream);

/* mpr_probe_instruction_rates: measurement support for the ALU roofline of the sweep (the per-update cost is priced
 * from the device's own instruction rates, not from a data sheet).  Times twelve probe kernels, each a fixed number of
 * wave-instructions in independent dependency chains over the whole device, and writes to cost_out (host,
 * n_out >= 12) the issue cost per wave-instruction of each relative to v_add_u32 = 1 (2 = half rate):
 * [0] v_add_u32, [1] v_mad_u64_u32, [2] v_mul_lo_u32, [3] v_mul_hi_u32, [4] v_bitop3_b32, [5] v_sin_f32,
 * [6] v_cos_f32, [7] v_exp_f32, [8] v_cvt_f32_u32, [9] v_xor_b32, and two pairs, each cost per instruction of the
 * pair: [10] v_mad_u64_u32 beside an independent v_add_u32 (0.5 would mean the two issue together), [11]
 * v_mad_u64_u32 whose high half a v_bitop3_b32 consumes (the shape of a Philox round).  add_ns_out (host, nullable):
 * device time per wave-instruction of v_add_u32, in ns.  workspace: device,
 * mpr_probe_instruction_rates_workspace_bytes() bytes (probe outputs).  Synchronises the stream. */
size_t mpr_probe_instruction_rates_workspace_bytes(void);
mpr_status mpr_probe_instruction_rates(double* cost_out, int32_t n_out, double* add_ns_out, void* workspace,
                                       size_t ws_bytes, void* stream);

/* ---- The 3D lattice (the extension to three dimensions that Sec. 4 names) ----
 * A D x H x W grid, site n = (z H + y) W + x; the Hamiltonian of Eq. (1) over the six nearest neighbours of the simple
 * cubic lattice (open boundaries); checkerboard colour (x + y + z) % 2; T-blocks of lb_d x lb_h x lb_w sites (ceil
 * division, numbered (bz nby + by) nbx + bx).  The random stream of a site is the plane's with the row index z H + y
 * in place of y.  Sides 1 .. 65535 with (D H) ceil(W / 4) < 2^32 (MPR_ERR_SHAPE otherwise); blocks >= 1 on every side.
 *
 * mpr_calibrate_temperature3d: Eq. (2) per 3D block (every site owns the bonds to its +x, +y and +z neighbour; a bond
 * between two samples counts for the block of its owner), then the energy matching and the median fill of
 * mpr_calibrate_temperature with a matching curve of the cubic lattice (mpr_reference_curve3d).  t[D*H*W], mask
 * [D*H*W] (device); curve_T / curve_e[n_curve] (device, double); T_out[B] (device, float); e_blocks_out[B] (double)
 * and nbonds_out[B] (int32) optional (NULL).  MPR_ERR_NO_SAMPLE_BONDS when no two samples are neighbours.
 * Synchronises the stream.  Workspace: mpr_calibrate3d_workspace_bytes. */
size_t mpr_calibrate3d_workspace_bytes(int64_t D, int64_t H, int64_t W, int32_t lb_d, int32_t lb_h, int32_t lb_w);
mpr_status mpr_calibrate_temperature3d(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W,
                                       int32_t lb_d, int32_t lb_h, int32_t lb_w, float q, float J,
                                       const double* curve_T, const double* curve_e, int32_t n_curve, float* T_out,
                                       double* e_blocks_out, int32_t* nbonds_out, void* workspace, size_t ws_bytes,
                                       void* stream);

/* mpr_reference_curve3d: the matching curve of the cubic lattice (the 3D counterpart of mpr_reference_curve): the
 * equilibrium energy per bond of the unconditional model at J = 1 on a periodic L x L x L lattice (3 L^3 bonds), for
 * each temperature T_grid[i] (device, float).  Chain i starts from t = 1/2, runs n_therm sweeps (colour 0, then 1),
 * then averages over n_meas sweeps; the chains use the reference-lattice stream (tag 2, realization i, scene 0) with
 * the row index z L + y.  e_out[nT] (device, double).  L even, 2 .. 512; nT 1 .. 65535.  Asynchronous.  Workspace:
 * mpr_reference_curve3d_workspace_bytes (the nT L^3 chain states and the energy partial sums). */
size_t mpr_reference_curve3d_workspace_bytes(int32_t nT, int32_t L);
mpr_status mpr_reference_curve3d(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm, int32_t n_meas,
                                 uint64_t seed, double* e_out, void* workspace, size_t ws_bytes, void* stream);

/* mpr_simulate3d: the conditional simulation of mpr_simulate on the 3D grid, with block temperatures and the single
 * checkerboard only (cfg->t_mode MPR_T_BLOCK, cfg->order MPR_ORDER_SC, cfg->coupling MPR_COUPLING_ISOTROPIC;
 * MPR_ERR_INVALID_ARG otherwise).  Start (block mean of the 3D block's samples, the global sample mean for a block
 * without samples, or a uniform draw, tag 1), the sweeps k = 1, 2, ... (colour 0 then colour 1, a gap site's update
 * over its in-grid neighbours among the six), the energy per bond e(k) over all (D-1)HW + D(H-1)W + DH(W-1) bonds,
 * the FIXED and AUTO stopping rules, the n_samp sampling sweeps and the accumulator are those of mpr_simulate.
 * t[D*H*W], mask[D*H*W], T_blocks[B] (device, float).  Outputs: state[n_real*D*H*W] (device, float; in: ignored,
 * out: final states), acc_out[D*H*W] (device, double), energy_out[k* + 1] (device, double, optional NULL; size
 * n_max + 1 for AUTO, n_eq + 1 for FIXED), *sweeps_done_out = k* (host, optional).  The chains run in place in a
 * realization-lane copy of the state held in the workspace (n_real rounded up to 64, times D H W floats).  FIXED is
 * asynchronous; AUTO synchronises the stream at every check; MPR_WARN_NOT_CONVERGED when n_max is reached.
 * Workspace: mpr_simulate3d_workspace_bytes.  Calls with the same arguments give bit-identical results. */
size_t mpr_simulate3d_workspace_bytes(int64_t D, int64_t H, int64_t W, int32_t lb_d, int32_t lb_h, int32_t lb_w,
                                      const mpr_sim_config* cfg);
mpr_status mpr_simulate3d(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W, const float* T_blocks,
                          int32_t lb_d, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, float* state,
                          double* acc_out, double* energy_out, int32_t* sweeps_done_out, void* workspace,
                          size_t ws_bytes, void* stream);

/* Message for the last non-OK status on the calling thread ("" if none). */
const char* mpr_last_error(void);

/* Version of this ABI (major * 10000 + minor * 100 + patch). */
int32_t mpr_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPR_H */
