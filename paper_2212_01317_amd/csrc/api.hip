// Host implementation of the C ABI declared in include/mpr.h: argument checks, workspace carving, kernel
// sequencing on the caller's stream, and the equilibrium test of Sec. 3.4.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "batched.hpp"
#include "mpr.h"
#include "lattice3d.hpp"
#include "mpr_internal.hpp"
#include "rl_start.hpp"

using mpr::Carve;

namespace {

thread_local std::string g_last_error;

mpr_status fail(mpr_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

mpr_status ok()
{
    g_last_error.clear();
    return MPR_OK;
}

#define MPR_HIP(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(MPR_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Scratch memory of the entry points that allocate nothing (mpr_calibrate_temperature_noalloc): a file-scope device
// array, one copy per device, held until the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address is taken once per device with hipGetSymbolAddress (with that device current)
// and only that address is passed to kernels.
__device__ __align__(256) unsigned char scratch[MPR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (looked up on the first call on that device).
mpr_status scratch_for_current_device(void** out)
{
    int dev = -1;
    MPR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MPR_ERR_INVALID_ARG, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MPR_ERR_HIP, "hipGetSymbolAddress returned a NULL address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MPR_OK;
}

mpr_status check_grid(int64_t H, int64_t W)
{
    if (H < 1 || W < 1) return fail(MPR_ERR_SHAPE, "grid %lld x %lld: both sides must be >= 1", (long long)H, (long long)W);
    if (H > (1 << 20) || W > (1 << 20) || H * W > ((int64_t)1 << 31) - 1)
        return fail(MPR_ERR_SHAPE, "grid %lld x %lld exceeds 2^31 - 1 sites or 2^20 per side", (long long)H,
                    (long long)W);
    return MPR_OK;
}

mpr_status check_blocks(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w)
{
    if (lb_h < 1 || lb_w < 1) return fail(MPR_ERR_SHAPE, "T-block %d x %d: both sides must be >= 1", lb_h, lb_w);
    const int64_t B = ((H + lb_h - 1) / lb_h) * ((W + lb_w - 1) / lb_w);
    if (B > ((int64_t)1 << 26)) return fail(MPR_ERR_SHAPE, "too many T-blocks (%lld)", (long long)B);
    return MPR_OK;
}

int64_t nblocks_of(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w)
{
    return ((H + lb_h - 1) / lb_h) * ((W + lb_w - 1) / lb_w);
}

// Temperatures the sweeps read: one per lb_h x lb_w block, or one per site (the 1 x 1 block layout).
int64_t t_count(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg)
{
    return cfg && cfg->t_mode == MPR_T_SITE ? H * W : ((H + lb_h - 1) / lb_h) * ((W + lb_w - 1) / lb_w);
}
int32_t t_lb(int32_t lb, const mpr_sim_config& c) { return c.t_mode == MPR_T_SITE ? 1 : lb; }

// mpr_simulate runs the realization-lane sweep (state with the realization innermost, one realization per lane)
// when the realizations fill the lanes of a wave (R >= 64) and the grid gives enough waves to fill the device,
// in the single-checkerboard order, with sides below 2^16 (the temperature-column reciprocal is exact there).
bool use_rl(int64_t H, int64_t W, const mpr_sim_config* cfg)
{
    if (!cfg || cfg->order != MPR_ORDER_SC || H >= 65536 || W >= 65536) return false;
    if (cfg->sweep_kernel == MPR_SWEEP_LANES || cfg->coupling == MPR_COUPLING_DIRECTIONAL) return true;
    if (cfg->sweep_kernel == MPR_SWEEP_TILES || cfg->n_real < 64) return false;
    return mpr::rl_geometry(H, W, cfg->n_real).n_items >= mpr::kRlMinWaves;
}

// ---- workspace layouts (the same code computes the size and carves the pointers) ----
struct MapWs {
    float *pmin, *pmax;
    unsigned long long *pcnt, *pbad, *counts;
    int nb;
};
size_t map_ws(Carve& c, int64_t n, MapWs* w)
{
    MapWs x;
    x.nb = mpr::map_reduce_blocks(n);
    x.pmin = c.take<float>(x.nb);
    x.pmax = c.take<float>(x.nb);
    x.pcnt = c.take<unsigned long long>(x.nb);
    x.pbad = c.take<unsigned long long>(x.nb);
    x.counts = c.take<unsigned long long>(2);
    if (w) *w = x;
    return c.used;
}

struct StatsWs {
    double *pS, *pTs;
    int *pN, *pNo;
};
size_t stats_ws(Carve& c, const mpr::StatsGeom& g, StatsWs* w)
{
    const int64_t np = g.B() * g.nchunk;
    StatsWs x;
    x.pS = c.take<double>(np);
    x.pTs = c.take<double>(np);
    x.pN = c.take<int>(np);
    x.pNo = c.take<int>(np);
    if (w) *w = x;
    return c.used;
}

struct CalWs {
    StatsWs st;
    double* S;
    int* N;
    unsigned* n_have;
};
size_t cal_ws(Carve& c, const mpr::StatsGeom& g, CalWs* w)
{
    CalWs x;
    stats_ws(c, g, &x.st);
    x.S = c.take<double>(g.B());
    x.N = c.take<int>(g.B());
    x.n_have = c.take<unsigned>(1);
    if (w) *w = x;
    return c.used;
}

int fused_tiles(int64_t H, int64_t W, int R);

bool auto_stop(int32_t stop_mode) { return stop_mode == MPR_STOP_AUTO || stop_mode == MPR_STOP_AUTO_CHAIN; }

struct SimWs {
    StatsWs st;
    double* Ts;
    int* No;
    float* gmean;
    mpr::TBand* tp;
    long long* epart;   // [R][max(ntiles, nfull)]
    double* e_real;     // [R]
    double* series;     // [cap + 1]
    double* hist;       // per-chain stop: every realization's energy after each sweep, [cap + 1][R]
    float* alt;         // [R][H][W] second state buffer (fused sweep)
    mpr::TBandDir* tpd; // directional coupling: per-block table
    float* rl[2];       // [HW][Rp] state buffers of the realization-lane sweep
    uint2* cells;       // its per-row window bits
};
size_t sim_ws(Carve& c, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, SimWs* w)
{
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    SimWs x;
    stats_ws(c, g, &x.st);
    x.Ts = c.take<double>(g.B());
    x.No = c.take<int>(g.B());
    x.gmean = c.take<float>(1);
    x.tp = c.take<mpr::TBand>(t_count(H, W, lb_h, lb_w, cfg));
    const int64_t R = cfg->n_real > 0 ? cfg->n_real : 1;
    const int nt = fused_tiles(H, W, (int)R);
    const int nfull = mpr::energy_full_parts(H, W);
    const bool rl = use_rl(H, W, cfg);
    const mpr::RlGeom rg = mpr::rl_geometry(H, W, (int)R);
    int64_t np = nt > nfull ? nt : nfull;
    if (rl && (int64_t)rg.nbands * rg.nseg > np) np = (int64_t)rg.nbands * rg.nseg;
    x.epart = c.take<long long>(np * R);
    x.e_real = c.take<double>(R);
    const int64_t cap = auto_stop(cfg->stop_mode) ? cfg->n_max : cfg->n_eq;
    x.series = c.take<double>((cap > 0 ? cap : 0) + 1);
    x.hist = cfg->stop_mode == MPR_STOP_AUTO_CHAIN ? c.take<double>(((cap > 0 ? cap : 0) + 1) * R) : nullptr;
    x.alt = rl ? nullptr : c.take<float>(R * H * W);
    x.tpd = cfg->coupling == MPR_COUPLING_DIRECTIONAL ? c.take<mpr::TBandDir>(nblocks_of(H, W, lb_h, lb_w)) : nullptr;
    x.rl[0] = rl ? c.take<float>(H * W * rg.Rp) : nullptr;
    x.rl[1] = rl ? c.take<float>(H * W * rg.Rp) : nullptr;
    x.cells = rl ? c.take<uint2>((H + 4) * rg.nbands) : nullptr;
    if (w) *w = x;
    return c.used;
}

struct RefWs {
    float* state;
    double* part;
    double* esum;
    int nparts;
};
size_t ref_ws(Carve& c, int32_t nT, int32_t L, RefWs* w)
{
    RefWs x;
    x.state = c.take<float>((int64_t)nT * L * L);
    x.nparts = mpr::ref_energy_parts(L);
    x.part = c.take<double>((int64_t)x.nparts * nT);
    x.esum = c.take<double>(nT);
    if (w) *w = x;
    return c.used;
}

mpr_status check_ws(void* ws, size_t have, size_t need)
{
    if (need > 0 && ws == nullptr) return fail(MPR_ERR_INVALID_ARG, "workspace is NULL (%zu bytes needed)", need);
    if (have < need) return fail(MPR_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, %zu needed", have, need);
    return MPR_OK;
}

// Equilibrium test (Sec. 3.4, reading): ordinary least-squares slope of the last n_fit energies against the
// sweep index; equilibrium once the slope no longer points away from the starting energy.
double ols_slope(const double* y, int n)
{
    double xm = 0.0, ym = 0.0;
    for (int j = 0; j < n; ++j) {
        xm += (double)j;
        ym += y[j];
    }
    xm /= (double)n;
    ym /= (double)n;
    double sxy = 0.0, sxx = 0.0;
    for (int j = 0; j < n; ++j) {
        sxy += ((double)j - xm) * (y[j] - ym);
        sxx += ((double)j - xm) * ((double)j - xm);
    }
    return sxx > 0.0 ? sxy / sxx : 0.0;
}

bool equilibrium_reached(double e0, const double* window, int n_fit)
{
    const double beta = ols_slope(window, n_fit);
    const double d = window[n_fit - 1] - e0;
    const double sigma0 = (double)((d > 0.0) - (d < 0.0));
    return beta * sigma0 <= 0.0;
}

// The per-chain form of the test: every realization applies it to its own energy series, a realization that has
// passed stays passed, and the scene is in equilibrium once all have passed.  The host keeps e_r(0) and the latch;
// at a check the last n_fit rows of the [k][R] history come over (hist = the device history).
struct ChainStop {
    int R = 0, n_fit = 0;
    std::vector<double> e0, win, y;
    std::vector<uint8_t> passed;
    hipError_t start(const double* hist, int R_, int n_fit_, hipStream_t s)
    {
        R = R_;
        n_fit = n_fit_;
        e0.resize((size_t)R);
        win.resize((size_t)R * n_fit);
        y.resize((size_t)n_fit);
        passed.assign((size_t)R, 0);
        return hipMemcpyAsync(e0.data(), hist, sizeof(double) * (size_t)R, hipMemcpyDeviceToHost, s);
    }
    // the check at sweep k (synchronises the stream)
    hipError_t check(const double* hist, int k, hipStream_t s, bool* all)
    {
        hipError_t e = hipMemcpyAsync(win.data(), hist + (int64_t)(k - n_fit + 1) * R, sizeof(double) * win.size(),
                                      hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        bool a = true;
        for (int r = 0; r < R; ++r) {
            if (!passed[(size_t)r]) {
                for (int j = 0; j < n_fit; ++j) y[(size_t)j] = win[(size_t)j * R + r];
                if (equilibrium_reached(e0[(size_t)r], y.data(), n_fit)) passed[(size_t)r] = 1;
            }
            a = a && passed[(size_t)r];
        }
        *all = a;
        return hipSuccess;
    }
};

mpr_status check_sim_config(const mpr_sim_config& c)
{
    if (!(c.q > 0.0f && c.q <= 0.5f) || !(c.J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    if (c.n_real < 1 || c.n_real > 65535) return fail(MPR_ERR_INVALID_ARG, "n_real must be in 1 .. 65535");
    if (c.real_offset < 0) return fail(MPR_ERR_INVALID_ARG, "real_offset must be >= 0");
    if (c.scene_id >= (1u << 28)) return fail(MPR_ERR_INVALID_ARG, "scene_id must be < 2^28");
    if (c.t_mode != MPR_T_BLOCK && c.t_mode != MPR_T_SITE) return fail(MPR_ERR_INVALID_ARG, "unknown t_mode %d", c.t_mode);
    if (c.order != MPR_ORDER_SC && c.order != MPR_ORDER_DC) return fail(MPR_ERR_INVALID_ARG, "unknown order %d", c.order);
    if (c.sweep_kernel < MPR_SWEEP_AUTO || c.sweep_kernel > MPR_SWEEP_LANES)
        return fail(MPR_ERR_INVALID_ARG, "unknown sweep_kernel %d", c.sweep_kernel);
    if (c.sweep_kernel == MPR_SWEEP_LANES && c.order != MPR_ORDER_SC)
        return fail(MPR_ERR_INVALID_ARG, "the realization-lane sweep runs the single-checkerboard order");
    if (c.coupling != MPR_COUPLING_ISOTROPIC && c.coupling != MPR_COUPLING_DIRECTIONAL)
        return fail(MPR_ERR_INVALID_ARG, "unknown coupling %d", c.coupling);
    if (c.coupling == MPR_COUPLING_DIRECTIONAL &&
        (c.order != MPR_ORDER_SC || c.t_mode != MPR_T_BLOCK || c.sweep_kernel == MPR_SWEEP_TILES))
        return fail(MPR_ERR_INVALID_ARG,
                    "directional coupling runs the single-checkerboard order with block temperatures on the "
                    "realization-lane sweep");
    return MPR_OK;
}


// Runs fused sweeps (one launch per sweep) alternating between two state buffers.
struct SweepRunner {
    mpr::SweepFusedArgs a;
    float* buf[2];
    int cur;
    double inv_norm;
    long long* epart;  // [R][ntiles]
    double* e_real;    // [R]
    hipStream_t s;

    SweepRunner(float* state, float* alt, const uint8_t* mask, int64_t H, int64_t W, const mpr::TBand* tp,
                int32_t lb_h, int32_t lb_w, const mpr_sim_config& c, long long* epart_, double* e_real_,
                hipStream_t s_)
    {
        int ntx, nty, rchunk, nchunks;
        const int tile_h = 32;
        mpr::fused_geometry(H, W, c.n_real, tile_h, &ntx, &nty, &rchunk, &nchunks);
        a.tile_h = tile_h;
        a.src = state;
        a.dst = alt;
        a.mask = mask;
        a.Tb = tp;
        a.H = (int)H;
        a.W = (int)W;
        a.lb_h = lb_h;
        a.lb_w = lb_w;
        a.nbx = (int)((W + lb_w - 1) / lb_w);
        a.ntx = ntx;
        a.nty = nty;
        a.ntiles = ntx * nty;
        a.Mw = (int)((W + 3) / 4);
        a.R = c.n_real;
        a.rchunk = rchunk;
        a.nchunks = nchunks;
        a.HW = H * W;
        a.real_offset = (uint32_t)c.real_offset;
        a.scene = c.scene_id;
        a.key0 = (uint32_t)(c.seed & 0xffffffffu);
        a.key1 = (uint32_t)(c.seed >> 32);
        a.q = c.q;
        a.J = c.J;
        a.delta_e = mpr::kDeltaE * c.J;
        a.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
        a.Jd = (double)c.J;
        a.e_partial = nullptr;
        buf[0] = state;
        buf[1] = alt;
        cur = 0;
        const int64_t nbonds = H * (W - 1) + W * (H - 1);
        inv_norm = nbonds > 0 ? 1.0 / (double)nbonds : 0.0;
        epart = epart_;
        e_real = e_real_;
        s = s_;
    }

    float* current() const { return buf[cur]; }

    // one sweep k; with e_dst set, e(k) is written there
    hipError_t run(uint32_t k, double* e_dst)
    {
        a.sweep = k;
        a.src = buf[cur];
        a.dst = buf[cur ^ 1];
        a.e_partial = e_dst ? epart : nullptr;
        hipError_t e = mpr::launch_sweep_fused(a, s);
        if (e != hipSuccess) return e;
        cur ^= 1;
        if (e_dst) e = mpr::launch_energy_reduce(epart, a.ntiles, a.R, inv_norm, e_real, e_dst, s);
        return e;
    }
};

int fused_tiles(int64_t H, int64_t W, int R)
{
    int ntx, nty, rc, nc;
    mpr::fused_geometry(H, W, R, 32, &ntx, &nty, &rc, &nc);
    return ntx * nty;
}

struct SweepWs {
    mpr::TBand* tp;
    long long* epart;
    double* e_real;
};
size_t sweep_ws(Carve& c, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, SweepWs* w)
{
    SweepWs x;
    x.tp = c.take<mpr::TBand>(t_count(H, W, lb_h, lb_w, cfg));
    const int64_t R = cfg->n_real > 0 ? cfg->n_real : 1;
    x.epart = c.take<long long>((int64_t)fused_tiles(H, W, (int)R) * R);
    x.e_real = c.take<double>(R);
    if (w) *w = x;
    return c.used;
}

struct BatchWs {
    mpr::BatchScene* scenes;
    mpr::BatchRun* runs;
    int* order;
    int64_t* prefix;
    mpr::BatchCtl* ctl;
    StatsWs st;           // init scratch, sized for the largest scene
    double* Ts;
    int* No;
    float* gmean;
    std::vector<mpr::TBand*> tp;
    std::vector<float*> alt;
    std::vector<long long*> epart;
    std::vector<double*> e_real, series;
};

void batch_geom(int64_t H, int64_t W, int R, int tile_h, int* ntx, int* nty, int* ntiles, int* rchunk, int* nchunks)
{
    mpr::fused_geometry(H, W, R, tile_h, ntx, nty, rchunk, nchunks);
    *ntiles = (*ntx) * (*nty);
}

// Realization chunk of every work item in a batch: the scenes supply the parallelism, so an item covers as many
// realizations as possible (its LDS set-up is then shared by all of them), down to what keeps at least 8 items per
// workgroup slot of the persistent grid.
int batch_rchunk(const mpr_scene* sc, int n, int R, int tile_h)
{
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) {
        int ntx, nty, nt, rc, nc;
        batch_geom(sc[i].H, sc[i].W, R, tile_h, &ntx, &nty, &nt, &rc, &nc);
        tiles += nt;
    }
    int rc = std::min(R, 64);
    while (rc > 1 && tiles * ((R + rc - 1) / rc) < 8 * 1024) rc = (rc + 1) / 2;
    return rc;
}

size_t batch_ws(Carve& c, const mpr_scene* sc, int n, const mpr_sim_config* cfg, BatchWs* w)
{
    BatchWs x;
    const int64_t R = cfg->n_real > 0 ? cfg->n_real : 1;
    x.scenes = c.take<mpr::BatchScene>(n);
    x.runs = c.take<mpr::BatchRun>(n);
    x.order = c.take<int>(n);
    x.prefix = c.take<int64_t>(n + 1);
    x.ctl = c.take<mpr::BatchCtl>(1);
    int64_t max_np = 1, max_B = 1;
    for (int i = 0; i < n; ++i) {
        mpr::StatsGeom g = mpr::stats_geom(sc[i].H, sc[i].W, sc[i].lb_h, sc[i].lb_w);
        max_np = std::max<int64_t>(max_np, g.B() * g.nchunk);
        max_B = std::max<int64_t>(max_B, g.B());
    }
    x.st.pS = c.take<double>(max_np);
    x.st.pTs = c.take<double>(max_np);
    x.st.pN = c.take<int>(max_np);
    x.st.pNo = c.take<int>(max_np);
    x.Ts = c.take<double>(max_B);
    x.No = c.take<int>(max_B);
    x.gmean = c.take<float>(1);
    const int64_t cap = cfg->stop_mode == MPR_STOP_AUTO ? cfg->n_max : cfg->n_eq;
    for (int i = 0; i < n; ++i) {
        const int64_t H = sc[i].H, W = sc[i].W;
        x.tp.push_back(c.take<mpr::TBand>(nblocks_of(H, W, sc[i].lb_h, sc[i].lb_w)));
        x.alt.push_back(c.take<float>(R * H * W));
        int ntx, nty, nt16, nt32, rc, nc;
        batch_geom(H, W, (int)R, 16, &ntx, &nty, &nt16, &rc, &nc);
        batch_geom(H, W, (int)R, 32, &ntx, &nty, &nt32, &rc, &nc);
        const int64_t np = std::max<int64_t>(std::max(nt16, nt32), mpr::energy_full_parts(H, W));
        x.epart.push_back(c.take<long long>(np * R));
        x.e_real.push_back(c.take<double>(R));
        x.series.push_back(sc[i].energy ? sc[i].energy : c.take<double>((cap > 0 ? cap : 0) + 1));
    }
    if (w) *w = std::move(x);
    return c.used;
}

// The lane batch: per scene its temperature table, window bits, two lane-layout state buffers and reductions.
// The scenes' starts run on kSetupLanes streams (the caller's and three private ones), each with its own scratch for
// the block means: with many small scenes one stream leaves the device mostly idle between their short launches.
constexpr int kSetupLanes = 4;

struct BatchLaneWs {
    mpr::BatchLaneScene* scenes;
    mpr::BatchRun* runs;
    int* order;
    int64_t* prefix;
    mpr::BatchLaneCtl* ctl;
    StatsWs st[kSetupLanes];
    double* Ts[kSetupLanes];
    int* No[kSetupLanes];
    float* gmean[kSetupLanes];
    int64_t* gaps;                 // [n] gap sites per scene (the XCD split of the work list)
    std::vector<mpr::TBand*> tp;
    std::vector<uint2*> cells;
    std::vector<float*> buf0, buf1;
    std::vector<long long*> epart;
    std::vector<double*> e_real, series;
};

size_t batchl_ws(Carve& c, const mpr_scene* sc, int n, const mpr_sim_config* cfg, BatchLaneWs* w)
{
    BatchLaneWs x;
    const int64_t R = cfg->n_real > 0 ? cfg->n_real : 1;
    x.scenes = c.take<mpr::BatchLaneScene>(n);
    x.runs = c.take<mpr::BatchRun>(n);
    x.order = c.take<int>(n);
    x.prefix = c.take<int64_t>(n + 1);
    x.ctl = c.take<mpr::BatchLaneCtl>(1);
    int64_t max_np = 1, max_B = 1;
    for (int i = 0; i < n; ++i) {
        mpr::StatsGeom g = mpr::stats_geom(sc[i].H, sc[i].W, sc[i].lb_h, sc[i].lb_w);
        max_np = std::max<int64_t>(max_np, g.B() * g.nchunk);
        max_B = std::max<int64_t>(max_B, g.B());
    }
    for (int j = 0; j < kSetupLanes; ++j) {
        x.st[j].pS = c.take<double>(max_np);
        x.st[j].pTs = c.take<double>(max_np);
        x.st[j].pN = c.take<int>(max_np);
        x.st[j].pNo = c.take<int>(max_np);
        x.Ts[j] = c.take<double>(max_B);
        x.No[j] = c.take<int>(max_B);
        x.gmean[j] = c.take<float>(1);
    }
    x.gaps = c.take<int64_t>(n);
    const int64_t cap = cfg->stop_mode == MPR_STOP_AUTO ? cfg->n_max : cfg->n_eq;
    for (int i = 0; i < n; ++i) {
        const int64_t H = sc[i].H, W = sc[i].W;
        const mpr::RlGeom g = mpr::rl_geometry_full(H, W, (int)R);
        x.tp.push_back(c.take<mpr::TBand>(nblocks_of(H, W, sc[i].lb_h, sc[i].lb_w)));
        x.cells.push_back(c.take<uint2>((H + 4) * (int64_t)g.nbands));
        x.buf0.push_back(c.take<float>((int64_t)g.Rp * H * W));
        x.buf1.push_back(c.take<float>((int64_t)g.Rp * H * W));
        const int64_t np = std::max<int64_t>((int64_t)g.nbands * g.nseg, mpr::energy_full_parts(H, W));
        x.epart.push_back(c.take<long long>(np * R));
        x.e_real.push_back(c.take<double>(R));
        x.series.push_back(sc[i].energy ? sc[i].energy : c.take<double>((cap > 0 ? cap : 0) + 1));
    }
    if (w) *w = std::move(x);
    return c.used;
}

// The energy partials of a start in the [R][H][W] layout: a block-mean start holds the same state in every
// realization (it has no random part), so realization 0's partials are computed and copied to the others.
hipError_t start_energy_partials(const float* state, int64_t H, int64_t W, int R, const mpr_sim_config& c,
                                 long long* partial, int nparts, hipStream_t s)
{
    const bool same = c.init_mode == MPR_INIT_BLOCK_MEAN;
    hipError_t e = mpr::launch_energy_full(state, H, W, same ? 1 : R, c.q, c.J, partial, nparts, s);
    if (e == hipSuccess && same) e = mpr::launch_rows_from_first(partial, nparts, R, s);
    return e;
}

// private streams of the batched starts (default priority, created once per thread and device)
hipStream_t setup_stream(int j)
{
    static thread_local hipStream_t ss[kMaxDevices][kSetupLanes - 1] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    hipStream_t& st = ss[dev][j];
    if (!st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    return st;
}

// events of one fork of the caller's stream into the setup streams and of their join, released on every return
struct SetupFork {
    hipEvent_t ev[kSetupLanes] = {};
    ~SetupFork()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// private stream used only to capture graphs (graphs are launched on the caller's stream), one per host thread and
// device
hipStream_t capture_stream()
{
    static thread_local hipStream_t cs[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    if (!cs[dev] && hipStreamCreateWithFlags(&cs[dev], hipStreamNonBlocking) != hipSuccess) cs[dev] = nullptr;
    return cs[dev];
}

}  // namespace

extern "C" {

int32_t mpr_abi_version(void) { return 10000; }

const char* mpr_last_error(void) { return g_last_error.c_str(); }

size_t mpr_block_energy_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t n_real)
{
    if (H < 1 || W < 1 || lb_h < 1 || lb_w < 1 || n_real < 1) return 0;
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    Carve c{nullptr, 0, 0};
    c.take<double>(g.B() * g.nchunk * (int64_t)n_real);
    return c.used;
}

mpr_status mpr_block_energy(const float* state, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w,
                            float q, float J, int32_t n_real, double* H_out, void* workspace, size_t ws_bytes,
                            void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!state || !mask || !H_out) return fail(MPR_ERR_INVALID_ARG, "mpr_block_energy: NULL pointer");
    if (!(q > 0.0f && q <= 0.5f) || !(J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    if (n_real < 1 || n_real > 65535) return fail(MPR_ERR_INVALID_ARG, "n_real must be in 1 .. 65535");
    st = check_ws(workspace, ws_bytes, mpr_block_energy_workspace_bytes(H, W, lb_h, lb_w, n_real));
    if (st != MPR_OK) return st;
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    double* part = c.take<double>(g.B() * g.nchunk * (int64_t)n_real);
    MPR_HIP(mpr::launch_block_energy(state, mask, g, 2.0 * mpr::kPi * (double)q, (double)J, n_real, part, H_out,
                                     S(stream)));
    return ok();
}

size_t mpr_temperature_grad_workspace_bytes(int64_t H, int64_t W, int32_t n_real)
{
    if (H < 1 || W < 1 || n_real < 1) return 0;
    Carve c{nullptr, 0, 0};
    c.take<double>((int64_t)mpr::grad_parts(H * W) * n_real);
    c.take<double>(n_real);
    return c.used;
}

mpr_status mpr_temperature_grad(const float* state, const double* H_blocks, const float* grad_zhat,
                                const uint8_t* mask, int64_t H, int64_t W, int32_t n_real, int64_t n_blocks,
                                const double* range, const float* T_blocks, double* dT_out, void* workspace,
                                size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if (!state || !H_blocks || !grad_zhat || !mask || !range || !T_blocks || !dT_out)
        return fail(MPR_ERR_INVALID_ARG, "mpr_temperature_grad: NULL pointer");
    if (n_real < 2 || n_real > 65535) return fail(MPR_ERR_INVALID_ARG, "n_real must be in 2 .. 65535");
    if (n_blocks < 1) return fail(MPR_ERR_INVALID_ARG, "n_blocks must be >= 1");
    st = check_ws(workspace, ws_bytes, mpr_temperature_grad_workspace_bytes(H, W, n_real));
    if (st != MPR_OK) return st;
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    double* part = c.take<double>((int64_t)mpr::grad_parts(H * W) * n_real);
    double* g = c.take<double>(n_real);
    MPR_HIP(mpr::launch_temperature_grad(state, H_blocks, grad_zhat, mask, H * W, n_real, n_blocks, range, T_blocks,
                                         part, g, dT_out, S(stream)));
    return ok();
}

size_t mpr_map_workspace_bytes(int64_t H, int64_t W)
{
    Carve c{nullptr, 0, 0};
    return map_ws(c, H * W, nullptr);
}

mpr_status mpr_map_angles(const float* z, const uint8_t* mask, int64_t H, int64_t W, float* t_out, double* range_out,
                          void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if (!z || !mask || !t_out || !range_out) return fail(MPR_ERR_INVALID_ARG, "mpr_map_angles: NULL pointer");
    const int64_t n = H * W;
    st = check_ws(workspace, ws_bytes, mpr_map_workspace_bytes(H, W));
    if (st != MPR_OK) return st;
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    MapWs w;
    map_ws(c, n, &w);
    hipStream_t s = S(stream);
    MPR_HIP(mpr::launch_map_reduce(z, mask, n, w.pmin, w.pmax, w.pcnt, w.pbad, w.nb, s));
    MPR_HIP(mpr::launch_map_finalize(w.pmin, w.pmax, w.pcnt, w.pbad, w.nb, range_out, w.counts, s));
    unsigned long long counts[2] = {0, 0};
    MPR_HIP(hipMemcpyAsync(counts, w.counts, sizeof counts, hipMemcpyDeviceToHost, s));
    MPR_HIP(hipStreamSynchronize(s));
    if (counts[0] == 0) return fail(MPR_ERR_NO_SAMPLES, "mpr_map_angles: the mask has no observed site");
    if (counts[1] != 0)
        return fail(MPR_ERR_NONFINITE_INPUT, "mpr_map_angles: %llu observed values are not finite", counts[1]);
    MPR_HIP(mpr::launch_map_apply(z, mask, n, range_out, t_out, s));
    return ok();
}

size_t mpr_block_stats_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w)
{
    if (H < 1 || W < 1 || lb_h < 1 || lb_w < 1) return 0;
    Carve c{nullptr, 0, 0};
    return stats_ws(c, mpr::stats_geom(H, W, lb_h, lb_w), nullptr);
}

mpr_status mpr_block_stats(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w,
                           float q, float J, double* S_out, int32_t* N_out, double* Tsum_out, int32_t* Nobs_out,
                           void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!t || !mask) return fail(MPR_ERR_INVALID_ARG, "mpr_block_stats: NULL input");
    if (!(q > 0.0f && q <= 0.5f) || !(J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    st = check_ws(workspace, ws_bytes, mpr_block_stats_workspace_bytes(H, W, lb_h, lb_w));
    if (st != MPR_OK) return st;
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    StatsWs w;
    stats_ws(c, g, &w);
    MPR_HIP(mpr::launch_block_stats(t, mask, g, 2.0 * mpr::kPi * (double)q, (double)J, w.pS, w.pN, w.pTs, w.pNo,
                                    S_out, N_out, Tsum_out, Nobs_out, S(stream)));
    return ok();
}

size_t mpr_reference_curve_workspace_bytes(int32_t nT, int32_t L)
{
    if (nT < 1 || L < 2) return 0;
    Carve c{nullptr, 0, 0};
    return ref_ws(c, nT, L, nullptr);
}

mpr_status mpr_reference_curve(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm, int32_t n_meas,
                               uint64_t seed, double* e_out, void* workspace, size_t ws_bytes, void* stream)
{
    if (!(q > 0.0f && q <= 0.5f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2");
    if (nT < 1 || nT > 65535) return fail(MPR_ERR_INVALID_ARG, "nT must be in 1 .. 65535");
    if (L < 2 || L > 4096 || (L & 1)) return fail(MPR_ERR_SHAPE, "L must be even and in 2 .. 4096");
    if (n_therm < 0 || n_meas < 1) return fail(MPR_ERR_INVALID_ARG, "need n_therm >= 0 and n_meas >= 1");
    if (!T_grid || !e_out) return fail(MPR_ERR_INVALID_ARG, "mpr_reference_curve: NULL pointer");
    mpr_status st = check_ws(workspace, ws_bytes, mpr_reference_curve_workspace_bytes(nT, L));
    if (st != MPR_OK) return st;
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    RefWs w;
    ref_ws(c, nT, L, &w);
    hipStream_t s = S(stream);
    MPR_HIP(mpr::launch_ref_fill(w.state, (int64_t)nT * L * L, 0.5f, s));
    mpr::RefArgs a;
    a.state = w.state;
    a.Tgrid = T_grid;
    a.L = L;
    a.Mw = (L + 3) / 4;
    a.key0 = (uint32_t)(seed & 0xffffffffu);
    a.key1 = (uint32_t)(seed >> 32);
    a.q = q;
    a.delta_e = mpr::kDeltaE;
    a.two_pi_q = 2.0 * mpr::kPi * (double)q;
    const double inv_norm = 1.0 / (2.0 * (double)L * (double)L);
    for (int32_t k = 1; k <= n_therm + n_meas; ++k) {
        a.sweep = (uint32_t)k;
        for (int colour = 0; colour < 2; ++colour) {
            a.colour = colour;
            MPR_HIP(mpr::launch_ref_half(a, nT, s));
        }
        if (k > n_therm) {
            MPR_HIP(mpr::launch_ref_energy(w.state, L, nT, q, w.part, w.nparts, s));
            MPR_HIP(mpr::launch_ref_accumulate(w.part, w.nparts, nT, inv_norm, w.esum, k == n_therm + 1 ? 1 : 0, s));
        }
    }
    MPR_HIP(mpr::launch_ref_finish(w.esum, nT, (double)n_meas, e_out, s));
    return ok();
}

size_t mpr_calibrate_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w)
{
    if (H < 1 || W < 1 || lb_h < 1 || lb_w < 1) return 0;
    Carve c{nullptr, 0, 0};
    return cal_ws(c, mpr::stats_geom(H, W, lb_h, lb_w), nullptr);
}

mpr_status mpr_calibrate_temperature(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h,
                                     int32_t lb_w, float q, float J, const double* curve_T, const double* curve_e,
                                     int32_t n_curve, float* T_out, double* e_blocks_out, int32_t* nbonds_out,
                                     void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!t || !mask || !curve_T || !curve_e || !T_out)
        return fail(MPR_ERR_INVALID_ARG, "mpr_calibrate_temperature: NULL pointer");
    if (n_curve < 1) return fail(MPR_ERR_INVALID_ARG, "n_curve must be >= 1");
    if (!(q > 0.0f && q <= 0.5f) || !(J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    st = check_ws(workspace, ws_bytes, mpr_calibrate_workspace_bytes(H, W, lb_h, lb_w));
    if (st != MPR_OK) return st;
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    CalWs w;
    cal_ws(c, g, &w);
    hipStream_t s = S(stream);
    MPR_HIP(mpr::launch_block_stats(t, mask, g, 2.0 * mpr::kPi * (double)q, (double)J, w.st.pS, w.st.pN, w.st.pTs,
                                    w.st.pNo, w.S, w.N, nullptr, nullptr, s));
    MPR_HIP(mpr::launch_calibrate(w.S, w.N, g.B(), (double)J, curve_T, curve_e, n_curve, T_out, e_blocks_out,
                                  nbonds_out, w.n_have, s));
    unsigned n_have = 0;
    MPR_HIP(hipMemcpyAsync(&n_have, w.n_have, sizeof n_have, hipMemcpyDeviceToHost, s));
    MPR_HIP(hipStreamSynchronize(s));
    if (n_have == 0)
        return fail(MPR_ERR_NO_SAMPLE_BONDS, "no pair of neighbouring samples: the temperature cannot be estimated");
    return ok();
}

mpr_status mpr_calibrate_temperature_noalloc(const float* t, const uint8_t* mask, int64_t H, int64_t W,
                                             int32_t lb_h, int32_t lb_w, float q, float J, const double* curve_T,
                                             const double* curve_e, int32_t n_curve, float* T_out,
                                             double* e_blocks_out, int32_t* nbonds_out, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    const size_t need = mpr_calibrate_workspace_bytes(H, W, lb_h, lb_w);
    if (need > (size_t)MPR_NOALLOC_SCRATCH_BYTES)
        return fail(MPR_ERR_WORKSPACE_TOO_SMALL,
                    "mpr_calibrate_temperature_noalloc: %lld x %lld with %d x %d blocks needs %zu bytes of scratch, "
                    "the static scratch holds %zu (use mpr_calibrate_temperature with a workspace)",
                    (long long)H, (long long)W, lb_h, lb_w, need, (size_t)MPR_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((st = scratch_for_current_device(&ws)) != MPR_OK) return st;
    // every scratch entry the calibration reads is written earlier in the same call: nothing has to start at zero
    return mpr_calibrate_temperature(t, mask, H, W, lb_h, lb_w, q, J, curve_T, curve_e, n_curve, T_out, e_blocks_out,
                                     nbonds_out, ws, (size_t)MPR_NOALLOC_SCRATCH_BYTES, stream);
}

mpr_status mpr_calibrate_directional(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h,
                                     int32_t lb_w, float q, float J, const double* curve_T, const double* curve_e,
                                     int32_t n_curve, float* Tx_out, float* Ty_out, void* workspace, size_t ws_bytes,
                                     void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!t || !mask || !curve_T || !curve_e || !Tx_out || !Ty_out)
        return fail(MPR_ERR_INVALID_ARG, "mpr_calibrate_directional: NULL pointer");
    if (n_curve < 1) return fail(MPR_ERR_INVALID_ARG, "n_curve must be >= 1");
    if (!(q > 0.0f && q <= 0.5f) || !(J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    st = check_ws(workspace, ws_bytes, mpr_calibrate_workspace_bytes(H, W, lb_h, lb_w));
    if (st != MPR_OK) return st;
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    CalWs w;
    cal_ws(c, g, &w);
    hipStream_t s = S(stream);
    const float floor_T = (float)(mpr::kTMinDirectional * (double)J);
    float* outs[2] = {Tx_out, Ty_out};
    for (int d = 0; d < 2; ++d) {
        // bonds 1: horizontal (a sample and its right neighbour), 2: vertical (a sample and its lower neighbour)
        MPR_HIP(mpr::launch_block_stats(t, mask, g, 2.0 * mpr::kPi * (double)q, (double)J, w.st.pS, w.st.pN,
                                        w.st.pTs, w.st.pNo, w.S, w.N, nullptr, nullptr, s, d + 1));
        MPR_HIP(mpr::launch_calibrate(w.S, w.N, g.B(), (double)J, curve_T, curve_e, n_curve, outs[d], nullptr,
                                      nullptr, w.n_have, s));
        unsigned n_have = 0;
        MPR_HIP(hipMemcpyAsync(&n_have, w.n_have, sizeof n_have, hipMemcpyDeviceToHost, s));
        MPR_HIP(hipStreamSynchronize(s));
        if (n_have == 0)
            return fail(MPR_ERR_NO_SAMPLE_BONDS, "no %s pair of neighbouring samples: T%s cannot be estimated",
                        d == 0 ? "horizontal" : "vertical", d == 0 ? "x" : "y");
        MPR_HIP(mpr::launch_floor(outs[d], g.B(), floor_T, s));
    }
    return ok();
}

size_t mpr_simulate_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg)
{
    if (!cfg || H < 1 || W < 1 || lb_h < 1 || lb_w < 1) return 0;
    Carve c{nullptr, 0, 0};
    return sim_ws(c, H, W, lb_h, lb_w, cfg, nullptr);
}

mpr_status mpr_simulate(const float* t, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks,
                        int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, float* state, double* acc_out,
                        double* energy_out, int32_t* sweeps_done_out, void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!cfg) return fail(MPR_ERR_INVALID_ARG, "cfg is NULL");
    if (!t || !mask || !T_blocks || !state || !acc_out) return fail(MPR_ERR_INVALID_ARG, "mpr_simulate: NULL pointer");
    const mpr_sim_config& c = *cfg;
    if ((st = check_sim_config(c)) != MPR_OK) return st;
    if (c.init_mode != MPR_INIT_RANDOM && c.init_mode != MPR_INIT_BLOCK_MEAN)
        return fail(MPR_ERR_INVALID_ARG, "unknown init_mode %d", c.init_mode);
    if (c.stop_mode != MPR_STOP_FIXED && !auto_stop(c.stop_mode))
        return fail(MPR_ERR_INVALID_ARG, "unknown stop_mode %d", c.stop_mode);
    if (c.n_samp < 0) return fail(MPR_ERR_INVALID_ARG, "n_samp must be >= 0");
    if (c.stop_mode == MPR_STOP_FIXED && c.n_eq < 0) return fail(MPR_ERR_INVALID_ARG, "n_eq must be >= 0");
    if (auto_stop(c.stop_mode) && (c.n_fit < 2 || c.n_f < 1 || c.n_max < 1))
        return fail(MPR_ERR_INVALID_ARG, "AUTO needs n_fit >= 2, n_f >= 1, n_max >= 1");
    if ((c.sweep_kernel == MPR_SWEEP_LANES || c.coupling == MPR_COUPLING_DIRECTIONAL) && (H >= 65536 || W >= 65536))
        return fail(MPR_ERR_SHAPE, "the realization-lane sweep (and the directional coupling) needs sides below 65536");
    st = check_ws(workspace, ws_bytes, mpr_simulate_workspace_bytes(H, W, lb_h, lb_w, cfg));
    if (st != MPR_OK) return st;

    hipStream_t s = S(stream);
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    SimWs w;
    sim_ws(cv, H, W, lb_h, lb_w, cfg, &w);
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    const int64_t B = g.B();
    const int64_t HW = H * W;
    const int R = c.n_real;
    const uint32_t key0 = (uint32_t)(c.seed & 0xffffffffu), key1 = (uint32_t)(c.seed >> 32);

    // start of the chains
    if (c.init_mode == MPR_INIT_BLOCK_MEAN) {
        MPR_HIP(mpr::launch_block_stats(t, mask, g, 2.0 * mpr::kPi * (double)c.q, (double)c.J, w.st.pS, w.st.pN,
                                        w.st.pTs, w.st.pNo, nullptr, nullptr, w.Ts, w.No, s));
        MPR_HIP(mpr::launch_global_mean(w.Ts, w.No, B, w.gmean, s));
    }
    mpr::InitArgs ia;
    ia.state = state;
    ia.state2 = w.alt;
    ia.t = t;
    ia.mask = mask;
    ia.Ts = w.Ts;
    ia.No = w.No;
    ia.gmean = w.gmean;
    ia.H = H;
    ia.W = W;
    ia.lb_h = lb_h;
    ia.lb_w = lb_w;
    ia.nbx = g.nbx;
    ia.R = R;
    ia.real_offset = (uint32_t)c.real_offset;
    ia.scene = c.scene_id;
    ia.key0 = key0;
    ia.key1 = key1;
    ia.mode = c.init_mode;
    // the realization-lane sweep starts straight in its two lane buffers (both hold the samples); the final state
    // moves back into `state`
    const bool rl = use_rl(H, W, cfg);
    if (rl) MPR_HIP(mpr::launch_rl_init(ia, mpr::rl_geometry(H, W, R).Rp, w.rl[0], w.rl[1], s));
    else MPR_HIP(mpr::launch_init(ia, s));
    const bool directional = c.coupling == MPR_COUPLING_DIRECTIONAL;
    if (directional) {
        MPR_HIP(mpr::launch_tpairs_directional(T_blocks, nblocks_of(H, W, lb_h, lb_w), c.J, mpr::kDeltaE * c.J,
                                               (float)(mpr::kTMinDirectional * (double)c.J), w.tpd, s));
    } else {
        MPR_HIP(mpr::launch_tpairs(T_blocks, t_count(H, W, lb_h, lb_w, cfg), c.J, mpr::kDeltaE * c.J, w.tp, s));
    }

    const bool need_energy = auto_stop(c.stop_mode) || energy_out != nullptr;
    SweepRunner runner(state, w.alt, mask, H, W, w.tp, t_lb(lb_h, c), t_lb(lb_w, c), c, w.epart, w.e_real, s);
    const int nfull = mpr::energy_full_parts(H, W);
    if (need_energy) {
        if (rl)
            MPR_HIP(mpr::launch_rl_energy_full(w.rl[0], H, W, R, c.q, w.epart, nfull,
                                               c.init_mode == MPR_INIT_BLOCK_MEAN, s));
        else MPR_HIP(start_energy_partials(state, H, W, R, c, w.epart, nfull, s));
        MPR_HIP(mpr::launch_energy_reduce(w.epart, nfull, R, runner.inv_norm, w.e_real, w.series, s));
    }
    // double checkerboard: in place in `state`, energy of the whole grid after the sweep
    const bool dc = c.order == MPR_ORDER_DC;
    mpr::DcArgs da;
    da.state = state;
    da.mask = mask;
    da.tb = w.tp;
    da.H = H;
    da.W = W;
    da.lb_h = lb_h;
    da.lb_w = lb_w;
    da.tb_h = t_lb(lb_h, c);
    da.tb_w = t_lb(lb_w, c);
    da.nbx_t = (int)((W + da.tb_w - 1) / da.tb_w);
    da.Mw = (int)((W + 3) / 4);
    da.R = R;
    da.real_offset = (uint32_t)c.real_offset;
    da.scene = c.scene_id;
    da.key0 = key0;
    da.key1 = key1;
    da.q = c.q;
    da.J = c.J;
    da.delta_e = mpr::kDeltaE * c.J;
    da.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
    da.Jd = (double)c.J;
    // realization-lane sweep: sweeps alternate between the two [HW][Rp] buffers
    mpr::RlArgs ra{};
    int rl_cur = 0;
    if (rl) {
        const mpr::RlGeom rg = mpr::rl_geometry(H, W, R);
        ra.H = (int)H;
        ra.W = (int)W;
        ra.R = R;
        ra.Rp = rg.Rp;
        ra.Mw = (int)((W + 3) / 4);
        ra.nbands = rg.nbands;
        ra.nseg = rg.nseg;
        ra.seg_rows = rg.seg_rows;
        ra.n_items = rg.n_items;
        ra.tb_h = t_lb(lb_h, c);
        ra.tb_w = t_lb(lb_w, c);
        ra.nbx_t = (int)((W + ra.tb_w - 1) / ra.tb_w);
        ra.nby_t = (int)((H + ra.tb_h - 1) / ra.tb_h);
        ra.tb_w_inv = ra.tb_w > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)ra.tb_w - 1) / (uint64_t)ra.tb_w) : 0u;
        ra.real_offset = (uint32_t)c.real_offset;
        ra.scene = c.scene_id;
        ra.key0 = key0;
        ra.key1 = key1;
        ra.q = c.q;
        ra.J = c.J;
        ra.delta_e = mpr::kDeltaE * c.J;
        ra.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
        ra.Jd = (double)c.J;
        MPR_HIP(mpr::launch_rl_cells(mask, H, W, w.cells, s));
    }
    const int rl_parts = rl ? ra.nbands * ra.nseg : 0;
    auto sweep = [&](uint32_t k, bool energy) -> hipError_t {
        if (rl) {
            ra.sweep = k;
            hipError_t e = mpr::launch_sweep_rl(ra, w.cells, w.tp, directional ? w.tpd : nullptr, w.rl[rl_cur],
                                                w.rl[rl_cur ^ 1], energy ? w.epart : nullptr, s);
            rl_cur ^= 1;
            if (e == hipSuccess && energy)
                e = mpr::launch_energy_reduce(w.epart, rl_parts, R, runner.inv_norm, w.e_real, w.series + k, s);
            return e;
        }
        if (!dc) return runner.run(k, energy ? w.series + k : nullptr);
        hipError_t e = mpr::launch_dc_sweep(da, k, s);
        if (e == hipSuccess && energy) e = mpr::launch_energy_full(state, H, W, R, c.q, c.J, w.epart, nfull, s);
        if (e == hipSuccess && energy)
            e = mpr::launch_energy_reduce(w.epart, nfull, R, runner.inv_norm, w.e_real, w.series + k, s);
        return e;
    };
    auto current = [&]() -> float* { return dc ? state : runner.current(); };

    const int32_t cap = auto_stop(c.stop_mode) ? c.n_max : c.n_eq;
    int32_t k = 0;
    bool converged = true;
    double e0 = 0.0;
    std::vector<double> window;
    const bool per_chain = c.stop_mode == MPR_STOP_AUTO_CHAIN;
    ChainStop chains;
    if (c.stop_mode == MPR_STOP_AUTO) {
        MPR_HIP(hipMemcpyAsync(&e0, w.series, sizeof(double), hipMemcpyDeviceToHost, s));
        window.resize((size_t)c.n_fit);
    }
    if (per_chain) {
        MPR_HIP(hipMemcpyAsync(w.hist, w.e_real, sizeof(double) * (size_t)R, hipMemcpyDeviceToDevice, s));
        MPR_HIP(chains.start(w.hist, R, c.n_fit, s));
    }
    while (k < cap) {
        ++k;
        MPR_HIP(sweep((uint32_t)k, need_energy));
        if (per_chain)
            MPR_HIP(hipMemcpyAsync(w.hist + (int64_t)k * R, w.e_real, sizeof(double) * (size_t)R,
                                   hipMemcpyDeviceToDevice, s));
        if (auto_stop(c.stop_mode)) {
            if (k >= c.n_fit + c.n_f && (k - c.n_fit) % c.n_f == 0) {
                bool done = false;
                if (per_chain) {
                    MPR_HIP(chains.check(w.hist, k, s, &done));
                } else {
                    MPR_HIP(hipMemcpyAsync(window.data(), w.series + (k - c.n_fit + 1), sizeof(double) * c.n_fit,
                                           hipMemcpyDeviceToHost, s));
                    MPR_HIP(hipStreamSynchronize(s));
                    done = equilibrium_reached(e0, window.data(), c.n_fit);
                }
                if (done) break;
            }
            if (k == c.n_max) converged = false;
        }
    }
    const int32_t k_star = k;
    if (c.n_samp == 0) {
        MPR_HIP(hipMemsetAsync(acc_out, 0, sizeof(double) * (size_t)HW, s));
    }
    for (int32_t si = 1; si <= c.n_samp; ++si) {
        MPR_HIP(sweep((uint32_t)(k_star + si), false));
        if (rl) MPR_HIP(mpr::launch_rl_accumulate(w.rl[rl_cur], mask, HW, R, si == 1 ? 1 : 0, acc_out, s));
        else MPR_HIP(mpr::launch_accumulate(current(), mask, HW, R, si == 1 ? 1 : 0, acc_out, s));
    }
    if (rl) {
        MPR_HIP(mpr::launch_rl_from_lanes(w.rl[rl_cur], HW, R, state, s));
    } else if (current() != state) {
        MPR_HIP(hipMemcpyAsync(state, current(), sizeof(float) * (size_t)(R * HW), hipMemcpyDeviceToDevice, s));
    }
    if (energy_out && need_energy) {
        MPR_HIP(hipMemcpyAsync(energy_out, w.series, sizeof(double) * (size_t)(k_star + 1), hipMemcpyDeviceToDevice,
                               s));
    }
    if (sweeps_done_out) *sweeps_done_out = k_star;
    if (!converged) return fail(MPR_WARN_NOT_CONVERGED, "equilibrium test not met after n_max = %d sweeps", c.n_max);
    return ok();
}

size_t mpr_sweep_workspace_bytes(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg)
{
    if (!cfg || H < 1 || W < 1 || lb_h < 1 || lb_w < 1) return 0;
    Carve c{nullptr, 0, 0};
    return sweep_ws(c, H, W, lb_h, lb_w, cfg, nullptr);
}

mpr_status mpr_sweep(float* state, float* state_alt, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks,
                     int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, int32_t k_first, int32_t n_sweeps,
                     double* energy_out, void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!cfg) return fail(MPR_ERR_INVALID_ARG, "cfg is NULL");
    if (!state || !state_alt || !mask || !T_blocks) return fail(MPR_ERR_INVALID_ARG, "mpr_sweep: NULL pointer");
    if (state == state_alt) return fail(MPR_ERR_INVALID_ARG, "mpr_sweep: state and state_alt must be distinct buffers");
    if ((st = check_sim_config(*cfg)) != MPR_OK) return st;
    if (cfg->order != MPR_ORDER_SC) return fail(MPR_ERR_INVALID_ARG, "mpr_sweep runs the single-checkerboard order");
    if (cfg->coupling != MPR_COUPLING_ISOTROPIC)
        return fail(MPR_ERR_INVALID_ARG, "mpr_sweep runs one temperature per block (isotropic coupling)");
    if (k_first < 1 || n_sweeps < 0) return fail(MPR_ERR_INVALID_ARG, "need k_first >= 1 and n_sweeps >= 0");
    st = check_ws(workspace, ws_bytes, mpr_sweep_workspace_bytes(H, W, lb_h, lb_w, cfg));
    if (st != MPR_OK) return st;
    hipStream_t s = S(stream);
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    SweepWs w;
    sweep_ws(cv, H, W, lb_h, lb_w, cfg, &w);
    MPR_HIP(mpr::launch_tpairs(T_blocks, t_count(H, W, lb_h, lb_w, cfg), cfg->J, mpr::kDeltaE * cfg->J, w.tp, s));
    SweepRunner runner(state, state_alt, mask, H, W, w.tp, t_lb(lb_h, *cfg), t_lb(lb_w, *cfg), *cfg, w.epart,
                       w.e_real, s);
    for (int32_t i = 0; i < n_sweeps; ++i)
        MPR_HIP(runner.run((uint32_t)(k_first + i), energy_out ? energy_out + i : nullptr));
    return ok();
}

mpr_status mpr_predict(const double* acc, const float* z, const uint8_t* mask, int64_t H, int64_t W,
                       int64_t n_samples, const double* range, float* zhat_out, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if (!acc || !z || !mask || !range || !zhat_out) return fail(MPR_ERR_INVALID_ARG, "mpr_predict: NULL pointer");
    if (n_samples < 1) return fail(MPR_ERR_INVALID_ARG, "n_samples must be >= 1");
    MPR_HIP(mpr::launch_predict(acc, z, mask, H * W, n_samples, range, zhat_out, S(stream)));
    return ok();
}

size_t mpr_validate_workspace_bytes(int64_t n)
{
    if (n < 0) return 0;
    Carve c{nullptr, 0, 0};
    c.take<double>((int64_t)3 * mpr::validate_blocks(n));
    return c.used;
}

mpr_status mpr_validate(const float* zhat, const float* truth, const uint8_t* eval_mask, int64_t n, double* out,
                        void* workspace, size_t ws_bytes, void* stream)
{
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(MPR_ERR_SHAPE, "n out of range");
    if (!out || (n > 0 && (!zhat || !truth || !eval_mask))) return fail(MPR_ERR_INVALID_ARG, "mpr_validate: NULL pointer");
    mpr_status st = check_ws(workspace, ws_bytes, mpr_validate_workspace_bytes(n));
    if (st != MPR_OK) return st;
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    const int nb = mpr::validate_blocks(n);
    double* part = c.take<double>((int64_t)3 * nb);
    MPR_HIP(mpr::launch_validate(zhat, truth, eval_mask, n, part, nb, out, S(stream)));
    return ok();
}

}  // extern "C"

extern "C" {

// The arguments of a batched call, checked once for the whole batch.
static mpr_status check_batched(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg, int32_t tile_h)
{
    if (!scenes || n_scenes < 1 || n_scenes > (1 << 20)) return fail(MPR_ERR_INVALID_ARG, "need 1 .. 2^20 scenes");
    if (!cfg) return fail(MPR_ERR_INVALID_ARG, "cfg is NULL");
    mpr_status st = check_sim_config(*cfg);
    if (st != MPR_OK) return st;
    const mpr_sim_config& c = *cfg;
    if (c.coupling != MPR_COUPLING_ISOTROPIC)
        return fail(MPR_ERR_INVALID_ARG, "the batched form runs one temperature per block (isotropic coupling)");
    if (c.init_mode != MPR_INIT_RANDOM && c.init_mode != MPR_INIT_BLOCK_MEAN)
        return fail(MPR_ERR_INVALID_ARG, "unknown init_mode %d", c.init_mode);
    if (c.stop_mode == MPR_STOP_AUTO_CHAIN)
        return fail(MPR_ERR_INVALID_ARG, "the batched form runs MPR_STOP_FIXED or MPR_STOP_AUTO (the per-chain test "
                                         "is available in mpr_simulate and mpr_simulate3d)");
    if (c.stop_mode != MPR_STOP_FIXED && c.stop_mode != MPR_STOP_AUTO)
        return fail(MPR_ERR_INVALID_ARG, "unknown stop_mode %d", c.stop_mode);
    if (c.n_samp < 0) return fail(MPR_ERR_INVALID_ARG, "n_samp must be >= 0");
    if (c.stop_mode == MPR_STOP_FIXED && c.n_eq < 1) return fail(MPR_ERR_INVALID_ARG, "batched FIXED mode needs n_eq >= 1");
    if (c.stop_mode == MPR_STOP_AUTO && (c.n_fit < 2 || c.n_f < 1 || c.n_max < 1))
        return fail(MPR_ERR_INVALID_ARG, "AUTO needs n_fit >= 2, n_f >= 1, n_max >= 1");
    if (tile_h != 0 && tile_h != 16 && tile_h != 32) return fail(MPR_ERR_INVALID_ARG, "tile_h must be 0, 16 or 32");
    if (c.t_mode != MPR_T_BLOCK) return fail(MPR_ERR_INVALID_ARG, "the batched form takes block temperatures only");
    if (c.order != MPR_ORDER_SC) return fail(MPR_ERR_INVALID_ARG, "the batched form runs the single-checkerboard order");
    for (int i = 0; i < n_scenes; ++i) {
        const mpr_scene& sc = scenes[i];
        if ((st = check_grid(sc.H, sc.W)) != MPR_OK) return st;
        if ((st = check_blocks(sc.H, sc.W, sc.lb_h, sc.lb_w)) != MPR_OK) return st;
        if (!sc.t || !sc.mask || !sc.T_blocks || !sc.state || !sc.acc)
            return fail(MPR_ERR_INVALID_ARG, "scene %d: NULL pointer", i);
        if (sc.scene_id >= (1u << 28)) return fail(MPR_ERR_INVALID_ARG, "scene %d: scene_id must be < 2^28", i);
    }
    return MPR_OK;
}

// The persistent tile-kernel batch over the scenes given (all of them run on the tile kernel).
static size_t batched_tiles_ws(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg)
{
    Carve c{nullptr, 0, 0};
    return batch_ws(c, scenes, n_scenes, cfg, nullptr);
}

static mpr_status batched_tiles(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg, int32_t tile_h,
                                int32_t* sweeps_done_out, int32_t* converged_out, int32_t* tile_h_used_out,
                                void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_batched(scenes, n_scenes, cfg, tile_h);
    if (st != MPR_OK) return st;
    const mpr_sim_config& c = *cfg;
    st = check_ws(workspace, ws_bytes, batched_tiles_ws(scenes, n_scenes, cfg));
    if (st != MPR_OK) return st;
    hipStream_t s = S(stream);
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    BatchWs w;
    batch_ws(cv, scenes, n_scenes, cfg, &w);
    const int R = c.n_real;
    const uint32_t key0 = (uint32_t)(c.seed & 0xffffffffu), key1 = (uint32_t)(c.seed >> 32);
    const bool energy = c.stop_mode == MPR_STOP_AUTO;
    bool any_energy_out = false;
    for (int i = 0; i < n_scenes; ++i) any_energy_out |= scenes[i].energy != nullptr;

    // ---- per-scene start, temperatures, e(0) ----
    const int rchunk_v[2] = {batch_rchunk(scenes, n_scenes, R, 16), batch_rchunk(scenes, n_scenes, R, 32)};
    std::vector<mpr::BatchScene> hs(n_scenes);
    std::vector<int64_t> work16(n_scenes), work32(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        const mpr_scene& sc = scenes[i];
        mpr::StatsGeom g = mpr::stats_geom(sc.H, sc.W, sc.lb_h, sc.lb_w);
        if (c.init_mode == MPR_INIT_BLOCK_MEAN) {
            MPR_HIP(mpr::launch_block_stats(sc.t, sc.mask, g, 2.0 * mpr::kPi * (double)c.q, (double)c.J, w.st.pS,
                                            w.st.pN, w.st.pTs, w.st.pNo, nullptr, nullptr, w.Ts, w.No, s));
            MPR_HIP(mpr::launch_global_mean(w.Ts, w.No, g.B(), w.gmean, s));
        }
        mpr::InitArgs ia;
        ia.state = sc.state;
        ia.state2 = w.alt[i];
        ia.t = sc.t;
        ia.mask = sc.mask;
        ia.Ts = w.Ts;
        ia.No = w.No;
        ia.gmean = w.gmean;
        ia.H = sc.H;
        ia.W = sc.W;
        ia.lb_h = sc.lb_h;
        ia.lb_w = sc.lb_w;
        ia.nbx = g.nbx;
        ia.R = R;
        ia.real_offset = (uint32_t)c.real_offset;
        ia.scene = sc.scene_id;
        ia.key0 = key0;
        ia.key1 = key1;
        ia.mode = c.init_mode;
        MPR_HIP(mpr::launch_init(ia, s));
        MPR_HIP(mpr::launch_tpairs(sc.T_blocks, g.B(), c.J, mpr::kDeltaE * c.J, w.tp[i], s));
        const int64_t nbonds = sc.H * (sc.W - 1) + sc.W * (sc.H - 1);
        const double inv_norm = nbonds > 0 ? 1.0 / (double)nbonds : 0.0;
        if (energy || sc.energy) {
            const int nfull = mpr::energy_full_parts(sc.H, sc.W);
            MPR_HIP(start_energy_partials(sc.state, sc.H, sc.W, R, c, w.epart[i], nfull, s));
            MPR_HIP(mpr::launch_energy_reduce(w.epart[i], nfull, R, inv_norm, w.e_real[i], w.series[i], s));
        }
        if (c.n_samp == 0) MPR_HIP(hipMemsetAsync(sc.acc, 0, sizeof(double) * (size_t)(sc.H * sc.W), s));
        mpr::BatchScene& d = hs[i];
        d.t = sc.t;
        d.mask = sc.mask;
        d.tp = w.tp[i];
        d.buf[0] = sc.state;
        d.buf[1] = w.alt[i];
        d.acc = sc.acc;
        d.epart = w.epart[i];
        d.e_real = w.e_real[i];
        d.series = w.series[i];
        d.H = (int)sc.H;
        d.W = (int)sc.W;
        d.lb_h = sc.lb_h;
        d.lb_w = sc.lb_w;
        d.nbx = g.nbx;
        d.Mw = (int)((sc.W + 3) / 4);
        for (int v = 0; v < 2; ++v) {
            int ntx, nty, nt, rc, nc;
            batch_geom(sc.H, sc.W, R, v ? 32 : 16, &ntx, &nty, &nt, &rc, &nc);
            rc = rchunk_v[v];
            nc = (R + rc - 1) / rc;
            d.ntx = ntx;
            d.nty[v] = nty;
            d.ntiles[v] = nt;
            d.rchunk[v] = rc;
            d.nchunks[v] = nc;
        }
        work16[i] = (int64_t)d.ntiles[0] * d.nchunks[0];
        work32[i] = (int64_t)d.ntiles[1] * d.nchunks[1];
        d.HW = sc.H * sc.W;
        d.scene = sc.scene_id;
        d.inv_norm = inv_norm;
    }
    // largest scenes first
    std::vector<int> order(n_scenes);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work32[a] > work32[b]; });
    int variant = tile_h == 16 ? 0 : 1;
    const int first_variant = tile_h == 0 ? 0 : variant;
    std::vector<int64_t> prefix(n_scenes + 1, 0);
    for (int i = 0; i < n_scenes; ++i)
        prefix[i + 1] = prefix[i] + (first_variant ? work32[order[i]] : work16[order[i]]);
    std::vector<mpr::BatchRun> runs(n_scenes, mpr::BatchRun{0, 0, 0, 1});
    mpr::BatchCtl ctl{0, n_scenes, 0ull};
    MPR_HIP(hipMemcpyAsync(w.scenes, hs.data(), sizeof(mpr::BatchScene) * n_scenes, hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.runs, runs.data(), sizeof(mpr::BatchRun) * n_scenes, hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.order, order.data(), sizeof(int) * n_scenes, hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.prefix, prefix.data(), sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, s));
    MPR_HIP(hipStreamSynchronize(s));     // the host arrays above must outlive the copies

    mpr::BatchDev b;
    b.scenes = w.scenes;
    b.runs = w.runs;
    b.order = w.order;
    b.prefix = w.prefix;
    b.ctl = w.ctl;
    b.n = n_scenes;
    b.cfg.R = R;
    b.cfg.real_offset = (uint32_t)c.real_offset;
    b.cfg.key0 = key0;
    b.cfg.key1 = key1;
    b.cfg.q = c.q;
    b.cfg.J = c.J;
    b.cfg.delta_e = mpr::kDeltaE * c.J;
    b.cfg.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
    b.cfg.Jd = (double)c.J;
    b.cfg.energy = (energy || any_energy_out) ? 1 : 0;
    b.cfg.stop_mode = c.stop_mode;
    b.cfg.n_fit = c.n_fit;
    b.cfg.n_f = c.n_f;
    b.cfg.n_max = c.n_max;
    b.cfg.n_eq = c.n_eq;
    b.cfg.n_samp = c.n_samp;
    int max_hw_blocks = 1;
    for (int i = 0; i < n_scenes; ++i)
        max_hw_blocks = std::max<int>(max_hw_blocks, (int)std::min<int64_t>((hs[i].HW + 255) / 256, 1024));
    const int grid = 256 * 4;              // four workgroups per CU, persistent
    const int32_t cap = c.stop_mode == MPR_STOP_AUTO ? c.n_max : c.n_eq;
    const int32_t total_max = cap + c.n_samp;
    int32_t done = 0;

    // ---- tile-height autotuning on the first two (real) sweeps ----
    if (tile_h == 0) {
        hipEvent_t ev[3];
        for (auto& e : ev) MPR_HIP(hipEventCreate(&e));
        MPR_HIP(hipEventRecord(ev[0], s));
        MPR_HIP(mpr::launch_batch_step(b, 0, 1, grid, max_hw_blocks, s));
        MPR_HIP(hipEventRecord(ev[1], s));
        MPR_HIP(mpr::launch_batch_step(b, 1, 1, grid, max_hw_blocks, s));
        MPR_HIP(hipEventRecord(ev[2], s));
        MPR_HIP(hipEventSynchronize(ev[2]));
        float t16 = 0.f, t32 = 0.f;
        MPR_HIP(hipEventElapsedTime(&t16, ev[0], ev[1]));
        MPR_HIP(hipEventElapsedTime(&t32, ev[1], ev[2]));
        for (auto& e : ev) MPR_HIP(hipEventDestroy(e));
        variant = t16 < t32 ? 0 : 1;
        done = 2;
        if (variant == 0) {                // the work list after sweep 2 was built for tiles of height 32
            MPR_HIP(hipMemcpyAsync(&runs[0], w.runs, sizeof(mpr::BatchRun) * n_scenes, hipMemcpyDeviceToHost, s));
            MPR_HIP(hipStreamSynchronize(s));
            int64_t acc = 0;
            for (int i = 0; i < n_scenes; ++i) {
                prefix[i] = acc;
                if (runs[order[i]].phase < 2) acc += work16[order[i]];
            }
            prefix[n_scenes] = acc;
            MPR_HIP(hipMemcpyAsync(w.prefix, prefix.data(), sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice,
                                   s));
            MPR_HIP(hipStreamSynchronize(s));
        }
    }
    if (tile_h_used_out) *tile_h_used_out = variant ? 32 : 16;

    // ---- the sweep loop: a graph of n_f sweeps replayed until every scene is done ----
    const int per_graph = c.stop_mode == MPR_STOP_AUTO ? std::max(1, c.n_f) : 5;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = capture_stream();
    if (cs) {
        hipGraph_t graph = nullptr;
        bool okc = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        for (int i = 0; okc && i < per_graph; ++i)
            okc = mpr::launch_batch_step(b, variant, variant, grid, max_hw_blocks, cs) == hipSuccess;
        hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (okc && ec == hipSuccess && graph) {
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
    int active = n_scenes;
    while (active > 0 && done < total_max + 1) {
        if (exec) {
            MPR_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int i = 0; i < per_graph; ++i) MPR_HIP(mpr::launch_batch_step(b, variant, variant, grid, max_hw_blocks, s));
        }
        done += per_graph;
        mpr::BatchCtl hc;
        MPR_HIP(hipMemcpyAsync(&hc, w.ctl, sizeof hc, hipMemcpyDeviceToHost, s));
        MPR_HIP(hipStreamSynchronize(s));
        active = hc.n_active;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (active > 0) return fail(MPR_ERR_HIP, "batched simulation did not finish within %d sweeps", total_max);

    // ---- results: final buffers into the callers' state, k* per scene ----
    MPR_HIP(hipMemcpyAsync(runs.data(), w.runs, sizeof(mpr::BatchRun) * n_scenes, hipMemcpyDeviceToHost, s));
    MPR_HIP(hipStreamSynchronize(s));
    bool all_converged = true;
    for (int i = 0; i < n_scenes; ++i) {
        const int total = runs[i].k_star + c.n_samp;
        if (total & 1)
            MPR_HIP(hipMemcpyAsync(scenes[i].state, w.alt[i], sizeof(float) * (size_t)(R * hs[i].HW),
                                   hipMemcpyDeviceToDevice, s));
        if (sweeps_done_out) sweeps_done_out[i] = runs[i].k_star;
        if (converged_out) converged_out[i] = runs[i].converged != 0 ? 1 : 0;
        all_converged &= runs[i].converged != 0;
    }
    if (!all_converged) return fail(MPR_WARN_NOT_CONVERGED, "some scenes reached n_max without equilibrium");
    return ok();
}

// The batch runs on the realization-lane sweep when the realizations fill a wave's lanes (64 or more; or when the
// lane sweep is asked for), every side is below 65536 and all scenes find their temperatures the same way (one
// persistent kernel instance serves them all); otherwise on the persistent tile-kernel batch.  Both give every
// scene its single-scene results.
static bool batch_on_lanes(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config& c)
{
    if (c.sweep_kernel == MPR_SWEEP_TILES) return false;
    if (c.sweep_kernel != MPR_SWEEP_LANES && c.n_real < 64) return false;
    const int tm = mpr::rl_tm(scenes[0].lb_w);
    for (int i = 0; i < n_scenes; ++i)
        if (scenes[i].H >= 65536 || scenes[i].W >= 65536 || mpr::rl_tm(scenes[i].lb_w) != tm) return false;
    return true;
}

static size_t batched_lanes_ws(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg)
{
    Carve c{nullptr, 0, 0};
    return batchl_ws(c, scenes, n_scenes, cfg, nullptr);
}

// All scenes in one persistent lane-sweep launch per sweep (k_batchl_sweep), chunks of sweeps replayed as a graph.
static mpr_status batched_lanes(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg,
                                int32_t* sweeps_done_out, int32_t* converged_out, void* workspace, size_t ws_bytes,
                                void* stream)
{
    const mpr_sim_config& c = *cfg;
    hipStream_t s = S(stream);
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    BatchLaneWs w;
    batchl_ws(cv, scenes, n_scenes, cfg, &w);
    const int R = c.n_real;
    const uint32_t key0 = (uint32_t)(c.seed & 0xffffffffu), key1 = (uint32_t)(c.seed >> 32);
    bool any_energy_out = false;
    for (int i = 0; i < n_scenes; ++i) any_energy_out |= scenes[i].energy != nullptr;
    const bool energy = c.stop_mode == MPR_STOP_AUTO || any_energy_out;

    std::vector<mpr::BatchLaneScene> hs(n_scenes);
    std::vector<int64_t> work(n_scenes);
    // fork: the setup streams start after the work the caller queued on its stream (the scenes' inputs)
    SetupFork fork;
    hipStream_t lane_stream[kSetupLanes] = {s};
    MPR_HIP(hipMemsetAsync(w.gaps, 0, sizeof(int64_t) * (size_t)n_scenes, s));
    MPR_HIP(hipEventCreateWithFlags(&fork.ev[0], hipEventDisableTiming));
    MPR_HIP(hipEventRecord(fork.ev[0], s));
    for (int j = 1; j < kSetupLanes; ++j) {
        lane_stream[j] = setup_stream(j - 1);
        if (!lane_stream[j]) return fail(MPR_ERR_HIP, "could not create a setup stream");
        MPR_HIP(hipStreamWaitEvent(lane_stream[j], fork.ev[0], 0));
    }
    for (int i = 0; i < n_scenes; ++i) {
        const mpr_scene& sc = scenes[i];
        const int lane = i % kSetupLanes;
        hipStream_t ss = lane_stream[lane];
        mpr::StatsGeom g = mpr::stats_geom(sc.H, sc.W, sc.lb_h, sc.lb_w);
        if (c.init_mode == MPR_INIT_BLOCK_MEAN) {
            const StatsWs& st = w.st[lane];
            MPR_HIP(mpr::launch_block_stats(sc.t, sc.mask, g, 2.0 * mpr::kPi * (double)c.q, (double)c.J, st.pS,
                                            st.pN, st.pTs, st.pNo, nullptr, nullptr, w.Ts[lane], w.No[lane], ss));
            MPR_HIP(mpr::launch_global_mean(w.Ts[lane], w.No[lane], g.B(), w.gmean[lane], ss));
        }
        mpr::InitArgs ia;
        ia.state = sc.state;
        ia.state2 = nullptr;
        ia.t = sc.t;
        ia.mask = sc.mask;
        ia.Ts = w.Ts[lane];
        ia.No = w.No[lane];
        ia.gmean = w.gmean[lane];
        ia.H = sc.H;
        ia.W = sc.W;
        ia.lb_h = sc.lb_h;
        ia.lb_w = sc.lb_w;
        ia.nbx = g.nbx;
        ia.R = R;
        ia.real_offset = (uint32_t)c.real_offset;
        ia.scene = sc.scene_id;
        ia.key0 = key0;
        ia.key1 = key1;
        ia.mode = c.init_mode;
        // (the start goes through the [R][H][W] state here: with many small scenes the per-site kernels of the
        // plane layout keep more of the device busy than the lane-layout start, which is written for large grids)
        MPR_HIP(mpr::launch_init(ia, ss));
        MPR_HIP(mpr::launch_tpairs(sc.T_blocks, g.B(), c.J, mpr::kDeltaE * c.J, w.tp[i], ss));
        const int64_t HW = sc.H * sc.W;
        const int64_t nbonds = sc.H * (sc.W - 1) + sc.W * (sc.H - 1);
        const double inv_norm = nbonds > 0 ? 1.0 / (double)nbonds : 0.0;
        if (energy) {
            const int nfull = mpr::energy_full_parts(sc.H, sc.W);
            MPR_HIP(start_energy_partials(sc.state, sc.H, sc.W, R, c, w.epart[i], nfull, ss));
            MPR_HIP(mpr::launch_energy_reduce(w.epart[i], nfull, R, inv_norm, w.e_real[i], w.series[i], ss));
        }
        if (c.n_samp == 0) MPR_HIP(hipMemsetAsync(sc.acc, 0, sizeof(double) * (size_t)HW, ss));
        MPR_HIP(mpr::launch_rl_cells(sc.mask, sc.H, sc.W, w.cells[i], ss));
        MPR_HIP(mpr::launch_count_gaps(sc.mask, HW, w.gaps + i, ss));
        MPR_HIP(mpr::launch_rl_to_lanes(sc.state, HW, R, w.buf0[i], w.buf1[i], ss));
        const mpr::RlGeom rg = mpr::rl_geometry_full(sc.H, sc.W, R);
        mpr::BatchLaneScene& d = hs[i];
        mpr::RlArgs& ra = d.a;
        ra = mpr::RlArgs{};
        ra.H = (int)sc.H;
        ra.W = (int)sc.W;
        ra.R = R;
        ra.Rp = rg.Rp;
        ra.Mw = (int)((sc.W + 3) / 4);
        ra.nbands = rg.nbands;
        ra.nseg = rg.nseg;
        ra.seg_rows = rg.seg_rows;
        ra.n_items = rg.n_items;
        ra.tb_h = sc.lb_h;
        ra.tb_w = sc.lb_w;
        ra.nbx_t = (int)((sc.W + sc.lb_w - 1) / sc.lb_w);
        ra.nby_t = (int)((sc.H + sc.lb_h - 1) / sc.lb_h);
        ra.tb_w_inv = sc.lb_w > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)sc.lb_w - 1) / (uint64_t)sc.lb_w) : 0u;
        ra.sweep = 0u;
        ra.real_offset = (uint32_t)c.real_offset;
        ra.scene = sc.scene_id;
        ra.key0 = key0;
        ra.key1 = key1;
        ra.q = c.q;
        ra.J = c.J;
        ra.delta_e = mpr::kDeltaE * c.J;
        ra.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
        ra.Jd = (double)c.J;
        d.cells = w.cells[i];
        d.tb = w.tp[i];
        d.buf[0] = w.buf0[i];
        d.buf[1] = w.buf1[i];
        d.acc = sc.acc;
        d.mask = sc.mask;
        d.epart = w.epart[i];
        d.e_real = w.e_real[i];
        d.series = w.series[i];
        d.HW = HW;
        d.work = rg.n_items;
        d.nparts = rg.nbands * rg.nseg;
        d.inv_norm = inv_norm;
        work[i] = rg.n_items;
    }
    // join: the caller's stream waits for the starts queued on the setup streams
    for (int j = 1; j < kSetupLanes; ++j) {
        MPR_HIP(hipEventCreateWithFlags(&fork.ev[j], hipEventDisableTiming));
        MPR_HIP(hipEventRecord(fork.ev[j], lane_stream[j]));
        MPR_HIP(hipStreamWaitEvent(s, fork.ev[j], 0));
    }
    // largest scenes first
    std::vector<int> order(n_scenes);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<int64_t> prefix(n_scenes + 1, 0);
    for (int i = 0; i < n_scenes; ++i) prefix[i + 1] = prefix[i] + work[order[i]];
    std::vector<mpr::BatchRun> runs(n_scenes, mpr::BatchRun{0, 0, 0, 1});
    mpr::BatchLaneCtl ctl{};
    ctl.n_active = n_scenes;
    MPR_HIP(hipMemcpyAsync(w.scenes, hs.data(), sizeof(mpr::BatchLaneScene) * n_scenes, hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.runs, runs.data(), sizeof(mpr::BatchRun) * n_scenes, hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.order, order.data(), sizeof(int) * n_scenes, hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.prefix, prefix.data(), sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice, s));
    MPR_HIP(hipMemcpyAsync(w.ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, s));
    MPR_HIP(hipStreamSynchronize(s));     // the host arrays above must outlive the copies

    mpr::BatchLaneDev b;
    b.scenes = w.scenes;
    b.runs = w.runs;
    b.order = w.order;
    b.prefix = w.prefix;
    b.ctl = w.ctl;
    b.n = n_scenes;
    b.tm = mpr::rl_tm(scenes[0].lb_w);
    b.gaps = w.gaps;
    b.cfg.R = R;
    b.cfg.real_offset = (uint32_t)c.real_offset;
    b.cfg.key0 = key0;
    b.cfg.key1 = key1;
    b.cfg.q = c.q;
    b.cfg.J = c.J;
    b.cfg.delta_e = mpr::kDeltaE * c.J;
    b.cfg.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
    b.cfg.Jd = (double)c.J;
    b.cfg.energy = energy ? 1 : 0;
    b.cfg.stop_mode = c.stop_mode;
    b.cfg.n_fit = c.n_fit;
    b.cfg.n_f = c.n_f;
    b.cfg.n_max = c.n_max;
    b.cfg.n_eq = c.n_eq;
    b.cfg.n_samp = c.n_samp;
    int acc_blocks = 1;
    for (int i = 0; i < n_scenes; ++i)
        acc_blocks = std::max<int>(acc_blocks, (int)std::min<int64_t>((hs[i].HW + 255) / 256, 1024));
    const int grid = 256 * 4 * mpr::kRlWaves;          // one wave per workgroup, every wave slot of the device
    const int32_t cap = c.stop_mode == MPR_STOP_AUTO ? c.n_max : c.n_eq;
    const int32_t total_max = cap + c.n_samp;
    MPR_HIP(mpr::launch_batchl_bounds(b, s));         // the XCD split of the first sweep's work list

    // the sweep loop: a graph of n_f sweeps replayed until every scene is done
    const int per_graph = c.stop_mode == MPR_STOP_AUTO ? std::max(1, c.n_f) : 5;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = capture_stream();
    if (cs) {
        hipGraph_t graph = nullptr;
        bool okc = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        for (int i = 0; okc && i < per_graph; ++i) okc = mpr::launch_batchl_step(b, grid, acc_blocks, cs) == hipSuccess;
        hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (okc && ec == hipSuccess && graph) {
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
    int active = n_scenes, done = 0;
    while (active > 0 && done < total_max + 1) {
        if (exec) {
            MPR_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int i = 0; i < per_graph; ++i) MPR_HIP(mpr::launch_batchl_step(b, grid, acc_blocks, s));
        }
        done += per_graph;
        mpr::BatchLaneCtl hc;
        MPR_HIP(hipMemcpyAsync(&hc, w.ctl, sizeof hc, hipMemcpyDeviceToHost, s));
        MPR_HIP(hipStreamSynchronize(s));
        active = hc.n_active;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (active > 0) return fail(MPR_ERR_HIP, "batched simulation did not finish within %d sweeps", total_max);

    // results: the final lane buffers into the callers' state, k* per scene
    MPR_HIP(hipMemcpyAsync(runs.data(), w.runs, sizeof(mpr::BatchRun) * n_scenes, hipMemcpyDeviceToHost, s));
    MPR_HIP(hipStreamSynchronize(s));
    bool all_converged = true;
    for (int i = 0; i < n_scenes; ++i) {
        const int total = runs[i].k_star + c.n_samp;
        MPR_HIP(mpr::launch_rl_from_lanes(hs[i].buf[total & 1], hs[i].HW, R, scenes[i].state, s));
        if (sweeps_done_out) sweeps_done_out[i] = runs[i].k_star;
        if (converged_out) converged_out[i] = runs[i].converged != 0 ? 1 : 0;
        all_converged &= runs[i].converged != 0;
    }
    if (!all_converged) return fail(MPR_WARN_NOT_CONVERGED, "some scenes reached n_max without equilibrium");
    return ok();
}

size_t mpr_simulate_batched_workspace_bytes(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg)
{
    if (!scenes || n_scenes < 1 || !cfg) return 0;
    for (int i = 0; i < n_scenes; ++i)
        if (scenes[i].H < 1 || scenes[i].W < 1 || scenes[i].lb_h < 1 || scenes[i].lb_w < 1) return 0;
    return batch_on_lanes(scenes, n_scenes, *cfg) ? batched_lanes_ws(scenes, n_scenes, cfg)
                                                  : batched_tiles_ws(scenes, n_scenes, cfg);
}

mpr_status mpr_simulate_batched(const mpr_scene* scenes, int32_t n_scenes, const mpr_sim_config* cfg, int32_t tile_h,
                                int32_t* sweeps_done_out, int32_t* converged_out, int32_t* tile_h_used_out,
                                void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_batched(scenes, n_scenes, cfg, tile_h);
    if (st != MPR_OK) return st;
    st = check_ws(workspace, ws_bytes, mpr_simulate_batched_workspace_bytes(scenes, n_scenes, cfg));
    if (st != MPR_OK) return st;
    if (batch_on_lanes(scenes, n_scenes, *cfg)) {
        if (tile_h_used_out) *tile_h_used_out = 0;
        return batched_lanes(scenes, n_scenes, cfg, sweeps_done_out, converged_out, workspace, ws_bytes, stream);
    }
    return batched_tiles(scenes, n_scenes, cfg, tile_h, sweeps_done_out, converged_out, tile_h_used_out, workspace,
                         ws_bytes, stream);
}

// ---- instruction-rate probe ----
size_t mpr_probe_instruction_rates_workspace_bytes(void) { return mpr::probe_out_bytes(); }

mpr_status mpr_probe_instruction_rates(double* cost_out, int32_t n_out, double* add_ns_out, void* workspace,
                                       size_t ws_bytes, void* stream)
{
    if (!cost_out || n_out < mpr::kProbeCount) return fail(MPR_ERR_INVALID_ARG, "cost_out needs %d entries", mpr::kProbeCount);
    mpr_status st = check_ws(workspace, ws_bytes, mpr::probe_out_bytes());
    if (st != MPR_OK) return st;
    double ns[mpr::kProbeCount];
    MPR_HIP(mpr::time_probes(static_cast<uint32_t*>(workspace), S(stream), ns));
    for (int i = 0; i < mpr::kProbeCount; ++i) cost_out[i] = ns[i] / ns[0];
    if (add_ns_out) *add_ns_out = ns[0] / mpr::probe_wave_instructions();
    return ok();
}

// ---- Sec. 2.2.3: site-specific temperatures ----
size_t mpr_sst_temperatures_workspace_bytes(int64_t H, int64_t W)
{
    if (H < 1 || W < 1) return 0;
    Carve c{nullptr, 0, 0};
    (void)c.take<double>(H * W);
    (void)c.take<double>(H * W);
    return c.used;
}

mpr_status mpr_sst_temperatures(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t r_s,
                                int32_t n_s, float* T_site_out, void* workspace, size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid(H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks(H, W, lb_h, lb_w)) != MPR_OK) return st;
    if (!T_blocks || !T_site_out) return fail(MPR_ERR_INVALID_ARG, "mpr_sst_temperatures: NULL pointer");
    if (r_s < 0 || r_s > 64 || n_s < 0 || n_s > 1000) return fail(MPR_ERR_INVALID_ARG, "need 0 <= r_s <= 64, 0 <= n_s <= 1000");
    st = check_ws(workspace, ws_bytes, mpr_sst_temperatures_workspace_bytes(H, W));
    if (st != MPR_OK) return st;
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    double* a = cv.take<double>(H * W);
    double* b = cv.take<double>(H * W);
    MPR_HIP(mpr::launch_sst(T_blocks, H, W, lb_h, lb_w, r_s, n_s, a, b, T_site_out, S(stream)));
    return ok();
}

}  // extern "C"

// ---- the 3D lattice (the extension to three dimensions of Sec. 4) ----
namespace {

mpr_status check_grid3(int64_t D, int64_t H, int64_t W)
{
    if (D < 1 || H < 1 || W < 1 || D > 65535 || H > 65535 || W > 65535)
        return fail(MPR_ERR_SHAPE, "3D grid %lld x %lld x %lld: sides must be in 1 .. 65535", (long long)D, (long long)H,
                    (long long)W);
    if ((D * H) * ((W + 3) / 4) >= ((int64_t)1 << 32))
        return fail(MPR_ERR_SHAPE, "3D grid too large for the 32-bit random-stream counter");
    return MPR_OK;
}

mpr_status check_blocks3(int32_t lb_d, int32_t lb_h, int32_t lb_w)
{
    if (lb_d < 1 || lb_h < 1 || lb_w < 1) return fail(MPR_ERR_SHAPE, "3D blocks: every side must be >= 1");
    return MPR_OK;
}

struct Cal3Ws {
    double *S, *Ts;
    int *N, *No;
    unsigned* n_have;
};
size_t cal3_ws(Carve& c, int64_t B, Cal3Ws* w)
{
    Cal3Ws x;
    x.S = c.take<double>(B);
    x.Ts = c.take<double>(B);
    x.N = c.take<int>(B);
    x.No = c.take<int>(B);
    x.n_have = c.take<unsigned>(1);
    if (w) *w = x;
    return c.used;
}

struct Sim3Ws {
    Cal3Ws st;
    float* gmean;
    mpr::TBand* tp;
    uint32_t* cells;
    float* lanes;        // [G][n][64]
    long long* epart;    // [R][max(nparts, energy3 parts)]
    double* e_real;
    double* series;
    double* hist;        // per-chain stop: [cap + 1][R]
};
struct Geom3 {
    int nbands, nzseg, zseg, Rp;
    int64_t n_all, B;
    int nparts;
};
Geom3 geom3(int64_t D, int64_t H, int64_t W, int32_t lb_d, int32_t lb_h, int32_t lb_w, int R)
{
    Geom3 g;
    g.nbands = (int)((W + mpr::kB3 - 1) / mpr::kB3);
    g.zseg = mpr::kZSeg3;
    g.nzseg = (int)((D + g.zseg - 1) / g.zseg);
    g.Rp = (R + 63) / 64 * 64;
    g.n_all = D * H * W;
    g.B = mpr::lat3_blocks(D, H, W, lb_d, lb_h, lb_w);
    g.nparts = (int)(H * g.nbands * g.nzseg);
    return g;
}
size_t sim3_ws(Carve& c, int64_t D, int64_t H, int64_t W, int32_t lb_d, int32_t lb_h, int32_t lb_w,
               const mpr_sim_config* cfg, Sim3Ws* w)
{
    const int R = cfg->n_real > 0 ? cfg->n_real : 1;
    const Geom3 g = geom3(D, H, W, lb_d, lb_h, lb_w, R);
    Sim3Ws x;
    cal3_ws(c, g.B, &x.st);
    x.gmean = c.take<float>(1);
    x.tp = c.take<mpr::TBand>(g.B);
    x.cells = c.take<uint32_t>(D * H * g.nbands);
    x.lanes = c.take<float>((int64_t)g.Rp * g.n_all);
    const int64_t np = std::max<int64_t>(g.nparts, mpr::energy3_parts(D, H, W));
    x.epart = c.take<long long>(np * R);
    x.e_real = c.take<double>(R);
    const int64_t cap = auto_stop(cfg->stop_mode) ? cfg->n_max : cfg->n_eq;
    x.series = c.take<double>((cap > 0 ? cap : 0) + 1);
    x.hist = cfg->stop_mode == MPR_STOP_AUTO_CHAIN ? c.take<double>(((cap > 0 ? cap : 0) + 1) * R) : nullptr;
    if (w) *w = x;
    return c.used;
}

}  // namespace

extern "C" {

size_t mpr_calibrate3d_workspace_bytes(int64_t D, int64_t H, int64_t W, int32_t lb_d, int32_t lb_h, int32_t lb_w)
{
    if (D < 1 || H < 1 || W < 1 || lb_d < 1 || lb_h < 1 || lb_w < 1) return 0;
    Carve c{nullptr, 0, 0};
    return cal3_ws(c, mpr::lat3_blocks(D, H, W, lb_d, lb_h, lb_w), nullptr);
}

mpr_status mpr_calibrate_temperature3d(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W,
                                       int32_t lb_d, int32_t lb_h, int32_t lb_w, float q, float J,
                                       const double* curve_T, const double* curve_e, int32_t n_curve, float* T_out,
                                       double* e_blocks_out, int32_t* nbonds_out, void* workspace, size_t ws_bytes,
                                       void* stream)
{
    mpr_status st = check_grid3(D, H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks3(lb_d, lb_h, lb_w)) != MPR_OK) return st;
    if (!t || !mask || !curve_T || !curve_e || !T_out)
        return fail(MPR_ERR_INVALID_ARG, "mpr_calibrate_temperature3d: NULL pointer");
    if (n_curve < 1) return fail(MPR_ERR_INVALID_ARG, "n_curve must be >= 1");
    if (!(q > 0.0f && q <= 0.5f) || !(J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    st = check_ws(workspace, ws_bytes, mpr_calibrate3d_workspace_bytes(D, H, W, lb_d, lb_h, lb_w));
    if (st != MPR_OK) return st;
    const int64_t B = mpr::lat3_blocks(D, H, W, lb_d, lb_h, lb_w);
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    Cal3Ws w;
    cal3_ws(c, B, &w);
    hipStream_t s = S(stream);
    MPR_HIP(mpr::launch_block_stats3(t, mask, D, H, W, lb_d, lb_h, lb_w, 2.0 * mpr::kPi * (double)q, (double)J, w.S,
                                     w.N, w.Ts, w.No, s));
    MPR_HIP(mpr::launch_calibrate(w.S, w.N, B, (double)J, curve_T, curve_e, n_curve, T_out, e_blocks_out, nbonds_out,
                                  w.n_have, s));
    unsigned n_have = 0;
    MPR_HIP(hipMemcpyAsync(&n_have, w.n_have, sizeof n_have, hipMemcpyDeviceToHost, s));
    MPR_HIP(hipStreamSynchronize(s));
    if (n_have == 0)
        return fail(MPR_ERR_NO_SAMPLE_BONDS, "no pair of neighbouring samples: the temperature cannot be estimated");
    return ok();
}

size_t mpr_reference_curve3d_workspace_bytes(int32_t nT, int32_t L)
{
    if (nT < 1 || L < 2) return 0;
    Carve c{nullptr, 0, 0};
    c.take<float>((int64_t)nT * L * L * L);
    c.take<double>((int64_t)mpr::ref3_energy_parts(L) * nT);
    c.take<double>(nT);
    return c.used;
}

mpr_status mpr_reference_curve3d(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm, int32_t n_meas,
                                 uint64_t seed, double* e_out, void* workspace, size_t ws_bytes, void* stream)
{
    if (!(q > 0.0f && q <= 0.5f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2");
    if (nT < 1 || nT > 65535) return fail(MPR_ERR_INVALID_ARG, "nT must be in 1 .. 65535");
    if (L < 2 || L > 512 || (L & 1)) return fail(MPR_ERR_SHAPE, "L must be even and in 2 .. 512");
    if (n_therm < 0 || n_meas < 1) return fail(MPR_ERR_INVALID_ARG, "need n_therm >= 0 and n_meas >= 1");
    if (!T_grid || !e_out) return fail(MPR_ERR_INVALID_ARG, "mpr_reference_curve3d: NULL pointer");
    mpr_status st = check_ws(workspace, ws_bytes, mpr_reference_curve3d_workspace_bytes(nT, L));
    if (st != MPR_OK) return st;
    Carve c{static_cast<char*>(workspace), 0, ws_bytes};
    float* state = c.take<float>((int64_t)nT * L * L * L);
    const int nparts = mpr::ref3_energy_parts(L);
    double* part = c.take<double>((int64_t)nparts * nT);
    double* esum = c.take<double>(nT);
    hipStream_t s = S(stream);
    MPR_HIP(mpr::launch_ref_fill(state, (int64_t)nT * L * L * L, 0.5f, s));
    const uint32_t key0 = (uint32_t)(seed & 0xffffffffu), key1 = (uint32_t)(seed >> 32);
    const double two_pi_q = 2.0 * mpr::kPi * (double)q;
    const double inv_norm = 1.0 / (3.0 * (double)L * (double)L * (double)L);
    for (int32_t k = 1; k <= n_therm + n_meas; ++k) {
        for (int colour = 0; colour < 2; ++colour)
            MPR_HIP(mpr::launch_ref3_half(state, T_grid, nT, L, (uint32_t)k, colour, q, mpr::kDeltaE3, key0, key1,
                                          two_pi_q, s));
        if (k > n_therm) {
            MPR_HIP(mpr::launch_ref3_energy(state, L, nT, q, part, nparts, s));
            MPR_HIP(mpr::launch_ref_accumulate(part, nparts, nT, inv_norm, esum, k == n_therm + 1 ? 1 : 0, s));
        }
    }
    MPR_HIP(mpr::launch_ref_finish(esum, nT, (double)n_meas, e_out, s));
    return ok();
}

size_t mpr_simulate3d_workspace_bytes(int64_t D, int64_t H, int64_t W, int32_t lb_d, int32_t lb_h, int32_t lb_w,
                                      const mpr_sim_config* cfg)
{
    if (!cfg || D < 1 || H < 1 || W < 1 || lb_d < 1 || lb_h < 1 || lb_w < 1) return 0;
    Carve c{nullptr, 0, 0};
    return sim3_ws(c, D, H, W, lb_d, lb_h, lb_w, cfg, nullptr);
}

mpr_status mpr_simulate3d(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W, const float* T_blocks,
                          int32_t lb_d, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, float* state,
                          double* acc_out, double* energy_out, int32_t* sweeps_done_out, void* workspace,
                          size_t ws_bytes, void* stream)
{
    mpr_status st = check_grid3(D, H, W);
    if (st != MPR_OK) return st;
    if ((st = check_blocks3(lb_d, lb_h, lb_w)) != MPR_OK) return st;
    if (!cfg) return fail(MPR_ERR_INVALID_ARG, "cfg is NULL");
    if (!t || !mask || !T_blocks || !state || !acc_out) return fail(MPR_ERR_INVALID_ARG, "mpr_simulate3d: NULL pointer");
    const mpr_sim_config& c = *cfg;
    if ((st = check_sim_config(c)) != MPR_OK) return st;
    if (c.init_mode != MPR_INIT_RANDOM && c.init_mode != MPR_INIT_BLOCK_MEAN)
        return fail(MPR_ERR_INVALID_ARG, "unknown init_mode %d", c.init_mode);
    if (c.stop_mode != MPR_STOP_FIXED && !auto_stop(c.stop_mode))
        return fail(MPR_ERR_INVALID_ARG, "unknown stop_mode %d", c.stop_mode);
    if (c.n_samp < 0) return fail(MPR_ERR_INVALID_ARG, "n_samp must be >= 0");
    if (c.stop_mode == MPR_STOP_FIXED && c.n_eq < 0) return fail(MPR_ERR_INVALID_ARG, "n_eq must be >= 0");
    if (auto_stop(c.stop_mode) && (c.n_fit < 2 || c.n_f < 1 || c.n_max < 1))
        return fail(MPR_ERR_INVALID_ARG, "AUTO needs n_fit >= 2, n_f >= 1, n_max >= 1");
    if (c.t_mode != MPR_T_BLOCK || c.order != MPR_ORDER_SC || c.coupling != MPR_COUPLING_ISOTROPIC)
        return fail(MPR_ERR_INVALID_ARG, "the 3D lattice runs block temperatures, the single checkerboard and one "
                                         "coupling");
    st = check_ws(workspace, ws_bytes, mpr_simulate3d_workspace_bytes(D, H, W, lb_d, lb_h, lb_w, cfg));
    if (st != MPR_OK) return st;
    hipStream_t s = S(stream);
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    Sim3Ws w;
    sim3_ws(cv, D, H, W, lb_d, lb_h, lb_w, cfg, &w);
    const int R = c.n_real;
    const Geom3 g = geom3(D, H, W, lb_d, lb_h, lb_w, R);
    const uint32_t key0 = (uint32_t)(c.seed & 0xffffffffu), key1 = (uint32_t)(c.seed >> 32);
    const int nbx = (int)((W + lb_w - 1) / lb_w), nby = (int)((H + lb_h - 1) / lb_h);

    if (c.init_mode == MPR_INIT_BLOCK_MEAN) {
        MPR_HIP(mpr::launch_block_stats3(t, mask, D, H, W, lb_d, lb_h, lb_w, 2.0 * mpr::kPi * (double)c.q, (double)c.J,
                                         w.st.S, w.st.N, w.st.Ts, w.st.No, s));
        MPR_HIP(mpr::launch_global_mean(w.st.Ts, w.st.No, g.B, w.gmean, s));
    }
    mpr::Init3Args ia;
    ia.state = state;
    ia.t = t;
    ia.mask = mask;
    ia.Ts = w.st.Ts;
    ia.No = w.st.No;
    ia.gmean = w.gmean;
    ia.D = D;
    ia.H = H;
    ia.W = W;
    ia.lb_d = lb_d;
    ia.lb_h = lb_h;
    ia.lb_w = lb_w;
    ia.nbx = nbx;
    ia.nby = nby;
    ia.R = R;
    ia.real_offset = (uint32_t)c.real_offset;
    ia.scene = c.scene_id;
    ia.key0 = key0;
    ia.key1 = key1;
    ia.mode = c.init_mode;
    MPR_HIP(mpr::launch_init3(ia, s));
    MPR_HIP(mpr::launch_tpairs(T_blocks, g.B, c.J, mpr::kDeltaE3 * c.J, w.tp, s));
    const int64_t nbonds = (W - 1) * H * D + W * (H - 1) * D + W * H * (D - 1);
    const double inv_norm = nbonds > 0 ? 1.0 / (double)nbonds : 0.0;
    const bool need_energy = auto_stop(c.stop_mode) || energy_out != nullptr;
    if (need_energy) {
        const int nfull = mpr::energy3_parts(D, H, W);
        MPR_HIP(mpr::launch_energy3_full(state, D, H, W, R, c.q, w.epart, nfull, s));
        MPR_HIP(mpr::launch_energy_reduce(w.epart, nfull, R, inv_norm, w.e_real, w.series, s));
    }
    MPR_HIP(mpr::launch_cells3(mask, D, H, W, g.nbands, w.cells, s));
    MPR_HIP(mpr::launch_rl_to_lanes(state, g.n_all, R, w.lanes, nullptr, s));

    mpr::Lat3Args a{};
    a.D = (int)D;
    a.H = (int)H;
    a.W = (int)W;
    a.R = R;
    a.Rp = g.Rp;
    a.Mw = (int)((W + 3) / 4);
    a.nbands = g.nbands;
    a.nzseg = g.nzseg;
    a.zseg = g.zseg;
    a.lb_d = lb_d;
    a.lb_h = lb_h;
    a.lb_w = lb_w;
    a.nbx = nbx;
    a.nby = nby;
    a.lbw_inv = lb_w > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)lb_w - 1) / (uint64_t)lb_w) : 0u;
    a.real_offset = (uint32_t)c.real_offset;
    a.scene = c.scene_id;
    a.key0 = key0;
    a.key1 = key1;
    a.q = c.q;
    a.J = c.J;
    a.delta_e = mpr::kDeltaE3 * c.J;
    a.two_pi_q = 2.0 * mpr::kPi * (double)c.q;
    a.Jd = (double)c.J;
    // one sweep: colour 0, then colour 1, each one launch over all rows (row tiles of kNW3 rows)
    a.nrows = (int)((H + mpr::kNW3 - 1) / mpr::kNW3);
    auto sweep = [&](uint32_t k, bool energy) -> hipError_t {
        a.sweep = k;
        for (int colour = 0; colour < 2; ++colour) {
            a.colour = colour;
            const hipError_t e = mpr::launch_sweep3(a, w.cells, w.tp, w.lanes,
                                                    energy && colour == 1 ? w.epart : nullptr, s);
            if (e != hipSuccess) return e;
        }
        if (energy) return mpr::launch_energy_reduce(w.epart, g.nparts, R, inv_norm, w.e_real, w.series + k, s);
        return hipSuccess;
    };

    const int32_t cap = auto_stop(c.stop_mode) ? c.n_max : c.n_eq;
    int32_t k = 0;
    bool converged = true;
    double e0 = 0.0;
    std::vector<double> window;
    const bool per_chain = c.stop_mode == MPR_STOP_AUTO_CHAIN;
    ChainStop chains;
    if (c.stop_mode == MPR_STOP_AUTO) {
        MPR_HIP(hipMemcpyAsync(&e0, w.series, sizeof(double), hipMemcpyDeviceToHost, s));
        window.resize((size_t)c.n_fit);
    }
    if (per_chain) {
        MPR_HIP(hipMemcpyAsync(w.hist, w.e_real, sizeof(double) * (size_t)R, hipMemcpyDeviceToDevice, s));
        MPR_HIP(chains.start(w.hist, R, c.n_fit, s));
    }
    while (k < cap) {
        ++k;
        MPR_HIP(sweep((uint32_t)k, need_energy));
        if (per_chain)
            MPR_HIP(hipMemcpyAsync(w.hist + (int64_t)k * R, w.e_real, sizeof(double) * (size_t)R,
                                   hipMemcpyDeviceToDevice, s));
        if (auto_stop(c.stop_mode)) {
            if (k >= c.n_fit + c.n_f && (k - c.n_fit) % c.n_f == 0) {
                bool done = false;
                if (per_chain) {
                    MPR_HIP(chains.check(w.hist, k, s, &done));
                } else {
                    MPR_HIP(hipMemcpyAsync(window.data(), w.series + (k - c.n_fit + 1), sizeof(double) * c.n_fit,
                                           hipMemcpyDeviceToHost, s));
                    MPR_HIP(hipStreamSynchronize(s));
                    done = equilibrium_reached(e0, window.data(), c.n_fit);
                }
                if (done) break;
            }
            if (k == c.n_max) converged = false;
        }
    }
    const int32_t k_star = k;
    if (c.n_samp == 0) MPR_HIP(hipMemsetAsync(acc_out, 0, sizeof(double) * (size_t)g.n_all, s));
    for (int32_t si = 1; si <= c.n_samp; ++si) {
        MPR_HIP(sweep((uint32_t)(k_star + si), false));
        MPR_HIP(mpr::launch_rl_accumulate(w.lanes, mask, g.n_all, R, si == 1 ? 1 : 0, acc_out, s));
    }
    MPR_HIP(mpr::launch_rl_from_lanes(w.lanes, g.n_all, R, state, s));
    if (energy_out && need_energy)
        MPR_HIP(hipMemcpyAsync(energy_out, w.series, sizeof(double) * (size_t)(k_star + 1), hipMemcpyDeviceToDevice, s));
    if (sweeps_done_out) *sweeps_done_out = k_star;
    if (!converged) return fail(MPR_WARN_NOT_CONVERGED, "equilibrium test not met after n_max = %d sweeps", c.n_max);
    return ok();
}

}  // extern "C"
