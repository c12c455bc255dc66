// Host implementation of the C ABI declared in include/mpr.h: argument checks, workspace carving, kernel
// sequencing on the caller's stream, and the equilibrium test of Sec. 3.4.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mpr.h"
#include "mpr_internal.hpp"

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

struct SimWs {
    StatsWs st;
    double* Ts;
    int* No;
    float* gmean;
    mpr::TPair* tp;
    double* epart;      // [R][max(ntiles, nfull)]
    double* e_real;     // [R]
    double* series;     // [cap + 1]
    float* alt;         // [R][H][W] second state buffer
};
size_t sim_ws(Carve& c, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, SimWs* w)
{
    mpr::StatsGeom g = mpr::stats_geom(H, W, lb_h, lb_w);
    SimWs x;
    stats_ws(c, g, &x.st);
    x.Ts = c.take<double>(g.B());
    x.No = c.take<int>(g.B());
    x.gmean = c.take<float>(1);
    x.tp = c.take<mpr::TPair>(g.B());
    const int64_t R = cfg->n_real > 0 ? cfg->n_real : 1;
    const int nt = fused_tiles(H, W, (int)R);
    const int nfull = mpr::energy_full_parts(H, W);
    x.epart = c.take<double>((int64_t)(nt > nfull ? nt : nfull) * R);
    x.e_real = c.take<double>(R);
    const int64_t cap = cfg->stop_mode == MPR_STOP_AUTO ? cfg->n_max : cfg->n_eq;
    x.series = c.take<double>((cap > 0 ? cap : 0) + 1);
    x.alt = c.take<float>(R * H * W);
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

mpr_status check_sim_config(const mpr_sim_config& c)
{
    if (!(c.q > 0.0f && c.q <= 0.5f) || !(c.J > 0.0f)) return fail(MPR_ERR_INVALID_ARG, "need 0 < q <= 1/2 and J > 0");
    if (c.n_real < 1 || c.n_real > 65535) return fail(MPR_ERR_INVALID_ARG, "n_real must be in 1 .. 65535");
    if (c.real_offset < 0) return fail(MPR_ERR_INVALID_ARG, "real_offset must be >= 0");
    if (c.scene_id >= (1u << 28)) return fail(MPR_ERR_INVALID_ARG, "scene_id must be < 2^28");
    return MPR_OK;
}

// Runs fused sweeps (one launch per sweep) alternating between two state buffers.
struct SweepRunner {
    mpr::SweepFusedArgs a;
    float* buf[2];
    int cur;
    double inv_norm;
    double* epart;     // [R][ntiles]
    double* e_real;    // [R]
    hipStream_t s;

    SweepRunner(float* state, float* alt, const uint8_t* mask, int64_t H, int64_t W, const mpr::TPair* tp,
                int32_t lb_h, int32_t lb_w, const mpr_sim_config& c, double* epart_, double* e_real_, hipStream_t s_)
    {
        int ntx, nty, rchunk, nchunks;
        mpr::fused_geometry(H, W, c.n_real, &ntx, &nty, &rchunk, &nchunks);
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
        inv_norm = nbonds > 0 ? 1.0 / ((double)c.J * (double)nbonds) : 0.0;
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
    mpr::fused_geometry(H, W, R, &ntx, &nty, &rc, &nc);
    return ntx * nty;
}

struct SweepWs {
    mpr::TPair* tp;
    double* epart;
    double* e_real;
};
size_t sweep_ws(Carve& c, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, const mpr_sim_config* cfg, SweepWs* w)
{
    SweepWs x;
    x.tp = c.take<mpr::TPair>(nblocks_of(H, W, lb_h, lb_w));
    const int64_t R = cfg->n_real > 0 ? cfg->n_real : 1;
    x.epart = c.take<double>((int64_t)fused_tiles(H, W, (int)R) * R);
    x.e_real = c.take<double>(R);
    if (w) *w = x;
    return c.used;
}

}  // namespace

extern "C" {

int32_t mpr_abi_version(void) { return 10000; }

const char* mpr_last_error(void) { return g_last_error.c_str(); }

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
    if (c.stop_mode != MPR_STOP_FIXED && c.stop_mode != MPR_STOP_AUTO)
        return fail(MPR_ERR_INVALID_ARG, "unknown stop_mode %d", c.stop_mode);
    if (c.n_samp < 0) return fail(MPR_ERR_INVALID_ARG, "n_samp must be >= 0");
    if (c.stop_mode == MPR_STOP_FIXED && c.n_eq < 0) return fail(MPR_ERR_INVALID_ARG, "n_eq must be >= 0");
    if (c.stop_mode == MPR_STOP_AUTO && (c.n_fit < 2 || c.n_f < 1 || c.n_max < 1))
        return fail(MPR_ERR_INVALID_ARG, "AUTO needs n_fit >= 2, n_f >= 1, n_max >= 1");
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
    MPR_HIP(mpr::launch_init(ia, s));
    MPR_HIP(mpr::launch_tpairs(T_blocks, B, w.tp, s));

    const bool need_energy = c.stop_mode == MPR_STOP_AUTO || energy_out != nullptr;
    SweepRunner runner(state, w.alt, mask, H, W, w.tp, lb_h, lb_w, c, w.epart, w.e_real, s);
    if (need_energy) {
        const int nfull = mpr::energy_full_parts(H, W);
        MPR_HIP(mpr::launch_energy_full(state, H, W, R, c.q, c.J, w.epart, nfull, s));
        MPR_HIP(mpr::launch_energy_reduce(w.epart, nfull, R, runner.inv_norm, w.e_real, w.series, s));
    }
    auto sweep = [&](uint32_t k, bool energy) -> hipError_t { return runner.run(k, energy ? w.series + k : nullptr); };

    const int32_t cap = c.stop_mode == MPR_STOP_AUTO ? c.n_max : c.n_eq;
    int32_t k = 0;
    bool converged = true;
    double e0 = 0.0;
    std::vector<double> window;
    if (c.stop_mode == MPR_STOP_AUTO) {
        MPR_HIP(hipMemcpyAsync(&e0, w.series, sizeof(double), hipMemcpyDeviceToHost, s));
        window.resize((size_t)c.n_fit);
    }
    while (k < cap) {
        ++k;
        MPR_HIP(sweep((uint32_t)k, need_energy));
        if (c.stop_mode == MPR_STOP_AUTO) {
            if (k >= c.n_fit + c.n_f && (k - c.n_fit) % c.n_f == 0) {
                MPR_HIP(hipMemcpyAsync(window.data(), w.series + (k - c.n_fit + 1), sizeof(double) * c.n_fit,
                                       hipMemcpyDeviceToHost, s));
                MPR_HIP(hipStreamSynchronize(s));
                if (equilibrium_reached(e0, window.data(), c.n_fit)) break;
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
        MPR_HIP(mpr::launch_accumulate(runner.current(), mask, HW, R, si == 1 ? 1 : 0, acc_out, s));
    }
    if (runner.current() != state) {
        MPR_HIP(hipMemcpyAsync(state, runner.current(), sizeof(float) * (size_t)(R * HW), hipMemcpyDeviceToDevice, s));
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
    if (k_first < 1 || n_sweeps < 0) return fail(MPR_ERR_INVALID_ARG, "need k_first >= 1 and n_sweeps >= 0");
    st = check_ws(workspace, ws_bytes, mpr_sweep_workspace_bytes(H, W, lb_h, lb_w, cfg));
    if (st != MPR_OK) return st;
    hipStream_t s = S(stream);
    Carve cv{static_cast<char*>(workspace), 0, ws_bytes};
    SweepWs w;
    sweep_ws(cv, H, W, lb_h, lb_w, cfg, &w);
    MPR_HIP(mpr::launch_tpairs(T_blocks, nblocks_of(H, W, lb_h, lb_w), w.tp, s));
    SweepRunner runner(state, state_alt, mask, H, W, w.tp, lb_h, lb_w, *cfg, w.epart, w.e_real, s);
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
