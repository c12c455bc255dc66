// Host sanitizer run of the library's host code (AddressSanitizer + UndefinedBehaviorSanitizer, host pass only):
// workspace-size queries over many shapes and configurations, the batched workspace rule over a few hundred scenes,
// and every argument check that must refuse a call before anything is enqueued.  No call here reaches the device.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mpr.h"

static int g_bad = 0;

static void expect(mpr_status got, mpr_status want, const char* what)
{
    if (got != want) {
        std::printf("FAIL %s: status %d, expected %d\n", what, (int)got, (int)want);
        g_bad = 1;
    } else if (want != MPR_OK && std::strlen(mpr_last_error()) == 0) {
        std::printf("FAIL %s: no error message\n", what);
        g_bad = 1;
    }
}

static mpr_sim_config base()
{
    mpr_sim_config c;
    std::memset(&c, 0, sizeof c);
    c.q = 0.5f;
    c.J = 1.0f;
    c.n_real = 64;
    c.init_mode = MPR_INIT_BLOCK_MEAN;
    c.stop_mode = MPR_STOP_AUTO;
    c.n_eq = 10;
    c.n_samp = 1;
    c.n_fit = 20;
    c.n_f = 5;
    c.n_max = 1000;
    c.seed = 7;
    return c;
}

int main()
{
    uint32_t s = 12345u;
    auto rnd = [&s](int lo, int hi) {
        s = s * 1664525u + 1013904223u;
        return lo + (int)((s >> 8) % (uint32_t)(hi - lo + 1));
    };
    // workspace queries over shapes and configurations
    size_t total = 0;
    for (int i = 0; i < 400; ++i) {
        const int64_t H = rnd(1, 3000), W = rnd(1, 3000);
        const int32_t lb_h = rnd(1, 70), lb_w = rnd(1, 70);
        mpr_sim_config c = base();
        c.n_real = rnd(1, 300);
        c.stop_mode = rnd(0, 1);
        c.t_mode = rnd(0, 1);
        c.sweep_kernel = rnd(0, 2);
        c.coupling = c.t_mode == MPR_T_BLOCK ? rnd(0, 1) : 0;
        total += mpr_simulate_workspace_bytes(H, W, lb_h, lb_w, &c);
        total += mpr_sweep_workspace_bytes(H, W, lb_h, lb_w, &c);
        total += mpr_calibrate_workspace_bytes(H, W, lb_h, lb_w);
        total += mpr_block_stats_workspace_bytes(H, W, lb_h, lb_w);
        total += mpr_map_workspace_bytes(H, W);
        total += mpr_sst_temperatures_workspace_bytes(H, W);
        total += mpr_block_energy_workspace_bytes(H, W, lb_h, lb_w, c.n_real);
        total += mpr_temperature_grad_workspace_bytes(H, W, c.n_real);
        total += mpr_validate_workspace_bytes(H * W);
    }
    total += mpr_reference_curve_workspace_bytes(121, 128);
    // the batched workspace rule over a batch with a spread of sizes (pointers are never dereferenced by the query)
    std::vector<mpr_scene> sc(300);
    static float f;
    static uint8_t u8;
    static double d;
    for (auto& x : sc) {
        std::memset(&x, 0, sizeof x);
        x.H = rnd(1, 2048);
        x.W = rnd(1, 2048);
        x.lb_h = x.lb_w = 16;
        x.t = &f;
        x.mask = &u8;
        x.T_blocks = &f;
        x.state = &f;
        x.acc = &d;
    }
    mpr_sim_config c = base();
    total += mpr_simulate_batched_workspace_bytes(sc.data(), (int32_t)sc.size(), &c);
    c.sweep_kernel = MPR_SWEEP_TILES;
    total += mpr_simulate_batched_workspace_bytes(sc.data(), (int32_t)sc.size(), &c);
    if (mpr_simulate_workspace_bytes(0, 5, 1, 1, &c) != 0 || mpr_simulate_workspace_bytes(5, 5, 1, 1, nullptr) != 0) {
        std::printf("FAIL workspace query of an invalid shape\n");
        g_bad = 1;
    }

    // refusals before anything is enqueued
    float* fp = &f;
    uint8_t* mp = &u8;
    double* dp = &d;
    char ws[64];
    expect(mpr_map_angles(fp, mp, 0, 4, fp, dp, ws, 64, nullptr), MPR_ERR_SHAPE, "map H = 0");
    expect(mpr_map_angles(nullptr, mp, 4, 4, fp, dp, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "map NULL z");
    expect(mpr_block_stats(fp, mp, 4, 4, 0, 2, 0.5f, 1.0f, dp, nullptr, nullptr, nullptr, ws, 64, nullptr),
           MPR_ERR_SHAPE, "stats lb_h = 0");
    expect(mpr_calibrate_temperature(fp, mp, 4, 4, 2, 2, 0.5f, 1.0f, dp, dp, 0, fp, nullptr, nullptr, ws, 64, nullptr),
           MPR_ERR_INVALID_ARG, "calibrate without curve points");
    mpr_sim_config bad = base();
    bad.q = 0.75f;
    int32_t k = 0;
    expect(mpr_simulate(fp, mp, 8, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "q > 1/2");
    bad = base();
    bad.n_real = 0;
    expect(mpr_simulate(fp, mp, 8, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "R = 0");
    bad = base();
    bad.init_mode = 9;
    expect(mpr_simulate(fp, mp, 8, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "init mode");
    bad = base();
    bad.n_fit = 1;
    expect(mpr_simulate(fp, mp, 8, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "n_fit");
    bad = base();
    bad.scene_id = 1u << 28;
    expect(mpr_simulate(fp, mp, 8, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "scene id");
    bad = base();
    bad.coupling = MPR_COUPLING_DIRECTIONAL;
    bad.sweep_kernel = MPR_SWEEP_TILES;
    expect(mpr_simulate(fp, mp, 8, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_INVALID_ARG,
           "directional on tiles");
    bad = base();
    bad.sweep_kernel = MPR_SWEEP_LANES;
    expect(mpr_simulate(fp, mp, 70000, 8, fp, 4, 4, &bad, fp, dp, nullptr, &k, ws, 64, nullptr), MPR_ERR_SHAPE,
           "lanes with a side of 70000");
    c = base();
    expect(mpr_simulate(fp, mp, 64, 64, fp, 16, 16, &c, fp, dp, nullptr, &k, ws, 64, nullptr),
           MPR_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    expect(mpr_simulate(fp, mp, 64, 64, fp, 16, 16, &c, fp, dp, nullptr, &k, nullptr, 0, nullptr), MPR_ERR_INVALID_ARG,
           "workspace NULL");
    expect(mpr_sweep(fp, fp, mp, 8, 8, fp, 4, 4, nullptr, 1, 1, nullptr, ws, 64, nullptr), MPR_ERR_INVALID_ARG,
           "sweep cfg NULL");
    expect(mpr_sst_temperatures(fp, 8, 8, 4, 4, -1, 2, fp, ws, 64, nullptr), MPR_ERR_INVALID_ARG, "sst r_s < 0");
    expect(mpr_simulate_batched(sc.data(), 0, &c, 0, nullptr, nullptr, nullptr, ws, 64, nullptr), MPR_ERR_INVALID_ARG,
           "batched without scenes");
    expect(mpr_simulate_batched(sc.data(), 4, &c, 24, nullptr, nullptr, nullptr, ws, 64, nullptr), MPR_ERR_INVALID_ARG,
           "batched tile_h 24");
    sc[2].state = nullptr;
    expect(mpr_simulate_batched(sc.data(), 4, &c, 0, nullptr, nullptr, nullptr, ws, 64, nullptr), MPR_ERR_INVALID_ARG,
           "batched NULL state");
    expect(mpr_temperature_grad(fp, dp, fp, mp, 8, 8, 1, 4, dp, fp, dp, ws, 64, nullptr), MPR_ERR_INVALID_ARG,
           "gradient with one realization");
    std::printf("host ABI sanitizer checks %s (workspace total %zu)\n", g_bad ? "FAILED" : "ok", total);
    return g_bad;
}
