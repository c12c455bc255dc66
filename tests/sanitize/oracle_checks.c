/* Host sanitizer run of the CPU oracle (AddressSanitizer + UndefinedBehaviorSanitizer): every oracle entry point on
 * small grids with ragged blocks, in every simulation mode, with edge shapes (1 x 1, 1 x W, H x 1).  The run ends
 * with status 0 only if no sanitizer report fired and the observed sites stayed fixed. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
void orc_site_uniforms(uint64_t seed, uint32_t scene, uint32_t tag, uint32_t sweep, uint32_t real, int64_t W,
                       int64_t x, int64_t y, double out[2]);
int orc_map_angles(const float* z, const uint8_t* mask, int64_t H, int64_t W, float* t, double range[2]);
void orc_block_stats(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, float q,
                     float J, double* S, int32_t* N, double* Tsum, int32_t* Nobs);
void orc_block_stats_directional(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h,
                                 int32_t lb_w, float q, float J, double* Sh, int32_t* Nh, double* Sv, int32_t* Nv);
int orc_calibrate_blocks(const double* S, const int32_t* N, int64_t B, float J, const double* curve_T,
                         const double* curve_e, int32_t n_curve, float* T_out);
double orc_energy(const float* s, int64_t H, int64_t W, float q, float J);
void orc_reference_curve(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm, int32_t n_meas,
                         uint64_t seed, double* e_out);
int32_t orc_simulate(const float* t, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks, int32_t lb_h,
                     int32_t lb_w, float q, float J, int32_t R, int32_t real_offset, int32_t init_mode,
                     int32_t stop_mode, int32_t n_eq, int32_t n_samp, int32_t n_fit, int32_t n_f, int32_t n_max,
                     uint64_t seed, uint32_t scene, int32_t t_per_site, int32_t order, int32_t directional,
                     float* state, double* acc, double* energy, int32_t* converged);
void orc_sst_temperatures(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t r_s,
                          int32_t n_s, float* T_site);
void orc_predict(const double* acc, const float* z, const uint8_t* mask, int64_t H, int64_t W, int64_t n_samples,
                 const double range[2], float* zhat);
void orc_validate(const float* zhat, const float* truth, const uint8_t* eval_mask, int64_t n, double out[2]);
void orc_block_energy(const float* s, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, float q,
                      float J, double* Hb);
void orc_temperature_grad(const float* states, const double* Hrb, const double* w, int64_t HW, int32_t R, int64_t B,
                          const float* T_blocks, double* dT);

static uint32_t lcg(uint32_t* s)
{
    *s = *s * 1664525u + 1013904223u;
    return *s >> 8;
}

static int run_case(int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, uint32_t seed)
{
    const int64_t HW = H * W;
    const int32_t R = 3, nmax = 40;
    const int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h, B = nbx * nby;
    float* z = malloc(sizeof(float) * HW);
    uint8_t* m = malloc(HW);
    float* t = malloc(sizeof(float) * HW);
    float* st = malloc(sizeof(float) * R * HW);
    double* acc = malloc(sizeof(double) * HW);
    double* en = malloc(sizeof(double) * (nmax + 1));
    float* zhat = malloc(sizeof(float) * HW);
    float* Tsite = malloc(sizeof(float) * HW);
    double *S = malloc(sizeof(double) * B), *Ts = malloc(sizeof(double) * B), *S2 = malloc(sizeof(double) * B);
    int32_t *N = malloc(sizeof(int32_t) * B), *No = malloc(sizeof(int32_t) * B), *N2 = malloc(sizeof(int32_t) * B);
    float* T = malloc(sizeof(float) * 2 * B);
    double* Hb = malloc(sizeof(double) * R * B);
    double* w = malloc(sizeof(double) * HW);
    double* dT = malloc(sizeof(double) * B);
    int bad = 0;
    for (int64_t n = 0; n < HW; ++n) {
        z[n] = (float)(lcg(&seed) % 1000) * 0.01f;
        m[n] = (uint8_t)(lcg(&seed) % 10 < 6);
        w[n] = m[n] ? 0.0 : 1.0;
    }
    m[0] = 1;
    double rng[2];
    if (orc_map_angles(z, m, H, W, t, rng) != 0) return 1;
    orc_block_stats(t, m, H, W, lb_h, lb_w, 0.5f, 1.0f, S, N, Ts, No);
    orc_block_stats_directional(t, m, H, W, lb_h, lb_w, 0.5f, 1.0f, S, N, S2, N2);
    for (int64_t b = 0; b < B; ++b) {
        T[b] = 0.05f + 0.01f * (float)(b % 7);
        T[B + b] = 0.08f + 0.02f * (float)(b % 5);
    }
    T[0] = 0.0f;
    orc_sst_temperatures(T, H, W, lb_h, lb_w, 1, 3, Tsite);
    for (int mode = 0; mode < 6; ++mode) {
        int32_t conv = 0;
        const int per_site = mode == 2, order = mode == 3, directional = mode == 4;
        const int32_t k = orc_simulate(t, m, H, W, per_site ? Tsite : T, lb_h, lb_w, 0.5f, 1.0f, R, 5, mode & 1,
                                       mode >= 5 ? 1 : 0, 7, 2, 4, 2, nmax, 0x1234567890ull + (uint64_t)mode, 9u,
                                       per_site, order, directional, st, acc, en, &conv);
        if (k < 0 || k > nmax) bad = 1;
        for (int32_t r = 0; r < R; ++r)
            for (int64_t n = 0; n < HW; ++n)
                if (m[n] && st[r * HW + n] != t[n]) bad = 1;
        orc_predict(acc, z, m, H, W, (int64_t)R * 2, rng, zhat);
        (void)orc_energy(st, H, W, 0.5f, 1.0f);
    }
    for (int32_t r = 0; r < R; ++r) orc_block_energy(st + r * HW, m, H, W, lb_h, lb_w, 0.5f, 1.0f, Hb + r * B);
    orc_temperature_grad(st, Hb, w, HW, R, B, T, dT);
    double out[2];
    orc_validate(zhat, z, m, HW, out);
    free(z); free(m); free(t); free(st); free(acc); free(en); free(zhat); free(Tsite); free(S); free(Ts); free(S2);
    free(N); free(No); free(N2); free(T); free(Hb); free(w); free(dT);
    return bad;
}

int main(void)
{
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    double u[2];
    orc_site_uniforms(~0ull, (1u << 28) - 1, 2, 0xffffffffu, 0xffffffffu, 7, 6, 3, u);
    const double cT[4] = {0.01, 0.1, 1.0, 10.0}, ce[4] = {-0.99, -0.95, -0.6, -0.45};
    const double Sb[3] = {-3.0, 0.0, -1.5};
    const int32_t Nb[3] = {4, 0, 2};
    float Tb[3];
    if (orc_calibrate_blocks(Sb, Nb, 3, 1.0f, cT, ce, 4, Tb) != 0) return 1;
    const float Tg[2] = {0.1f, 1.0f};
    double e[2];
    orc_reference_curve(0.5f, Tg, 2, 6, 3, 3, 7u, e);
    int bad = 0;
    bad |= run_case(1, 1, 1, 1, 1u);
    bad |= run_case(1, 9, 4, 4, 2u);
    bad |= run_case(7, 1, 3, 2, 3u);
    bad |= run_case(13, 17, 5, 6, 4u);
    bad |= run_case(16, 16, 16, 16, 5u);
    printf("oracle sanitizer checks %s\n", bad ? "FAILED" : "ok");
    return bad;
}
