/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the SV-MPR conditional Monte Carlo method
 * (Lach & Zukovic, "Fast gap-filling of massive data by local-equilibrium conditional simulations on GPU",
 * arXiv 2212.01317).  Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the HIP library; the two sides meet only in the seeded input
 * generators and in the published definition of the Philox4x32-10 counter-based generator, which each side
 * implements on its own.
 *
 * Every function names the passage of the paper it follows.  Where the paper is silent the reading taken is
 * stated at the function (the readings are listed together in the design notes of the repository).
 *
 * Conventions used throughout:
 *   - grids are row-major, site n = y*W + x, 0 <= x < W, 0 <= y < H;
 *   - mask[n] != 0 marks a sample (observed) site (the set G_S of Sec. 2.1), 0 marks a gap (G_P);
 *   - spin angles are stored in turns t in [0, 1]: phi = 2*pi*t (Sec. 2.1 maps the data linearly onto [0, 2*pi]);
 *   - colour of a site c(n) = (x + y) mod 2; the two colours are the interpenetrating sub-grids A and B of
 *     Sec. 2.2.2; colour 0 is updated first in every sweep;
 *   - open (free) boundaries: a site has up to four in-grid nearest neighbours, taken in the order
 *     up, left, right, down;
 *   - T-block of a site b(n) = (y / lb_h) * nbx + (x / lb_w), nbx = ceil(W / lb_w).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * Ten rounds of the Philox S-box on a 128-bit counter with a 64-bit key; the key is advanced by the Weyl
 * constants between rounds.  The paper does not name its generator; this counter-based one lets every
 * (realization, sweep, site) draw be computed independently and in any order.
 * ---------------------------------------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Stream layout (a reading: the paper is silent on the generator).
 *   key = (low 32 bits of seed, high 32 bits of seed)
 *   ctr = (pair, sweep, realization, scene << 4 | tag << 1 | colour)
 * Sites of one colour in row y sit at x = x0, x0+2, x0+4, ... with x0 = (y + colour) & 1.  Consecutive such sites
 * are paired: pair m of row y holds x0 + 4m (words 0 and 1) and x0 + 4m + 2 (words 2 and 3); its index is
 * y * ((W + 3) / 4) + m.  For any site, m = x >> 2 and the half (which word pair) is (x >> 1) & 1.
 * A word becomes a uniform on [0, 1) as (w >> 8) * 2^-24, exact in FP32 and FP64. */
enum { ORC_TAG_SWEEP = 0, ORC_TAG_INIT = 1, ORC_TAG_REFCURVE = 2 };

static double u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

static void site_uniforms(uint64_t seed, uint32_t scene, uint32_t tag, uint32_t sweep, uint32_t real,
                          int64_t W, int64_t x, int64_t y, double* u1, double* u2)
{
    uint32_t colour = (uint32_t)((x + y) & 1);
    uint32_t pair = (uint32_t)(y * ((W + 3) / 4) + (x >> 2));
    uint32_t ctr[4] = { pair, sweep, real, (scene << 4) | (tag << 1) | colour };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int half = (int)((x >> 1) & 1);
    *u1 = u24(w[2 * half]);
    *u2 = u24(w[2 * half + 1]);
}

/* Exposed for tests: the two uniforms a site draws in a given stream. */
void orc_site_uniforms(uint64_t seed, uint32_t scene, uint32_t tag, uint32_t sweep, uint32_t real, int64_t W,
                       int64_t x, int64_t y, double out[2])
{
    site_uniforms(seed, scene, tag, sweep, real, W, x, y, &out[0], &out[1]);
}

/* ------------------------------------------------------------------------------------------------------------
 * Sec. 2.1: the data are mapped linearly onto the spin-angle interval.  Reading: the observed minimum goes to
 * angle 0 and the observed maximum to 2*pi (t = 1 turn); a constant field maps to t = 0.  Gap sites get t = 0.
 * Returns 0, or -1 when there is no observed site, or -2 when an observed value is not finite.
 * ---------------------------------------------------------------------------------------------------------- */
int orc_map_angles(const float* z, const uint8_t* mask, int64_t H, int64_t W, float* t, double range[2])
{
    int64_t n_obs = 0;
    double zmin = INFINITY, zmax = -INFINITY;
    for (int64_t n = 0; n < H * W; ++n) {
        if (!mask[n]) continue;
        if (!isfinite(z[n])) return -2;
        double v = (double)z[n];
        if (v < zmin) zmin = v;
        if (v > zmax) zmax = v;
        ++n_obs;
    }
    if (n_obs == 0) return -1;
    double span = zmax - zmin;
    for (int64_t n = 0; n < H * W; ++n) {
        if (!mask[n] || span == 0.0) {
            t[n] = 0.0f;
        } else {
            t[n] = (float)(((double)z[n] - zmin) / span);
        }
    }
    range[0] = zmin;
    range[1] = zmax;
    return 0;
}

/* Threads the realization loops of orc_simulate run on: 1 in the plain build, the OpenMP team size in the parallel
 * build of the CPU baseline. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. (1): the energy of one bond of the MPR Hamiltonian, -J cos(q (phi_a - phi_b)), with phi = 2*pi*t. */
static double bond_energy(double t_a, double t_b, double two_pi_q, double J)
{
    return -J * cos(two_pi_q * (t_a - t_b));
}

double orc_bond_energy(float t_a, float t_b, float q, float J)
{
    return bond_energy((double)t_a, (double)t_b, 2.0 * ORC_PI * (double)q, (double)J);
}

/* ------------------------------------------------------------------------------------------------------------
 * Eq. (2) evaluated per T-block (Sec. 2.2.2, block-specific parameter inference).  Every site owns the bonds to
 * its right and lower neighbour, so each bond is counted once; a bond belongs to the block of its owner.
 * Only bonds whose both ends are samples enter: S[b] = sum of their energies, N[b] = their number.
 * Tsum[b] and Nobs[b] are the sum and the count of the observed t in the block (used by the block-mean start).
 * ---------------------------------------------------------------------------------------------------------- */
void orc_block_stats(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w,
                     float q, float J, double* S, int32_t* N, double* Tsum, int32_t* Nobs)
{
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int64_t b = 0; b < nbx * nby; ++b) {
        S[b] = 0.0;
        N[b] = 0;
        Tsum[b] = 0.0;
        Nobs[b] = 0;
    }
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t n = y * W + x;
            if (!mask[n]) continue;
            int64_t b = (y / lb_h) * nbx + (x / lb_w);
            Tsum[b] += (double)t[n];
            Nobs[b] += 1;
            if (x + 1 < W && mask[n + 1]) {
                S[b] += bond_energy(t[n], t[n + 1], tpq, J);
                N[b] += 1;
            }
            if (y + 1 < H && mask[n + W]) {
                S[b] += bond_energy(t[n], t[n + W], tpq, J);
                N[b] += 1;
            }
        }
    }
}

/* Directional form of the block statistics for the directional-coupling extension (Sec. 4 suggests distinguishing
 * the exchange interaction by direction, keeping the parameters local to blocks): the sample-bond energies of Eq. (2)
 * split by the direction of the bond, horizontal (a site and its right neighbour) into Sh, Nh and vertical (a site
 * and its lower neighbour) into Sv, Nv; a bond belongs to the block of its owner as above. */
void orc_block_stats_directional(const float* t, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h,
                                 int32_t lb_w, float q, float J, double* Sh, int32_t* Nh, double* Sv, int32_t* Nv)
{
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int64_t b = 0; b < nbx * nby; ++b) {
        Sh[b] = 0.0;
        Nh[b] = 0;
        Sv[b] = 0.0;
        Nv[b] = 0;
    }
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t n = y * W + x;
            if (!mask[n]) continue;
            int64_t b = (y / lb_h) * nbx + (x / lb_w);
            if (x + 1 < W && mask[n + 1]) {
                Sh[b] += bond_energy(t[n], t[n + 1], tpq, J);
                Nh[b] += 1;
            }
            if (y + 1 < H && mask[n + W]) {
                Sv[b] += bond_energy(t[n], t[n + W], tpq, J);
                Nv[b] += 1;
            }
        }
    }
}

/* ------------------------------------------------------------------------------------------------------------
 * Temperature by specific-energy matching (Sec. 2.1; per block in Sec. 2.2.2).
 * Reading: the matching curve e_ref(T) is the equilibrium energy per bond of the unconditional MPR model at
 * J = 1 (computed by orc_reference_curve); a block's T is the inverse of that curve at its per-bond sample energy
 * e_b = S_b / (J N_b), scaled by J.  The tabulated curve is first made non-decreasing by a running maximum; the
 * inverse is piecewise linear in (e, log T) between table points, linear in T between (e=-1, T=0) and the first
 * point (the harmonic low-T law is linear), and saturates at the last table temperature.
 * ---------------------------------------------------------------------------------------------------------- */
double orc_curve_inverse(double e, const double* curve_T, const double* curve_e, int32_t n)
{
    if (e <= -1.0) return 0.0;
    /* running maximum of the tabulated energies */
    double prev = curve_e[0];
    if (e <= prev) {
        double denom = prev + 1.0;
        return denom > 0.0 ? curve_T[0] * (e + 1.0) / denom : curve_T[0];
    }
    for (int32_t i = 1; i < n; ++i) {
        double cur = curve_e[i] > prev ? curve_e[i] : prev;
        if (cur >= e) {
            if (cur == prev) return curve_T[i];
            double lam = (e - prev) / (cur - prev);
            return exp((1.0 - lam) * log(curve_T[i - 1]) + lam * log(curve_T[i]));
        }
        prev = cur;
    }
    return curve_T[n - 1];
}

static int cmp_float(const void* a, const void* b)
{
    float fa = *(const float*)a, fb = *(const float*)b;
    return (fa > fb) - (fa < fb);
}

/* Sec. 2.2.2: blocks with sample bonds get T_b = J g(e_b); a block with no sample bond gets the median of the
 * block temperatures that could be estimated (reading: for an even count, the mean of the two middle values).
 * T is stored in FP32.  Returns 0, or -1 when no block has a sample bond. */
int orc_calibrate_blocks(const double* S, const int32_t* N, int64_t B, float J, const double* curve_T,
                         const double* curve_e, int32_t n_curve, float* T_out)
{
    float* have = (float*)malloc(sizeof(float) * (size_t)(B > 0 ? B : 1));
    int64_t n_have = 0;
    for (int64_t b = 0; b < B; ++b) {
        if (N[b] > 0) {
            double e_b = S[b] / ((double)J * (double)N[b]);
            T_out[b] = (float)((double)J * orc_curve_inverse(e_b, curve_T, curve_e, n_curve));
            have[n_have++] = T_out[b];
        }
    }
    if (n_have == 0) {
        free(have);
        return -1;
    }
    qsort(have, (size_t)n_have, sizeof(float), cmp_float);
    float med;
    if (n_have % 2 == 1) {
        med = have[n_have / 2];
    } else {
        med = (float)(((double)have[n_have / 2 - 1] + (double)have[n_have / 2]) * 0.5);
    }
    for (int64_t b = 0; b < B; ++b)
        if (N[b] == 0) T_out[b] = med;
    free(have);
    return 0;
}

/* ------------------------------------------------------------------------------------------------------------
 * One Metropolis update of gap site (x, y) under Eq. (1) with the other spins held fixed.
 * Reading of the proposal (the paper leaves it to earlier work): an independent uniform angle t' = u1.
 * dE = -J * sum over in-grid neighbours j (up, left, right, down) of [cos 2*pi*q(t'-t_j) - cos 2*pi*q(t-t_j)].
 * Accept iff u2 < exp(-dE/T) when T > 0, iff dE <= 0 when T = 0.
 * `periodic` wraps the neighbours (used for the unconditional reference lattice only).
 * ---------------------------------------------------------------------------------------------------------- */
static void metropolis_site(float* s, int64_t H, int64_t W, int64_t x, int64_t y, double T, double two_pi_q,
                            double J, double u1, double u2, int periodic)
{
    int64_t n = y * W + x;
    double t_old = (double)s[n];
    double t_new = (double)(float)u1;
    int64_t nb[4];
    int cnt = 0;
    if (periodic) {
        nb[cnt++] = ((y + H - 1) % H) * W + x;
        nb[cnt++] = y * W + (x + W - 1) % W;
        nb[cnt++] = y * W + (x + 1) % W;
        nb[cnt++] = ((y + 1) % H) * W + x;
    } else {
        if (y > 0) nb[cnt++] = n - W;
        if (x > 0) nb[cnt++] = n - 1;
        if (x + 1 < W) nb[cnt++] = n + 1;
        if (y + 1 < H) nb[cnt++] = n + W;
    }
    double acc = 0.0;
    for (int i = 0; i < cnt; ++i) {
        double tj = (double)s[nb[i]];
        acc += cos(two_pi_q * (t_new - tj)) - cos(two_pi_q * (t_old - tj));
    }
    double dE = -J * acc;
    int accept;
    if (T > 0.0) {
        accept = u2 < exp(-dE / T);
    } else {
        accept = dE <= 0.0;
    }
    if (accept) s[n] = (float)t_new;
}

/* Directional coupling (the extension of Sec. 4): every site carries two temperatures, Tx for its horizontal bonds
 * and Ty for its vertical bonds, so the Boltzmann factor of an update is exp(-dEh/Tx - dEv/Ty) with
 * dEh = -J * [left and right terms] and dEv = -J * [up and down terms] of the sum of metropolis_site (equivalently
 * couplings J and J Tx/Ty at temperature Tx).  Both temperatures are > 0.  Accept iff u2 < exp(w) with
 * w = J ah / Tx + J av / Ty, ah = left + right, av = up + down, each term cos 2 pi q (t' - t_j) - cos 2 pi q (t - t_j). */
static void metropolis_site_directional(float* s, int64_t H, int64_t W, int64_t x, int64_t y, double Tx, double Ty,
                                        double two_pi_q, double J, double u1, double u2)
{
    int64_t n = y * W + x;
    double t_old = (double)s[n];
    double t_new = (double)(float)u1;
    double ah = 0.0, av = 0.0;
    if (y > 0) {
        double tj = (double)s[n - W];
        av += cos(two_pi_q * (t_new - tj)) - cos(two_pi_q * (t_old - tj));
    }
    if (x > 0) {
        double tj = (double)s[n - 1];
        ah += cos(two_pi_q * (t_new - tj)) - cos(two_pi_q * (t_old - tj));
    }
    if (x + 1 < W) {
        double tj = (double)s[n + 1];
        ah += cos(two_pi_q * (t_new - tj)) - cos(two_pi_q * (t_old - tj));
    }
    if (y + 1 < H) {
        double tj = (double)s[n + W];
        av += cos(two_pi_q * (t_new - tj)) - cos(two_pi_q * (t_old - tj));
    }
    double w = J * ah / Tx + J * av / Ty;
    if (u2 < exp(w)) s[n] = (float)t_new;
}

/* Single-checkerboard sweep with directional block temperatures: Tx[b] = T[b], Ty[b] = T[B + b]. */
void orc_sweep_directional(float* s, const uint8_t* mask, int64_t H, int64_t W, const float* T, int32_t lb_h,
                           int32_t lb_w, float q, float J, uint64_t seed, uint32_t scene, uint32_t real,
                           uint32_t sweep)
{
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h;
    int64_t B = nbx * nby;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int colour = 0; colour < 2; ++colour) {
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = (y + colour) & 1; x < W; x += 2) {
                if (mask[y * W + x]) continue;
                int64_t b = (y / lb_h) * nbx + (x / lb_w);
                double u1, u2;
                site_uniforms(seed, scene, ORC_TAG_SWEEP, sweep, real, W, x, y, &u1, &u2);
                metropolis_site_directional(s, H, W, x, y, (double)T[b], (double)T[B + b], tpq, (double)J, u1, u2);
            }
        }
    }
}

/* Sec. 2.2.2, double checkerboard (DC): the grid is divided into the lb_h x lb_w blocks, coloured like a
 * checkerboard by (block row + block column) % 2; one sweep = the gap sites of colour 0, then of colour 1, inside
 * the even blocks, then the same inside the odd blocks.  Sites of one such phase share no bond.  The temperature of
 * a site is read from T with the tb_h x tb_w layout (the blocks themselves, or 1 x 1 for one temperature per
 * site).  The random numbers of a site are those of the single-checkerboard order. */
void orc_sweep_dc(float* s, const uint8_t* mask, int64_t H, int64_t W, const float* T, int32_t tb_h, int32_t tb_w,
                  int32_t lb_h, int32_t lb_w, float q, float J, uint64_t seed, uint32_t scene, uint32_t real,
                  uint32_t sweep)
{
    int64_t nbx_t = (W + tb_w - 1) / tb_w;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int parity = 0; parity < 2; ++parity) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t y = 0; y < H; ++y) {
                for (int64_t x = (y + colour) & 1; x < W; x += 2) {
                    if (mask[y * W + x]) continue;
                    if ((int)(((y / lb_h) + (x / lb_w)) & 1) != parity) continue;
                    double Tn = (double)T[(y / tb_h) * nbx_t + (x / tb_w)];
                    double u1, u2;
                    site_uniforms(seed, scene, ORC_TAG_SWEEP, sweep, real, W, x, y, &u1, &u2);
                    metropolis_site(s, H, W, x, y, Tn, tpq, (double)J, u1, u2, 0);
                }
            }
        }
    }
}

/* Sec. 2.2.2, single checkerboard: one sweep = all gap sites of colour 0, then all gap sites of colour 1.  Sites
 * of one colour share no bond, so their order inside a half-sweep does not matter.  Each site uses the
 * temperature of its T-block (the same block layout as the energy estimate). */
void orc_sweep(float* s, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks, int32_t lb_h,
               int32_t lb_w, float q, float J, uint64_t seed, uint32_t scene, uint32_t real, uint32_t sweep)
{
    int64_t nbx = (W + lb_w - 1) / lb_w;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int colour = 0; colour < 2; ++colour) {
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = (y + colour) & 1; x < W; x += 2) {
                if (mask[y * W + x]) continue;
                double T = (double)T_blocks[(y / lb_h) * nbx + (x / lb_w)];
                double u1, u2;
                site_uniforms(seed, scene, ORC_TAG_SWEEP, sweep, real, W, x, y, &u1, &u2);
                metropolis_site(s, H, W, x, y, T, tpq, (double)J, u1, u2, 0);
            }
        }
    }
}

/* Whole-grid specific energy (Sec. 3.3, Fig. 9): sum of Eq. (1) over all bonds, divided by J times the number of
 * bonds, so that it is an energy per bond in [-1, 1]. */
double orc_energy(const float* s, int64_t H, int64_t W, float q, float J)
{
    double tpq = 2.0 * ORC_PI * (double)q;
    double sum = 0.0;
    int64_t nbonds = 0;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t n = y * W + x;
            if (x + 1 < W) {
                sum += bond_energy(s[n], s[n + 1], tpq, (double)J);
                ++nbonds;
            }
            if (y + 1 < H) {
                sum += bond_energy(s[n], s[n + W], tpq, (double)J);
                ++nbonds;
            }
        }
    }
    return nbonds > 0 ? sum / ((double)J * (double)nbonds) : 0.0;
}

/* ------------------------------------------------------------------------------------------------------------
 * The matching curve: equilibrium energy per bond of the unconditional MPR model (every site free) at J = 1 on a
 * periodic L x L lattice (L even), for each temperature of T_grid.  Each temperature i is its own chain
 * (realization index i in the reference stream), started from the uniform state t = 1/2, run n_therm sweeps to
 * equilibrate and n_meas more sweeps over which the per-bond energy (2 L^2 bonds) is averaged.
 * ---------------------------------------------------------------------------------------------------------- */
/* One sweep of chain `chain` of the unconditional periodic lattice (all sites free, J = 1). */
static void reference_sweep(float* s, int32_t L, double T, double tpq, uint64_t seed, uint32_t chain, uint32_t k)
{
    for (int colour = 0; colour < 2; ++colour) {
        for (int64_t y = 0; y < L; ++y) {
            for (int64_t x = (y + colour) & 1; x < L; x += 2) {
                double u1, u2;
                site_uniforms(seed, 0u, ORC_TAG_REFCURVE, k, chain, L, x, y, &u1, &u2);
                metropolis_site(s, L, L, x, y, T, tpq, 1.0, u1, u2, 1);
            }
        }
    }
}

static double periodic_energy(const float* s, int32_t L, double tpq)
{
    double sum = 0.0;
    for (int64_t y = 0; y < L; ++y) {
        for (int64_t x = 0; x < L; ++x) {
            double tn = (double)s[y * L + x];
            sum += bond_energy(tn, (double)s[y * L + (x + 1) % L], tpq, 1.0);
            sum += bond_energy(tn, (double)s[((y + 1) % L) * L + x], tpq, 1.0);
        }
    }
    return sum / (2.0 * (double)L * (double)L);
}

void orc_reference_curve(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm, int32_t n_meas,
                         uint64_t seed, double* e_out)
{
    double tpq = 2.0 * ORC_PI * (double)q;
    float* s = (float*)malloc(sizeof(float) * (size_t)L * (size_t)L);
    for (int32_t i = 0; i < nT; ++i) {
        double T = (double)T_grid[i];
        for (int64_t n = 0; n < (int64_t)L * L; ++n) s[n] = 0.5f;
        double acc_e = 0.0;
        for (int32_t k = 1; k <= n_therm + n_meas; ++k) {
            reference_sweep(s, L, T, tpq, seed, (uint32_t)i, (uint32_t)k);
            if (k > n_therm) acc_e += periodic_energy(s, L, tpq);
        }
        e_out[i] = n_meas > 0 ? acc_e / (double)n_meas : 0.0;
    }
    free(s);
}

/* The state of chain `chain` of the reference lattice at temperature T after n_sweeps sweeps from t = 1/2: a
 * sample of the unconditional MPR model (used to check that calibration recovers T on a fully observed field). */
void orc_unconditional_sample(float q, float T, int32_t L, int32_t n_sweeps, uint64_t seed, uint32_t chain,
                              float* state_out)
{
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int64_t n = 0; n < (int64_t)L * L; ++n) state_out[n] = 0.5f;
    for (int32_t k = 1; k <= n_sweeps; ++k) reference_sweep(state_out, L, (double)T, tpq, seed, chain, (uint32_t)k);
}

/* ------------------------------------------------------------------------------------------------------------
 * Equilibrium test (Sec. 3.4: memory length n_fit of the energy series, a check every n_f sweeps, the first
 * after n_fit + n_f sweeps).  Reading of the test: beta is the ordinary least-squares slope of the last n_fit
 * energies against the sweep index; equilibrium is declared once beta no longer points away from the starting
 * energy, i.e. beta * sign(e(k) - e(0)) <= 0.
 * ---------------------------------------------------------------------------------------------------------- */
double orc_ols_slope(const double* y, int32_t n)
{
    double xm = 0.0, ym = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        xm += (double)j;
        ym += y[j];
    }
    xm /= (double)n;
    ym /= (double)n;
    double sxy = 0.0, sxx = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        sxy += ((double)j - xm) * (y[j] - ym);
        sxx += ((double)j - xm) * ((double)j - xm);
    }
    return sxx > 0.0 ? sxy / sxx : 0.0;
}

/* e[0..k] is the energy series (e[0] before the first sweep).  Returns 1 when the check at sweep k declares
 * equilibrium, 0 otherwise (also when k is not a check point). */
int orc_stop_check(const double* e, int32_t k, int32_t n_fit, int32_t n_f)
{
    if (k < n_fit + n_f || (k - n_fit) % n_f != 0) return 0;
    double beta = orc_ols_slope(e + (k - n_fit + 1), n_fit);
    double d = e[k] - e[0];
    double sigma0 = (d > 0.0) - (d < 0.0);
    return beta * sigma0 <= 0.0;
}

/* The per-chain variant of the test (a reading of Sec. 3.3 / 3.4: the energy of Fig. 9 is that of one simulation of
 * the whole grid, averaged over realizations only for the figure).  ser[j * R + r] is chain r's own whole-grid
 * energy after sweep j (j = 0 .. k).  At a check point every chain that has not yet passed applies the test of
 * orc_stop_check to its own series, and a chain that passes stays passed (passed[r] = 1: its equilibrium sweep is
 * that check); the scene stops at the first check where every chain has passed, so its k* is the largest of the
 * chains' own equilibrium sweeps.  Returns 1 then, 0 otherwise (also when k is not a check point). */
int orc_stop_check_chains(const double* ser, int32_t R, int32_t k, int32_t n_fit, int32_t n_f, uint8_t* passed)
{
    if (k < n_fit + n_f || (k - n_fit) % n_f != 0) return 0;
    double* y = (double*)malloc(sizeof(double) * (size_t)n_fit);
    int all = 1;
    for (int32_t r = 0; r < R; ++r) {
        if (!passed[r]) {
            for (int32_t j = 0; j < n_fit; ++j) y[j] = ser[(int64_t)(k - n_fit + 1 + j) * R + r];
            double beta = orc_ols_slope(y, n_fit);
            double d = ser[(int64_t)k * R + r] - ser[r];
            double sigma0 = (d > 0.0) - (d < 0.0);
            if (beta * sigma0 <= 0.0) passed[r] = 1;
        }
        all = all && passed[r];
    }
    free(y);
    return all;
}

/* ------------------------------------------------------------------------------------------------------------
 * Full conditional simulation of one scene (Sec. 2.1 / 2.2.2 / 3.3 / 3.4), all realizations in lockstep:
 *   1. start: gap sites get the block mean of the observed t (SV-MPR, Sec. 3.3; reading: a block without samples
 *      gets the global observed mean) or a uniform draw from the init stream (MPR, random start);
 *   2. e(0), then sweeps k = 1, 2, ... each followed by the realization-averaged whole-grid energy e(k);
 *      FIXED mode stops after n_eq sweeps, AUTO mode applies orc_stop_check to e(k) and the cap n_max, the
 *      per-chain AUTO mode (stop_mode 2) applies orc_stop_check_chains to every realization's own energy series;
 *   3. n_samp further sweeps (continuing the sweep counter), after each of which the gap values of every
 *      realization are added to acc (Sec. 2.1: the prediction is the mean of the conditional distribution).
 * t: mapped angles (observed sites used); state: [R][H][W] out; acc: [H][W] out (only gap sites accumulate);
 * energy: [n_max + 1 (AUTO) or n_eq + 1 (FIXED)] out, e(0..k*).  Returns k* (sweeps before sampling), and sets
 * *converged to 0 when AUTO hit n_max.
 * ---------------------------------------------------------------------------------------------------------- */
int32_t orc_simulate(const float* t, const uint8_t* mask, int64_t H, int64_t W, const float* T_blocks,
                     int32_t lb_h, int32_t lb_w, float q, float J, int32_t R, int32_t real_offset,
                     int32_t init_mode /* 0 random, 1 block mean */,
                     int32_t stop_mode /* 0 fixed, 1 auto, 2 auto per chain */,
                     int32_t n_eq, int32_t n_samp, int32_t n_fit, int32_t n_f, int32_t n_max, uint64_t seed,
                     uint32_t scene, int32_t t_per_site /* 0: T_blocks per block, 1: T_blocks[H*W] per site */,
                     int32_t order /* 0: single checkerboard, 1: double checkerboard over the lb_h x lb_w blocks */,
                     int32_t directional /* 1: T_blocks = [Tx of the B blocks, Ty of the B blocks], SC order */,
                     float* state, double* acc, double* energy, int32_t* converged)
{
    /* the temperature layout the sweeps read: blocks of lb_h x lb_w, or one temperature per site (SST) */
    const int32_t tb_h = t_per_site ? 1 : lb_h, tb_w = t_per_site ? 1 : lb_w;
    /* directional coupling: both temperatures raised to at least fl32(1e-3 J) */
    float* T_dir = NULL;
    if (directional) {
        int64_t nb = ((W + lb_w - 1) / lb_w) * ((H + lb_h - 1) / lb_h);
        float floor_T = (float)(1e-3 * (double)J);
        T_dir = (float*)malloc(sizeof(float) * (size_t)(2 * nb));
        for (int64_t i = 0; i < 2 * nb; ++i) T_dir[i] = T_blocks[i] > floor_T ? T_blocks[i] : floor_T;
        T_blocks = T_dir;
    }
    int64_t HW = H * W;
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h;
    int64_t B = nbx * nby;
    double* S = (double*)malloc(sizeof(double) * (size_t)B);
    int32_t* N = (int32_t*)malloc(sizeof(int32_t) * (size_t)B);
    double* Tsum = (double*)malloc(sizeof(double) * (size_t)B);
    int32_t* Nobs = (int32_t*)malloc(sizeof(int32_t) * (size_t)B);
    orc_block_stats(t, mask, H, W, lb_h, lb_w, q, J, S, N, Tsum, Nobs);
    double all_sum = 0.0;
    int64_t all_cnt = 0;
    for (int64_t b = 0; b < B; ++b) {
        all_sum += Tsum[b];
        all_cnt += Nobs[b];
    }
    float global_mean = all_cnt > 0 ? (float)(all_sum / (double)all_cnt) : 0.0f;

    /* Realizations are independent chains: with OpenMP (the parallel build of the CPU baseline) they are spread over
     * threads; every sum over realizations is still taken in realization order, so both builds agree bit for bit. */
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < R; ++r) {
        float* s = state + (int64_t)r * HW;
        uint32_t real = (uint32_t)(r + real_offset);
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = 0; x < W; ++x) {
                int64_t n = y * W + x;
                if (mask[n]) {
                    s[n] = t[n];
                } else if (init_mode == 1) {
                    int64_t b = (y / lb_h) * nbx + (x / lb_w);
                    s[n] = Nobs[b] > 0 ? (float)(Tsum[b] / (double)Nobs[b]) : global_mean;
                } else {
                    double u1, u2;
                    site_uniforms(seed, scene, ORC_TAG_INIT, 0u, real, W, x, y, &u1, &u2);
                    s[n] = (float)u1;
                }
            }
        }
    }
    for (int64_t n = 0; n < HW; ++n) acc[n] = 0.0;

    int32_t k_cap = stop_mode != 0 ? n_max : n_eq;
    double* e_r = (double*)malloc(sizeof(double) * (size_t)R);
    /* per-chain mode: every chain's series, [k][R], and the chains that have passed */
    double* ser = stop_mode == 2 ? (double*)malloc(sizeof(double) * (size_t)R * (size_t)(k_cap + 1)) : NULL;
    uint8_t* passed = stop_mode == 2 ? (uint8_t*)calloc((size_t)R, 1) : NULL;
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < R; ++r) e_r[r] = orc_energy(state + (int64_t)r * HW, H, W, q, J);
    double e0 = 0.0;
    for (int32_t r = 0; r < R; ++r) e0 += e_r[r];
    energy[0] = e0 / (double)R;
    if (ser)
        for (int32_t r = 0; r < R; ++r) ser[r] = e_r[r];
    int32_t k = 0;
    *converged = 1;
    while (k < k_cap) {
        ++k;
#pragma omp parallel for schedule(static)
        for (int32_t r = 0; r < R; ++r) {
            float* s = state + (int64_t)r * HW;
            if (directional)
                orc_sweep_directional(s, mask, H, W, T_blocks, lb_h, lb_w, q, J, seed, scene,
                                      (uint32_t)(r + real_offset), (uint32_t)k);
            else if (order == 1)
                orc_sweep_dc(s, mask, H, W, T_blocks, tb_h, tb_w, lb_h, lb_w, q, J, seed, scene,
                             (uint32_t)(r + real_offset), (uint32_t)k);
            else
                orc_sweep(s, mask, H, W, T_blocks, tb_h, tb_w, q, J, seed, scene, (uint32_t)(r + real_offset),
                          (uint32_t)k);
            e_r[r] = orc_energy(s, H, W, q, J);
        }
        double ek = 0.0;
        for (int32_t r = 0; r < R; ++r) ek += e_r[r];
        energy[k] = ek / (double)R;
        if (ser)
            for (int32_t r = 0; r < R; ++r) ser[(int64_t)k * R + r] = e_r[r];
        if (stop_mode == 1 && orc_stop_check(energy, k, n_fit, n_f)) break;
        if (stop_mode == 2 && orc_stop_check_chains(ser, R, k, n_fit, n_f, passed)) break;
        if (stop_mode != 0 && k == n_max) *converged = 0;
    }
    free(ser);
    free(passed);
    int32_t k_star = k;
    for (int32_t s_i = 1; s_i <= n_samp; ++s_i) {
#pragma omp parallel for schedule(static)
        for (int32_t r = 0; r < R; ++r) {
            float* s = state + (int64_t)r * HW;
            if (directional)
                orc_sweep_directional(s, mask, H, W, T_blocks, lb_h, lb_w, q, J, seed, scene,
                                      (uint32_t)(r + real_offset), (uint32_t)(k_star + s_i));
            else if (order == 1)
                orc_sweep_dc(s, mask, H, W, T_blocks, tb_h, tb_w, lb_h, lb_w, q, J, seed, scene,
                             (uint32_t)(r + real_offset), (uint32_t)(k_star + s_i));
            else
                orc_sweep(s, mask, H, W, T_blocks, tb_h, tb_w, q, J, seed, scene, (uint32_t)(r + real_offset),
                          (uint32_t)(k_star + s_i));
        }
        for (int32_t r = 0; r < R; ++r) {
            const float* s = state + (int64_t)r * HW;
            for (int64_t n = 0; n < HW; ++n)
                if (!mask[n]) acc[n] += (double)s[n];
        }
    }
    free(e_r);
    free(S);
    free(N);
    free(Tsum);
    free(Nobs);
    free(T_dir);
    return k_star;
}

/* ------------------------------------------------------------------------------------------------------------
 * Sec. 2.2.3 (SST, site-specific temperatures): starting from the block temperatures (every site takes the value of
 * its block), the temperature of every site is replaced n_s times in succession by the mean over the surrounding
 * area of radius r_s.  Readings: the area is the (2 r_s + 1) x (2 r_s + 1) square of sites around the site, cut at
 * the grid edges (the mean is over the sites inside the grid); each pass reads the previous pass only; FP64, the
 * window summed row by row from the top left; one rounding to FP32 at the end.
 * ---------------------------------------------------------------------------------------------------------- */
void orc_sst_temperatures(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t r_s,
                          int32_t n_s, float* T_site)
{
    int64_t HW = H * W, nbx = (W + lb_w - 1) / lb_w;
    double* a = (double*)malloc(sizeof(double) * (size_t)HW);
    double* b = (double*)malloc(sizeof(double) * (size_t)HW);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) a[y * W + x] = (double)T_blocks[(y / lb_h) * nbx + (x / lb_w)];
    for (int32_t pass = 0; pass < n_s; ++pass) {
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = 0; x < W; ++x) {
                double sum = 0.0;
                int64_t cnt = 0;
                for (int64_t yy = y - r_s; yy <= y + r_s; ++yy) {
                    if (yy < 0 || yy >= H) continue;
                    for (int64_t xx = x - r_s; xx <= x + r_s; ++xx) {
                        if (xx < 0 || xx >= W) continue;
                        sum += a[yy * W + xx];
                        ++cnt;
                    }
                }
                b[y * W + x] = sum / (double)cnt;
            }
        }
        double* tmp = a;
        a = b;
        b = tmp;
    }
    for (int64_t n = 0; n < HW; ++n) T_site[n] = (float)a[n];
    free(a);
    free(b);
}

/* ------------------------------------------------------------------------------------------------------------
 * Sec. 2.1: after equilibrium the gap spins are back-transformed; the prediction is the mean of the conditional
 * distribution, estimated by the mean of the n_samples accumulated states.  Observed sites keep their value.
 * ---------------------------------------------------------------------------------------------------------- */
void orc_predict(const double* acc, const float* z, const uint8_t* mask, int64_t H, int64_t W, int64_t n_samples,
                 const double range[2], float* zhat)
{
    double zmin = range[0], span = range[1] - range[0];
    for (int64_t n = 0; n < H * W; ++n) {
        if (mask[n]) {
            zhat[n] = z[n];
        } else {
            double tbar = acc[n] / (double)n_samples;
            zhat[n] = (float)(zmin + span * tbar);
        }
    }
}

/* Eq. (3) and Eq. (4): average absolute error and root average squared error over the evaluated sites. */
void orc_validate(const float* zhat, const float* truth, const uint8_t* eval_mask, int64_t n, double out[2])
{
    double sa = 0.0, s2 = 0.0;
    int64_t P = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!eval_mask[i]) continue;
        double e = (double)truth[i] - (double)zhat[i];
        sa += fabs(e);
        s2 += e * e;
        ++P;
    }
    out[0] = P > 0 ? sa / (double)P : 0.0;
    out[1] = P > 0 ? sqrt(s2 / (double)P) : 0.0;
}

/* ------------------------------------------------------------------------------------------------------------
 * Gradient of the realization-averaged prediction with respect to the block temperatures (a project addition
 * built on Sec. 2.2.2).  For a density proportional to exp(-sum_b H_b / T_b), d<f>/dT_b = Cov(f, H_b) / T_b^2.
 * H_b is the part of Eq. (1) attributed to block b: every bond with at least one gap end, counted in the block of
 * its gap end; a bond between two gaps in different blocks counts one half in each.  Bonds between two samples do
 * not depend on the state and are left out.
 * ---------------------------------------------------------------------------------------------------------- */
void orc_block_energy(const float* s, const uint8_t* mask, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w,
                      float q, float J, double* Hb)
{
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int64_t b = 0; b < nbx * nby; ++b) Hb[b] = 0.0;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t n = y * W + x;
            if (mask[n]) continue;
            int64_t b = (y / lb_h) * nbx + (x / lb_w);
            int64_t nb[4];
            int cnt = 0;
            if (y > 0) nb[cnt++] = n - W;
            if (x > 0) nb[cnt++] = n - 1;
            if (x + 1 < W) nb[cnt++] = n + 1;
            if (y + 1 < H) nb[cnt++] = n + W;
            for (int i = 0; i < cnt; ++i) {
                double share = mask[nb[i]] ? 1.0 : 0.5;
                Hb[b] += share * bond_energy((double)s[n], (double)s[nb[i]], tpq, (double)J);
            }
        }
    }
}

/* g_r = sum over sites of w * t_r (w = dL/dzhat * (zmax - zmin) at gaps, 0 at samples: with one sampling sweep
 * E[zhat] = zmin + (zmax - zmin) E[t]);
 * dT[b] = [sum_r (g_r - mean g)(H_rb - mean H_b) / (R - 1)] / T_b^2, all in FP64 (R >= 2; T_b = 0 gives 0). */
void orc_temperature_grad(const float* states, const double* Hrb, const double* w, int64_t HW, int32_t R, int64_t B,
                          const float* T_blocks, double* dT)
{
    double* g = (double*)malloc(sizeof(double) * (size_t)R);
    double gm = 0.0;
    for (int32_t r = 0; r < R; ++r) {
        double acc = 0.0;
        const float* s = states + (int64_t)r * HW;
        for (int64_t n = 0; n < HW; ++n) acc += w[n] * (double)s[n];
        g[r] = acc;
        gm += acc;
    }
    gm /= (double)R;
    for (int64_t b = 0; b < B; ++b) {
        double hm = 0.0;
        for (int32_t r = 0; r < R; ++r) hm += Hrb[(int64_t)r * B + b];
        hm /= (double)R;
        double cov = 0.0;
        for (int32_t r = 0; r < R; ++r) cov += (g[r] - gm) * (Hrb[(int64_t)r * B + b] - hm);
        cov /= (double)(R - 1);
        double T = (double)T_blocks[b];
        dT[b] = T > 0.0 ? cov / (T * T) : 0.0;
    }
    free(g);
}

/* ============================================================================================================
 * The three-dimensional lattice (the extension to 3D named in Sec. 4).  Reading: the same model on a D x H x W grid
 * of sites n = (z*H + y)*W + x with the six nearest neighbours of the simple cubic lattice and open boundaries; the
 * two colours of the checkerboard are c = (x + y + z) mod 2 (sites of one colour share no bond); the temperature
 * blocks are lb_d x lb_h x lb_w boxes, b = ((z/lb_d)*nby + y/lb_h)*nbx + x/lb_w; every site owns the bonds to its
 * +x, +y and +z neighbours.  The random-number stream is that of the plane with the row index r = z*H + y in place
 * of y and the colour (x + y + z) mod 2: pair index r*((W + 3)/4) + (x >> 2), words 2*((x >> 1) & 1) and the next.
 * On one plane (D = 1) every function below is the two-dimensional one.
 * ============================================================================================================ */
static void site_uniforms3(uint64_t seed, uint32_t scene, uint32_t tag, uint32_t sweep, uint32_t real, int64_t H,
                           int64_t W, int64_t x, int64_t y, int64_t z, double* u1, double* u2)
{
    uint32_t colour = (uint32_t)((x + y + z) & 1);
    int64_t row = z * H + y;
    uint32_t pair = (uint32_t)(row * ((W + 3) / 4) + (x >> 2));
    uint32_t ctr[4] = { pair, sweep, real, (scene << 4) | (tag << 1) | colour };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int half = (int)((x >> 1) & 1);
    *u1 = u24(w[2 * half]);
    *u2 = u24(w[2 * half + 1]);
}

void orc_site_uniforms3(uint64_t seed, uint32_t scene, uint32_t tag, uint32_t sweep, uint32_t real, int64_t H,
                        int64_t W, int64_t x, int64_t y, int64_t z, double out[2])
{
    site_uniforms3(seed, scene, tag, sweep, real, H, W, x, y, z, &out[0], &out[1]);
}

/* Eq. (2) per 3D block: sample-bond energies and counts over the +x, +y, +z bonds whose ends are both samples, and
 * the sum and count of the observed t. */
void orc_block_stats3(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W, int32_t lb_d,
                      int32_t lb_h, int32_t lb_w, float q, float J, double* S, int32_t* N, double* Tsum, int32_t* Nobs)
{
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h, nbz = (D + lb_d - 1) / lb_d;
    double tpq = 2.0 * ORC_PI * (double)q;
    int64_t HW = H * W;
    for (int64_t b = 0; b < nbx * nby * nbz; ++b) {
        S[b] = 0.0;
        N[b] = 0;
        Tsum[b] = 0.0;
        Nobs[b] = 0;
    }
    for (int64_t z = 0; z < D; ++z) {
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = 0; x < W; ++x) {
                int64_t n = z * HW + y * W + x;
                if (!mask[n]) continue;
                int64_t b = ((z / lb_d) * nby + y / lb_h) * nbx + x / lb_w;
                Tsum[b] += (double)t[n];
                Nobs[b] += 1;
                if (x + 1 < W && mask[n + 1]) {
                    S[b] += bond_energy(t[n], t[n + 1], tpq, J);
                    N[b] += 1;
                }
                if (y + 1 < H && mask[n + W]) {
                    S[b] += bond_energy(t[n], t[n + W], tpq, J);
                    N[b] += 1;
                }
                if (z + 1 < D && mask[n + HW]) {
                    S[b] += bond_energy(t[n], t[n + HW], tpq, J);
                    N[b] += 1;
                }
            }
        }
    }
}

/* One Metropolis update of gap site (x, y, z): the proposal and the test of metropolis_site, over the in-grid
 * neighbours in the order back (z - 1), up, left, right, down, front (z + 1); `periodic` wraps them (reference
 * lattice only). */
static void metropolis_site3(float* s, int64_t D, int64_t H, int64_t W, int64_t x, int64_t y, int64_t z, double T,
                             double two_pi_q, double J, double u1, double u2, int periodic)
{
    int64_t HW = H * W;
    int64_t n = z * HW + y * W + x;
    double t_old = (double)s[n];
    double t_new = (double)(float)u1;
    int64_t nb[6];
    int cnt = 0;
    if (periodic) {
        nb[cnt++] = ((z + D - 1) % D) * HW + y * W + x;
        nb[cnt++] = z * HW + ((y + H - 1) % H) * W + x;
        nb[cnt++] = z * HW + y * W + (x + W - 1) % W;
        nb[cnt++] = z * HW + y * W + (x + 1) % W;
        nb[cnt++] = z * HW + ((y + 1) % H) * W + x;
        nb[cnt++] = ((z + 1) % D) * HW + y * W + x;
    } else {
        if (z > 0) nb[cnt++] = n - HW;
        if (y > 0) nb[cnt++] = n - W;
        if (x > 0) nb[cnt++] = n - 1;
        if (x + 1 < W) nb[cnt++] = n + 1;
        if (y + 1 < H) nb[cnt++] = n + W;
        if (z + 1 < D) nb[cnt++] = n + HW;
    }
    double acc = 0.0;
    for (int i = 0; i < cnt; ++i) {
        double tj = (double)s[nb[i]];
        acc += cos(two_pi_q * (t_new - tj)) - cos(two_pi_q * (t_old - tj));
    }
    double dE = -J * acc;
    int accept;
    if (T > 0.0) {
        accept = u2 < exp(-dE / T);
    } else {
        accept = dE <= 0.0;
    }
    if (accept) s[n] = (float)t_new;
}

/* Single-checkerboard sweep of the 3D grid: all gap sites of colour 0, then of colour 1, each with the temperature
 * of its block. */
void orc_sweep3(float* s, const uint8_t* mask, int64_t D, int64_t H, int64_t W, const float* T_blocks, int32_t lb_d,
                int32_t lb_h, int32_t lb_w, float q, float J, uint64_t seed, uint32_t scene, uint32_t real,
                uint32_t sweep)
{
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h;
    double tpq = 2.0 * ORC_PI * (double)q;
    for (int colour = 0; colour < 2; ++colour) {
        for (int64_t z = 0; z < D; ++z) {
            for (int64_t y = 0; y < H; ++y) {
                for (int64_t x = (y + z + colour) & 1; x < W; x += 2) {
                    if (mask[(z * H + y) * W + x]) continue;
                    double T = (double)T_blocks[((z / lb_d) * nby + y / lb_h) * nbx + x / lb_w];
                    double u1, u2;
                    site_uniforms3(seed, scene, ORC_TAG_SWEEP, sweep, real, H, W, x, y, z, &u1, &u2);
                    metropolis_site3(s, D, H, W, x, y, z, T, tpq, (double)J, u1, u2, 0);
                }
            }
        }
    }
}

/* Whole-grid specific energy of the 3D grid: Eq. (1) summed over all bonds, divided by J times their number. */
double orc_energy3(const float* s, int64_t D, int64_t H, int64_t W, float q, float J)
{
    double tpq = 2.0 * ORC_PI * (double)q;
    int64_t HW = H * W;
    double sum = 0.0;
    int64_t nbonds = 0;
    for (int64_t z = 0; z < D; ++z) {
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = 0; x < W; ++x) {
                int64_t n = z * HW + y * W + x;
                if (x + 1 < W) {
                    sum += bond_energy(s[n], s[n + 1], tpq, (double)J);
                    ++nbonds;
                }
                if (y + 1 < H) {
                    sum += bond_energy(s[n], s[n + W], tpq, (double)J);
                    ++nbonds;
                }
                if (z + 1 < D) {
                    sum += bond_energy(s[n], s[n + HW], tpq, (double)J);
                    ++nbonds;
                }
            }
        }
    }
    return nbonds > 0 ? sum / ((double)J * (double)nbonds) : 0.0;
}

/* The matching curve of the 3D model: equilibrium energy per bond of the unconditional model at J = 1 on a periodic
 * L x L x L lattice (L even), one chain per temperature (realization index i of the reference stream), started
 * from t = 1/2, n_therm sweeps, then the per-bond energy (3 L^3 bonds) averaged over n_meas sweeps. */
void orc_reference_curve3(float q, const float* T_grid, int32_t nT, int32_t L, int32_t n_therm, int32_t n_meas,
                          uint64_t seed, double* e_out)
{
    double tpq = 2.0 * ORC_PI * (double)q;
    int64_t L3 = (int64_t)L * L * L, L2 = (int64_t)L * L;
    float* s = (float*)malloc(sizeof(float) * (size_t)L3);
    for (int32_t i = 0; i < nT; ++i) {
        double T = (double)T_grid[i];
        for (int64_t n = 0; n < L3; ++n) s[n] = 0.5f;
        double acc_e = 0.0;
        for (int32_t k = 1; k <= n_therm + n_meas; ++k) {
            for (int colour = 0; colour < 2; ++colour) {
                for (int64_t z = 0; z < L; ++z) {
                    for (int64_t y = 0; y < L; ++y) {
                        for (int64_t x = (y + z + colour) & 1; x < L; x += 2) {
                            double u1, u2;
                            site_uniforms3(seed, 0u, ORC_TAG_REFCURVE, (uint32_t)k, (uint32_t)i, L, L, x, y, z, &u1,
                                           &u2);
                            metropolis_site3(s, L, L, L, x, y, z, T, tpq, 1.0, u1, u2, 1);
                        }
                    }
                }
            }
            if (k > n_therm) {
                double sum = 0.0;
                for (int64_t z = 0; z < L; ++z)
                    for (int64_t y = 0; y < L; ++y)
                        for (int64_t x = 0; x < L; ++x) {
                            double tn = (double)s[z * L2 + y * L + x];
                            sum += bond_energy(tn, (double)s[z * L2 + y * L + (x + 1) % L], tpq, 1.0);
                            sum += bond_energy(tn, (double)s[z * L2 + ((y + 1) % L) * L + x], tpq, 1.0);
                            sum += bond_energy(tn, (double)s[((z + 1) % L) * L2 + y * L + x], tpq, 1.0);
                        }
                acc_e += sum / (3.0 * (double)L3);
            }
        }
        e_out[i] = n_meas > 0 ? acc_e / (double)n_meas : 0.0;
    }
    free(s);
}

/* Conditional simulation of one 3D scene, all realizations in lockstep, with the steps of orc_simulate (block-mean
 * or uniform start, energy series e(0..k), FIXED or AUTO stop by orc_stop_check with the cap n_max, n_samp sampling
 * sweeps accumulated into acc), single-checkerboard order and block temperatures.  Returns k*; *converged as in
 * orc_simulate. */
int32_t orc_simulate3(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W, const float* T_blocks,
                      int32_t lb_d, int32_t lb_h, int32_t lb_w, float q, float J, int32_t R, int32_t real_offset,
                      int32_t init_mode, int32_t stop_mode, int32_t n_eq, int32_t n_samp, int32_t n_fit, int32_t n_f,
                      int32_t n_max, uint64_t seed, uint32_t scene, float* state, double* acc, double* energy,
                      int32_t* converged)
{
    int64_t n_all = D * H * W;
    int64_t nbx = (W + lb_w - 1) / lb_w, nby = (H + lb_h - 1) / lb_h, nbz = (D + lb_d - 1) / lb_d;
    int64_t B = nbx * nby * nbz;
    double* S = (double*)malloc(sizeof(double) * (size_t)B);
    int32_t* N = (int32_t*)malloc(sizeof(int32_t) * (size_t)B);
    double* Tsum = (double*)malloc(sizeof(double) * (size_t)B);
    int32_t* Nobs = (int32_t*)malloc(sizeof(int32_t) * (size_t)B);
    orc_block_stats3(t, mask, D, H, W, lb_d, lb_h, lb_w, q, J, S, N, Tsum, Nobs);
    double all_sum = 0.0;
    int64_t all_cnt = 0;
    for (int64_t b = 0; b < B; ++b) {
        all_sum += Tsum[b];
        all_cnt += Nobs[b];
    }
    float global_mean = all_cnt > 0 ? (float)(all_sum / (double)all_cnt) : 0.0f;
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < R; ++r) {
        float* s = state + (int64_t)r * n_all;
        uint32_t real = (uint32_t)(r + real_offset);
        for (int64_t z = 0; z < D; ++z) {
            for (int64_t y = 0; y < H; ++y) {
                for (int64_t x = 0; x < W; ++x) {
                    int64_t n = (z * H + y) * W + x;
                    if (mask[n]) {
                        s[n] = t[n];
                    } else if (init_mode == 1) {
                        int64_t b = ((z / lb_d) * nby + y / lb_h) * nbx + x / lb_w;
                        s[n] = Nobs[b] > 0 ? (float)(Tsum[b] / (double)Nobs[b]) : global_mean;
                    } else {
                        double u1, u2;
                        site_uniforms3(seed, scene, ORC_TAG_INIT, 0u, real, H, W, x, y, z, &u1, &u2);
                        s[n] = (float)u1;
                    }
                }
            }
        }
    }
    for (int64_t n = 0; n < n_all; ++n) acc[n] = 0.0;
    int32_t k_cap = stop_mode != 0 ? n_max : n_eq;
    double* e_r = (double*)malloc(sizeof(double) * (size_t)R);
    double* ser = stop_mode == 2 ? (double*)malloc(sizeof(double) * (size_t)R * (size_t)(k_cap + 1)) : NULL;
    uint8_t* passed = stop_mode == 2 ? (uint8_t*)calloc((size_t)R, 1) : NULL;
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < R; ++r) e_r[r] = orc_energy3(state + (int64_t)r * n_all, D, H, W, q, J);
    double e0 = 0.0;
    for (int32_t r = 0; r < R; ++r) e0 += e_r[r];
    energy[0] = e0 / (double)R;
    if (ser)
        for (int32_t r = 0; r < R; ++r) ser[r] = e_r[r];
    int32_t k = 0;
    *converged = 1;
    while (k < k_cap) {
        ++k;
#pragma omp parallel for schedule(static)
        for (int32_t r = 0; r < R; ++r) {
            float* s = state + (int64_t)r * n_all;
            orc_sweep3(s, mask, D, H, W, T_blocks, lb_d, lb_h, lb_w, q, J, seed, scene, (uint32_t)(r + real_offset),
                       (uint32_t)k);
            e_r[r] = orc_energy3(s, D, H, W, q, J);
        }
        double ek = 0.0;
        for (int32_t r = 0; r < R; ++r) ek += e_r[r];
        energy[k] = ek / (double)R;
        if (ser)
            for (int32_t r = 0; r < R; ++r) ser[(int64_t)k * R + r] = e_r[r];
        if (stop_mode == 1 && orc_stop_check(energy, k, n_fit, n_f)) break;
        if (stop_mode == 2 && orc_stop_check_chains(ser, R, k, n_fit, n_f, passed)) break;
        if (stop_mode != 0 && k == n_max) *converged = 0;
    }
    free(ser);
    free(passed);
    int32_t k_star = k;
    for (int32_t s_i = 1; s_i <= n_samp; ++s_i) {
#pragma omp parallel for schedule(static)
        for (int32_t r = 0; r < R; ++r)
            orc_sweep3(state + (int64_t)r * n_all, mask, D, H, W, T_blocks, lb_d, lb_h, lb_w, q, J, seed, scene,
                       (uint32_t)(r + real_offset), (uint32_t)(k_star + s_i));
        for (int32_t r = 0; r < R; ++r) {
            const float* s = state + (int64_t)r * n_all;
            for (int64_t n = 0; n < n_all; ++n)
                if (!mask[n]) acc[n] += (double)s[n];
        }
    }
    free(e_r);
    free(S);
    free(N);
    free(Tsum);
    free(Nobs);
    return k_star;
}
