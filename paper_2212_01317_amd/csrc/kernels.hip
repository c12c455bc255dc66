// gfx950 kernels of the SV-MPR conditional simulation (Lach & Zukovic, arXiv 2212.01317).
//
// Built with -ffp-contract=off: every FP64 expression that must reproduce the published-formula arithmetic
// (map, bond energies, the exact Metropolis decision, prediction) is evaluated exactly as written; the FP32 hot
// path uses explicit fmaf where a fused multiply-add is wanted.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "metropolis.hpp"

namespace mpr {

// ------------------------------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of one value per thread over a workgroup of NT threads; result valid in thread 0.  Fixed order.
template <int NT, class T>
__device__ __forceinline__ T block_sum(T v, T* lds /* NT / 64 entries */)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------------------------------------------------
// Sec. 2.1: linear map of the samples onto angles
// ------------------------------------------------------------------------------------------------------------
constexpr int MAP_NT = 256;

int map_reduce_blocks(int64_t n)
{
    int64_t b = (n + (int64_t)MAP_NT * 16 - 1) / ((int64_t)MAP_NT * 16);
    return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

__global__ __launch_bounds__(MAP_NT) void k_map_reduce(const float* __restrict__ z, const uint8_t* __restrict__ mask,
                                                        int64_t n, float* pmin, float* pmax, unsigned long long* pcnt,
                                                        unsigned long long* pbad)
{
    __shared__ float smn[MAP_NT], smx[MAP_NT];
    __shared__ unsigned long long sc[MAP_NT], sb[MAP_NT];
    float mn = INFINITY, mx = -INFINITY;
    unsigned long long cnt = 0, bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * MAP_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MAP_NT) {
        if (mask[i]) {
            const float v = z[i];
            if (isfinite(v)) {
                mn = fminf(mn, v);
                mx = fmaxf(mx, v);
            } else {
                ++bad;
            }
            ++cnt;
        }
    }
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    sc[threadIdx.x] = cnt;
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int s = MAP_NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smn[threadIdx.x] = fminf(smn[threadIdx.x], smn[threadIdx.x + s]);
            smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + s]);
            sc[threadIdx.x] += sc[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmin[blockIdx.x] = smn[0];
        pmax[blockIdx.x] = smx[0];
        pcnt[blockIdx.x] = sc[0];
        pbad[blockIdx.x] = sb[0];
    }
}

__global__ __launch_bounds__(MAP_NT) void k_map_finalize(const float* pmin, const float* pmax,
                                                          const unsigned long long* pcnt,
                                                          const unsigned long long* pbad, int nblocks, double* range,
                                                          unsigned long long* counts)
{
    __shared__ float smn[MAP_NT], smx[MAP_NT];
    __shared__ unsigned long long sc[MAP_NT], sb[MAP_NT];
    float mn = INFINITY, mx = -INFINITY;
    unsigned long long cnt = 0, bad = 0;
    for (int i = threadIdx.x; i < nblocks; i += MAP_NT) {
        mn = fminf(mn, pmin[i]);
        mx = fmaxf(mx, pmax[i]);
        cnt += pcnt[i];
        bad += pbad[i];
    }
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    sc[threadIdx.x] = cnt;
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int s = MAP_NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smn[threadIdx.x] = fminf(smn[threadIdx.x], smn[threadIdx.x + s]);
            smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + s]);
            sc[threadIdx.x] += sc[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        range[0] = (double)smn[0];
        range[1] = (double)smx[0];
        counts[0] = sc[0];
        counts[1] = sb[0];
    }
}

__global__ __launch_bounds__(MAP_NT) void k_map_apply(const float* __restrict__ z, const uint8_t* __restrict__ mask,
                                                       int64_t n, const double* __restrict__ range,
                                                       float* __restrict__ t)
{
    const int64_t i = (int64_t)blockIdx.x * MAP_NT + threadIdx.x;
    if (i >= n) return;
    const double zmin = range[0];
    const double span = range[1] - range[0];
    float v = 0.0f;
    if (mask[i] && span != 0.0) v = (float)(((double)z[i] - zmin) / span);
    t[i] = v;
}

hipError_t launch_map_reduce(const float* z, const uint8_t* mask, int64_t n, float* pmin, float* pmax,
                             unsigned long long* pcnt, unsigned long long* pbad, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_map_reduce, dim3(nblocks), dim3(MAP_NT), 0, s, z, mask, n, pmin, pmax, pcnt, pbad);
    return hipGetLastError();
}

hipError_t launch_map_finalize(const float* pmin, const float* pmax, const unsigned long long* pcnt,
                               const unsigned long long* pbad, int nblocks, double* range, unsigned long long* counts,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_map_finalize, dim3(1), dim3(MAP_NT), 0, s, pmin, pmax, pcnt, pbad, nblocks, range, counts);
    return hipGetLastError();
}

hipError_t launch_map_apply(const float* z, const uint8_t* mask, int64_t n, const double* range, float* t,
                            hipStream_t s)
{
    const int64_t nb = (n + MAP_NT - 1) / MAP_NT;
    hipLaunchKernelGGL(k_map_apply, dim3((unsigned)nb), dim3(MAP_NT), 0, s, z, mask, n, range, t);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Eq. (2) per T-block (Sec. 2.2.2): sample-bond energies and counts, sample-angle sums and counts.
// One workgroup per (block, chunk of block rows); a second pass sums the chunks of a block in order.
// ------------------------------------------------------------------------------------------------------------
constexpr int STATS_NT = 256;

StatsGeom stats_geom(int64_t H, int64_t W, int lb_h, int lb_w)
{
    StatsGeom g;
    g.H = H;
    g.W = W;
    g.lb_h = lb_h;
    g.lb_w = lb_w;
    g.nbx = (int)((W + lb_w - 1) / lb_w);
    g.nby = (int)((H + lb_h - 1) / lb_h);
    const int64_t ew = lb_w < W ? lb_w : W;
    const int64_t eh = lb_h < H ? lb_h : H;
    int64_t G = 4096 / ew;
    if (G < 1) G = 1;
    if (G > eh) G = eh;
    g.G = (int)G;
    g.nchunk = (int)((eh + G - 1) / G);
    return g;
}

__global__ __launch_bounds__(STATS_NT) void k_block_stats(const float* __restrict__ t,
                                                           const uint8_t* __restrict__ mask, StatsGeom g,
                                                           double two_pi_q, double J, int bonds, double* pS,
                                                           int* pN, double* pTs, int* pNo)
{
    __shared__ double lds_d[STATS_NT / 64];
    __shared__ int lds_i[STATS_NT / 64];
    const int b = blockIdx.x / g.nchunk, c = blockIdx.x % g.nchunk;
    const int by = b / g.nbx, bx = b % g.nbx;
    const int64_t yb = (int64_t)by * g.lb_h;
    int64_t y_start = yb + (int64_t)c * g.G;
    int64_t y_end = yb + (int64_t)(c + 1) * g.G;
    if (y_end > yb + g.lb_h) y_end = yb + g.lb_h;
    if (y_end > g.H) y_end = g.H;
    const int64_t x_start = (int64_t)bx * g.lb_w;
    int64_t x_end = x_start + g.lb_w;
    if (x_end > g.W) x_end = g.W;
    const int64_t rows = y_end - y_start, cols = x_end - x_start;
    double S = 0.0, Ts = 0.0;
    int N = 0, No = 0;
    if (rows > 0 && cols > 0) {
        for (int64_t i = threadIdx.x; i < rows * cols; i += STATS_NT) {
            const int64_t y = y_start + i / cols, x = x_start + i % cols;
            const int64_t n = y * g.W + x;
            if (!mask[n]) continue;
            const double tn = (double)t[n];
            Ts += tn;
            ++No;
            if ((bonds & 1) && x + 1 < g.W && mask[n + 1]) {
                S += -J * cos(two_pi_q * (tn - (double)t[n + 1]));
                ++N;
            }
            if ((bonds & 2) && y + 1 < g.H && mask[n + g.W]) {
                S += -J * cos(two_pi_q * (tn - (double)t[n + g.W]));
                ++N;
            }
        }
    }
    S = block_sum<STATS_NT>(S, lds_d);
    Ts = block_sum<STATS_NT>(Ts, lds_d);
    N = block_sum<STATS_NT>(N, lds_i);
    No = block_sum<STATS_NT>(No, lds_i);
    if (threadIdx.x == 0) {
        pS[blockIdx.x] = S;
        pN[blockIdx.x] = N;
        pTs[blockIdx.x] = Ts;
        pNo[blockIdx.x] = No;
    }
}

__global__ __launch_bounds__(256) void k_block_stats_final(const double* pS, const int* pN, const double* pTs,
                                                            const int* pNo, int64_t B, int nchunk, double* S, int* N,
                                                            double* Ts, int* No)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    double s = 0.0, ts = 0.0;
    int nn = 0, no = 0;
    for (int c = 0; c < nchunk; ++c) {
        const int64_t i = b * nchunk + c;
        s += pS[i];
        nn += pN[i];
        ts += pTs[i];
        no += pNo[i];
    }
    if (S) S[b] = s;
    if (N) N[b] = nn;
    if (Ts) Ts[b] = ts;
    if (No) No[b] = no;
}

hipError_t launch_block_stats(const float* t, const uint8_t* mask, const StatsGeom& g, double two_pi_q, double J,
                              double* pS, int* pN, double* pTs, int* pNo, double* S, int* N, double* Ts, int* No,
                              hipStream_t s, int bonds)
{
    const int64_t B = g.B();
    const int64_t nwg = B * g.nchunk;
    hipLaunchKernelGGL(k_block_stats, dim3((unsigned)nwg), dim3(STATS_NT), 0, s, t, mask, g, two_pi_q, J, bonds, pS,
                       pN, pTs, pNo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_block_stats_final, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, pS, pN, pTs, pNo, B,
                       g.nchunk, S, N, Ts, No);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Energy matching (Sec. 2.1, Sec. 2.2.2): inverse of the matching curve, median fill of blocks without bonds.
// ------------------------------------------------------------------------------------------------------------
__device__ double curve_inverse(double e, const double* cT, const double* ce, int n)
{
    if (e <= -1.0) return 0.0;
    double prev = ce[0];
    if (e <= prev) {
        const double denom = prev + 1.0;
        return denom > 0.0 ? cT[0] * (e + 1.0) / denom : cT[0];
    }
    for (int i = 1; i < n; ++i) {
        const double cur = ce[i] > prev ? ce[i] : prev;
        if (cur >= e) {
            if (cur == prev) return cT[i];
            const double lam = (e - prev) / (cur - prev);
            return exp((1.0 - lam) * log(cT[i - 1]) + lam * log(cT[i]));
        }
        prev = cur;
    }
    return cT[n - 1];
}

__global__ __launch_bounds__(256) void k_calibrate(const double* S, const int* N, int64_t B, double J,
                                                    const double* cT, const double* ce, int nc, float* T_out,
                                                    double* e_out, int* nb_out)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    const int nb = N[b];
    double e = 0.0;
    float T = -1.0f;   // marker: filled by the median pass
    if (nb > 0) {
        e = S[b] / (J * (double)nb);
        T = (float)(J * curve_inverse(e, cT, ce, nc));
    }
    T_out[b] = T;
    if (e_out) e_out[b] = e;
    if (nb_out) nb_out[b] = nb;
}

constexpr int MED_NT = 1024;

// k-th smallest (0-based) of the T values of blocks with N > 0, by a 4-pass 8-bit radix select on the FP32 bit
// patterns (T >= 0, so the bit patterns are ordered like the values).
__device__ float radix_select(const float* T, const int* N, int64_t B, unsigned k, unsigned* hist, unsigned* sh)
{
    unsigned prefix = 0u, pmask = 0u;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += MED_NT) hist[i] = 0u;
        __syncthreads();
        for (int64_t b = threadIdx.x; b < B; b += MED_NT) {
            if (N[b] > 0) {
                const unsigned key = __float_as_uint(T[b]);
                if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned cum = 0u, d = 0u;
            for (d = 0u; d < 256u; ++d) {
                if (cum + hist[d] > k) break;
                cum += hist[d];
            }
            sh[0] = prefix | (d << shift);
            sh[1] = k - cum;
        }
        __syncthreads();
        prefix = sh[0];
        k = sh[1];
        pmask |= 255u << shift;
        __syncthreads();
    }
    return __uint_as_float(prefix);
}

__global__ __launch_bounds__(MED_NT) void k_median_fill(float* T, const int* N, int64_t B, unsigned* n_have)
{
    __shared__ unsigned hist[256];
    __shared__ unsigned sh[2];
    __shared__ unsigned scount[MED_NT / 64];
    unsigned cnt = 0;
    for (int64_t b = threadIdx.x; b < B; b += MED_NT) cnt += N[b] > 0 ? 1u : 0u;
    cnt = block_sum<MED_NT>(cnt, scount);
    if (threadIdx.x == 0) sh[0] = cnt;
    __syncthreads();
    const unsigned count = sh[0];
    __syncthreads();
    if (threadIdx.x == 0) *n_have = count;
    if (count == 0u) return;
    const float lo = radix_select(T, N, B, (count - 1u) / 2u, hist, sh);
    float med = lo;
    if ((count & 1u) == 0u) {
        const float hi = radix_select(T, N, B, count / 2u, hist, sh);
        med = (float)(((double)lo + (double)hi) * 0.5);
    }
    for (int64_t b = threadIdx.x; b < B; b += MED_NT)
        if (N[b] == 0) T[b] = med;
}

hipError_t launch_calibrate(const double* S, const int* N, int64_t B, double J, const double* cT, const double* ce,
                            int nc, float* T_out, double* e_out, int* nb_out, unsigned* n_have, hipStream_t s)
{
    hipLaunchKernelGGL(k_calibrate, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, S, N, B, J, cT, ce, nc,
                       T_out, e_out, nb_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_median_fill, dim3(1), dim3(MED_NT), 0, s, T_out, N, B, n_have);
    return hipGetLastError();
}

// One wave: the block sums are read 64 at a time (one coalesced load per lane) and added in block order from the
// lanes' registers (reads of fixed lanes, independent of the sum), one sequential FP64 sum with the rounding of a loop
// over the blocks (a loop of single loads waited for each load in turn).
__global__ __launch_bounds__(64) void k_global_mean(const double* Ts, const int* No, int64_t B, float* gmean)
{
    if (blockIdx.x != 0) return;
    const int lane = (int)threadIdx.x;
    double sum = 0.0;
    long long cnt = 0;
    for (int64_t b0 = 0; b0 < B; b0 += 64) {
        const int64_t b = b0 + lane;
        const double t = b < B ? Ts[b] : 0.0;
        const int n = b < B ? No[b] : 0;
        const int tlo = __double2loint(t), thi = __double2hiint(t);
        const int m = B - b0 < 64 ? (int)(B - b0) : 64;
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            if (j < m) {
                sum += __hiloint2double(__builtin_amdgcn_readlane(thi, j), __builtin_amdgcn_readlane(tlo, j));
                cnt += __builtin_amdgcn_readlane(n, j);
            }
        }
    }
    if (lane == 0) *gmean = cnt > 0 ? (float)(sum / (double)cnt) : 0.0f;
}

hipError_t launch_global_mean(const double* Ts, const int* No, int64_t B, float* gmean, hipStream_t s)
{
    hipLaunchKernelGGL(k_global_mean, dim3(1), dim3(64), 0, s, Ts, No, B, gmean);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_tpairs(const float* T, int64_t B, float J, float delta, TBand* tp)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    tp[b] = make_tband(T[b], J, delta);
}

hipError_t launch_tpairs(const float* T, int64_t B, float J, float delta, TBand* tp, hipStream_t s)
{
    hipLaunchKernelGGL(k_tpairs, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, T, B, J, delta, tp);
    return hipGetLastError();
}

// Directional coupling: per block {Tx, Ty} from T[b], T[B + b] raised to at least `floor`, the scales
// kx = J log2(e) / Tx, ky = J log2(e) / Ty of the two field components and the error band of the filter.
__global__ __launch_bounds__(256) void k_tpairs_directional(const float* __restrict__ T, int64_t B, float J,
                                                             float delta, float floor_T, TBandDir* __restrict__ out)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    out[b] = make_tband_directional(fmaxf(T[b], floor_T), fmaxf(T[B + b], floor_T), J, delta);
}

hipError_t launch_tpairs_directional(const float* T, int64_t B, float J, float delta, float floor_T, TBandDir* out,
                                     hipStream_t s)
{
    hipLaunchKernelGGL(k_tpairs_directional, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, T, B, J, delta,
                       floor_T, out);
    return hipGetLastError();
}

// out[i] = max(T[i], floor_T)
__global__ __launch_bounds__(256) void k_floor(float* __restrict__ T, int64_t n, float floor_T)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) T[i] = fmaxf(T[i], floor_T);
}

hipError_t launch_floor(float* T, int64_t n, float floor_T, hipStream_t s)
{
    hipLaunchKernelGGL(k_floor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, n, floor_T);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Start of the chains (Sec. 3.3): block means of the sample angles (SV-MPR) or uniform draws (MPR).
// ------------------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(InitArgs a)
{
    const int64_t HW = a.H * a.W;
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (n >= HW) return;
    const int64_t y = n / a.W, x = n % a.W;
    float v;
    if (a.mask[n]) {
        v = a.t[n];
    } else if (a.mode == 1) {
        const int64_t b = (y / a.lb_h) * a.nbx + (x / a.lb_w);
        v = a.No[b] > 0 ? (float)(a.Ts[b] / (double)a.No[b]) : *a.gmean;
    } else {
        const uint32_t Mw = (uint32_t)((a.W + 3) / 4);
        const uint32_t pair = (uint32_t)y * Mw + (uint32_t)(x >> 2);
        const uint32_t colour = (uint32_t)((x + y) & 1);
        const U4 w = philox4x32_10(pair, 0u, a.real_offset + (uint32_t)r, ctr_word3(a.scene, TAG_INIT, colour),
                                   a.key0, a.key1);
        v = u24(((x >> 1) & 1) ? w.z : w.x);
    }
    a.state[(int64_t)r * HW + n] = v;
    if (a.state2) a.state2[(int64_t)r * HW + n] = v;
}

hipError_t launch_init(const InitArgs& a, hipStream_t s)
{
    const int64_t HW = a.H * a.W;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((HW + 255) / 256), (unsigned)a.R), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Whole-grid energy of the current states (used for e(0)): every site's right and lower bond, FP32 terms,
// FP64 per-workgroup sums.  partial layout [R][part].
constexpr int EN_NT = 256;

int energy_full_parts(int64_t H, int64_t W)
{
    const int64_t HW = H * W;
    int64_t p = (HW + EN_NT * 8 - 1) / (EN_NT * 8);
    return (int)(p < 1 ? 1 : (p > 4096 ? 4096 : p));
}

__device__ __forceinline__ int fix24(float x) { return __float2int_rn(x * 16777216.0f); }

__global__ __launch_bounds__(EN_NT) void k_energy_full(const float* __restrict__ state, int64_t H, int64_t W, float q,
                                                        float J, long long* partial)
{
    __shared__ long long s_red[EN_NT / 64];
    (void)J;
    const int r = blockIdx.y;
    const int64_t HW = H * W;
    const float* st = state + (int64_t)r * HW;
    long long acc = 0;
    for (int64_t n = (int64_t)blockIdx.x * EN_NT + threadIdx.x; n < HW; n += (int64_t)gridDim.x * EN_NT) {
        const int64_t y = n / W, x = n - y * W;
        const float tn = st[n];
        float e = 0.0f;                                   // energy of the site's right and lower bonds / J
        if (x + 1 < W) e -= cos_rev(q * (tn - st[n + 1]));
        if (y + 1 < H) e -= cos_rev(q * (tn - st[n + W]));
        acc += fix24(e);
    }
    const long long tot = block_sum<EN_NT>(acc, s_red);
    if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = tot;
}

hipError_t launch_energy_full(const float* state, int64_t H, int64_t W, int R, float q, float J, long long* partial,
                              int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_full, dim3((unsigned)nparts, (unsigned)R), dim3(EN_NT), 0, s, state, H, W, q, J,
                       partial);
    return hipGetLastError();
}

// e_real[r] = (sum over parts of partial[r][p]) * unit * inv_norm (integer sum: order-free), one workgroup per
// realization; then e_out = mean over realizations (in order).
__global__ __launch_bounds__(256) void k_energy_real(const long long* __restrict__ partial, int nparts,
                                                      double inv_norm, double* e_real)
{
    __shared__ long long s_red[4];
    const int r = blockIdx.x;
    const long long* row = partial + (int64_t)r * nparts;
    long long s = 0;
    for (int p = threadIdx.x; p < nparts; p += 256) s += row[p];
    s = block_sum<256>(s, s_red);
    if (threadIdx.x == 0) e_real[r] = ((double)s * kFixUnit) * inv_norm;
}

__global__ void k_energy_mean(const double* e_real, int R, double* e_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += e_real[r];
    *e_out = s / (double)R;
}

hipError_t launch_energy_reduce(const long long* partial, int nparts, int R, double inv_norm, double* e_real,
                                double* e_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_real, dim3((unsigned)R), dim3(256), 0, s, partial, nparts, inv_norm, e_real);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_mean, dim3(1), dim3(64), 0, s, e_real, R, e_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Sampling (Sec. 2.1): acc[n] += sum over realizations (in order) of the gap angle; first pass starts from 0.
// ------------------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accumulate(const float* __restrict__ state, const uint8_t* __restrict__ mask,
                                                     int64_t HW, int R, int first, double* __restrict__ acc)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= HW) return;
    if (mask[n]) {
        if (first) acc[n] = 0.0;
        return;
    }
    double a = first ? 0.0 : acc[n];
    for (int r = 0; r < R; ++r) a += (double)state[(int64_t)r * HW + n];
    acc[n] = a;
}

hipError_t launch_accumulate(const float* state, const uint8_t* mask, int64_t HW, int R, int first, double* acc,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, state, mask, HW, R, first,
                       acc);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Back-transform of the conditional mean (Sec. 2.1) and the validation measures (Eq. 3, Eq. 4).
// ------------------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_predict(const double* __restrict__ acc, const float* __restrict__ z,
                                                  const uint8_t* __restrict__ mask, int64_t n, int64_t n_samples,
                                                  const double* __restrict__ range, float* __restrict__ zhat)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (mask[i]) {
        zhat[i] = z[i];
        return;
    }
    const double zmin = range[0], span = range[1] - range[0];
    const double tbar = acc[i] / (double)n_samples;
    zhat[i] = (float)(zmin + span * tbar);
}

hipError_t launch_predict(const double* acc, const float* z, const uint8_t* mask, int64_t n, int64_t n_samples,
                          const double* range, float* zhat, hipStream_t s)
{
    hipLaunchKernelGGL(k_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc, z, mask, n, n_samples,
                       range, zhat);
    return hipGetLastError();
}

constexpr int VAL_NT = 256;

int validate_blocks(int64_t n)
{
    int64_t b = (n + VAL_NT * 16 - 1) / (VAL_NT * 16);
    return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

__global__ __launch_bounds__(VAL_NT) void k_validate_part(const float* __restrict__ zhat,
                                                           const float* __restrict__ truth,
                                                           const uint8_t* __restrict__ ev, int64_t n, double* part)
{
    __shared__ double s_red[VAL_NT / 64];
    double sa = 0.0, s2 = 0.0, cnt = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * VAL_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VAL_NT) {
        if (!ev[i]) continue;
        const double e = (double)truth[i] - (double)zhat[i];
        sa += fabs(e);
        s2 += e * e;
        cnt += 1.0;
    }
    sa = block_sum<VAL_NT>(sa, s_red);
    s2 = block_sum<VAL_NT>(s2, s_red);
    cnt = block_sum<VAL_NT>(cnt, s_red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = sa;
        part[3 * blockIdx.x + 1] = s2;
        part[3 * blockIdx.x + 2] = cnt;
    }
}

__global__ void k_validate_final(const double* part, int nblocks, double* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sa = 0.0, s2 = 0.0, cnt = 0.0;
    for (int i = 0; i < nblocks; ++i) {
        sa += part[3 * i];
        s2 += part[3 * i + 1];
        cnt += part[3 * i + 2];
    }
    out[0] = cnt > 0.0 ? sa / cnt : 0.0;
    out[1] = cnt > 0.0 ? sqrt(s2 / cnt) : 0.0;
}

hipError_t launch_validate(const float* zhat, const float* truth, const uint8_t* ev, int64_t n, double* part,
                           int nblocks, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_validate_part, dim3(nblocks), dim3(VAL_NT), 0, s, zhat, truth, ev, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_validate_final, dim3(1), dim3(64), 0, s, part, nblocks, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Matching curve: the unconditional MPR model on a periodic L x L lattice, one chain per temperature.
// ------------------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ref_fill(float* state, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) state[i] = v;
}

hipError_t launch_ref_fill(float* state, int64_t n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(k_ref_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, state, n, v);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ref_half(RefArgs a)
{
    const int chain = blockIdx.y;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int L = a.L;
    if (p >= L * a.Mw) return;
    const int y = p / a.Mw, m = p - y * a.Mw;
    const int xa = 4 * m + ((y + a.colour) & 1);
    if (xa >= L) return;
    float* st = a.state + (int64_t)chain * L * L;
    const float T = a.Tgrid[chain];
    const TBand tb = make_tband(T, 1.0f, a.delta_e);
    const U4 w = philox_x3((uint32_t)p, a.sweep, (uint32_t)chain, ctr_word3(0u, TAG_REFLAT, a.colour), a.key0,
                               a.key1);
    const int yu = (y + L - 1) % L, yd = (y + 1) % L;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int x = xa + 2 * h;
        if (x >= L) break;
        const int xl = (x + L - 1) % L, xr = (x + 1) % L;
        float nb[4];
        nb[0] = st[yu * L + x];
        nb[1] = st[y * L + xl];
        nb[2] = st[y * L + xr];
        nb[3] = st[yd * L + x];
        float Cx = 0.0f, Sy = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float ang = a.q * nb[j];
            Cx += cos_rev(ang);
            Sy += sin_rev(ang);
        }
        const float to = st[y * L + x];
        const float co = cos_rev(a.q * to), so = sin_rev(a.q * to);
        const float tpv = u24(h ? w.z : w.x);
        const uint32_t wa = h ? w.w : w.y;
        const float u2 = u24(wa);
        const float cp = cos_rev(a.q * tpv), sp = sin_rev(a.q * tpv);
        const float X = fmaf(cp - co, Cx, (sp - so) * Sy);
        int dec = filter32(X, (float)(wa >> 8), tb, 1.0f, a.delta_e);
        if (dec < 0) dec = exact64(tpv, to, nb[0], nb[1], nb[2], nb[3], 15u, a.two_pi_q, 1.0, T, u2) ? 1 : 0;
        if (dec) st[y * L + x] = tpv;
    }
}

hipError_t launch_ref_half(const RefArgs& a, int nT, hipStream_t s)
{
    const int np = a.L * a.Mw;
    hipLaunchKernelGGL(k_ref_half, dim3((unsigned)((np + 255) / 256), (unsigned)nT), dim3(256), 0, s, a);
    return hipGetLastError();
}

int ref_energy_parts(int L)
{
    const int64_t n = (int64_t)L * L;
    int64_t p = (n + 256 * 8 - 1) / (256 * 8);
    return (int)(p < 1 ? 1 : (p > 1024 ? 1024 : p));
}

__global__ __launch_bounds__(256) void k_ref_energy(const float* __restrict__ state, int L, float q, double* partial)
{
    __shared__ double s_red[4];
    const int chain = blockIdx.y;
    const float* st = state + (int64_t)chain * L * L;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < (int64_t)L * L; n += (int64_t)gridDim.x * 256) {
        const int y = (int)(n / L), x = (int)(n - (int64_t)y * L);
        const float tn = st[n];
        const float e = -cos_rev(q * (tn - st[y * L + (x + 1) % L])) - cos_rev(q * (tn - st[((y + 1) % L) * L + x]));
        acc += (double)e;
    }
    const double tot = block_sum<256>(acc, s_red);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * gridDim.y + chain] = tot;
}

hipError_t launch_ref_energy(const float* state, int L, int nT, float q, double* partial, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_ref_energy, dim3((unsigned)nparts, (unsigned)nT), dim3(256), 0, s, state, L, q, partial);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ref_accumulate(const double* partial, int nparts, int nT, double inv_norm,
                                                         double* e_sum, int first)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nT) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += partial[(int64_t)p * nT + i];
    const double e = s * inv_norm;
    e_sum[i] = first ? e : e_sum[i] + e;
}

hipError_t launch_ref_accumulate(const double* partial, int nparts, int nT, double inv_norm, double* e_sum, int first,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_ref_accumulate, dim3((unsigned)((nT + 255) / 256)), dim3(256), 0, s, partial, nparts, nT,
                       inv_norm, e_sum, first);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ref_finish(const double* e_sum, int nT, double n_meas, double* e_out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nT) return;
    e_out[i] = n_meas > 0.0 ? e_sum[i] / n_meas : 0.0;
}

hipError_t launch_ref_finish(const double* e_sum, int nT, double n_meas, double* e_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_ref_finish, dim3((unsigned)((nT + 255) / 256)), dim3(256), 0, s, e_sum, nT, n_meas, e_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------------------
// Sec. 2.2.3 (SST): the block map spread to the sites, then n_s passes of the mean over the (2 r_s + 1)^2 square
// around each site cut at the grid edges, in FP64 with the window summed row by row from the top left (the oracle's
// order), one rounding to FP32 at the end.
__global__ __launch_bounds__(256) void k_sst_spread(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h,
                                                    int32_t lb_w, double* a)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= H * W) return;
    const int64_t y = n / W, x = n - y * W, nbx = (W + lb_w - 1) / lb_w;
    a[n] = (double)T_blocks[(y / lb_h) * nbx + (x / lb_w)];
}

__global__ __launch_bounds__(256) void k_sst_pass(const double* __restrict__ a, double* __restrict__ b, int64_t H,
                                                  int64_t W, int32_t r)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= H * W) return;
    const int64_t y = n / W, x = n - y * W;
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t yy = y - r; yy <= y + r; ++yy) {
        if (yy < 0 || yy >= H) continue;
        for (int64_t xx = x - r; xx <= x + r; ++xx) {
            if (xx < 0 || xx >= W) continue;
            sum += a[yy * W + xx];
            ++cnt;
        }
    }
    b[n] = sum / (double)cnt;
}

__global__ __launch_bounds__(256) void k_sst_round(const double* a, int64_t n, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)a[i];
}

hipError_t launch_sst(const float* T_blocks, int64_t H, int64_t W, int32_t lb_h, int32_t lb_w, int32_t r_s,
                      int32_t n_s, double* a, double* b, float* out, hipStream_t s)
{
    const int64_t n = H * W;
    const dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_sst_spread, grid, dim3(256), 0, s, T_blocks, H, W, lb_h, lb_w, a);
    hipError_t e = hipGetLastError();
    for (int32_t p = 0; p < n_s && e == hipSuccess; ++p) {
        hipLaunchKernelGGL(k_sst_pass, grid, dim3(256), 0, s, a, b, H, W, r_s);
        e = hipGetLastError();
        double* tmp = a;
        a = b;
        b = tmp;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sst_round, grid, dim3(256), 0, s, a, n, out);
    return hipGetLastError();
}

}  // namespace mpr
