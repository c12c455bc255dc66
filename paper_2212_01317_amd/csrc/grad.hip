// Gradient of the realization-averaged prediction with respect to the block temperatures.
//
// For a density proportional to exp(-sum_b H_b / T_b) the derivative of an expectation is
// d<f>/dT_b = Cov(f, H_b) / T_b^2 (score function).  H_b is the part of Eq. (1) attributed to block b: every bond
// with at least one gap end, counted in the block of its gap end, one half in each block for a bond between two gaps
// of different blocks (bonds between samples are constant).  With one sampling sweep, E[zhat] = zmin + span E[t], so
// for a loss L(zhat) the estimate over R realizations is Cov_r(g_r, H_rb) / T_b^2 with g_r = sum_v w_v t_rv and
// w_v = dL/dzhat_v * span at gaps.  Everything here is FP64 and reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mpr_internal.hpp"

namespace mpr {

namespace {

template <class T>
__device__ __forceinline__ T wave_sum64(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double block_sum256(double v, double* lds)
{
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    __syncthreads();
    return s;
}

}  // namespace

// One workgroup per (block, chunk of block rows, realization): partial H over the gap sites of the chunk.
__global__ __launch_bounds__(256) void k_block_energy(const float* __restrict__ state, const uint8_t* __restrict__ mask,
                                                       StatsGeom g, double two_pi_q, double J, int64_t HW,
                                                       double* part /* [R][B * nchunk] */)
{
    __shared__ double lds[4];
    const int64_t wg = blockIdx.x;                // block * nchunk + chunk
    const int r = blockIdx.y;
    const int b = (int)(wg / g.nchunk), c = (int)(wg % g.nchunk);
    const int by = b / g.nbx, bx = b % g.nbx;
    const int64_t yb = (int64_t)by * g.lb_h;
    int64_t y0 = yb + (int64_t)c * g.G, y1 = yb + (int64_t)(c + 1) * g.G;
    if (y1 > yb + g.lb_h) y1 = yb + g.lb_h;
    if (y1 > g.H) y1 = g.H;
    const int64_t x0 = (int64_t)bx * g.lb_w;
    int64_t x1 = x0 + g.lb_w;
    if (x1 > g.W) x1 = g.W;
    const int64_t rows = y1 - y0, cols = x1 - x0;
    const float* s = state + (int64_t)r * HW;
    double acc = 0.0;
    if (rows > 0 && cols > 0) {
        for (int64_t i = threadIdx.x; i < rows * cols; i += 256) {
            const int64_t y = y0 + i / cols, x = x0 + i % cols;
            const int64_t n = y * g.W + x;
            if (mask[n]) continue;
            const double tn = (double)s[n];
            int64_t nb[4];
            int cnt = 0;
            if (y > 0) nb[cnt++] = n - g.W;
            if (x > 0) nb[cnt++] = n - 1;
            if (x + 1 < g.W) nb[cnt++] = n + 1;
            if (y + 1 < g.H) nb[cnt++] = n + g.W;
            for (int k = 0; k < cnt; ++k) {
                const double share = mask[nb[k]] ? 1.0 : 0.5;
                acc += share * (-J * cos(two_pi_q * (tn - (double)s[nb[k]])));
            }
        }
    }
    acc = block_sum256(acc, lds);
    if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + wg] = acc;
}

__global__ __launch_bounds__(256) void k_block_energy_final(const double* part, int64_t B, int nchunk, int R,
                                                             double* Hrb /* [R][B] */)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= B * R) return;
    const int64_t r = i / B, b = i % B;
    const double* p = part + r * B * nchunk + b * nchunk;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += p[c];
    Hrb[i] = s;
}

hipError_t launch_block_energy(const float* state, const uint8_t* mask, const StatsGeom& g, double two_pi_q,
                               double J, int R, double* part, double* Hrb, hipStream_t s)
{
    const int64_t nwg = g.B() * g.nchunk;
    hipLaunchKernelGGL(k_block_energy, dim3((unsigned)nwg, (unsigned)R), dim3(256), 0, s, state, mask, g, two_pi_q, J,
                       g.H * g.W, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = g.B() * R;
    hipLaunchKernelGGL(k_block_energy_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, g.B(), g.nchunk,
                       R, Hrb);
    return hipGetLastError();
}

// g_r = sum_v w_v t_rv with w_v = grad_zhat_v * span at gaps: one workgroup per (realization, part of the grid),
// then the parts of a realization are summed in order.
__global__ __launch_bounds__(256) void k_grad_g_part(const float* __restrict__ state, const float* __restrict__ gz,
                                                      const uint8_t* __restrict__ mask, int64_t HW,
                                                      const double* __restrict__ range, double* part /* [R][P] */)
{
    __shared__ double lds[4];
    const int r = blockIdx.y;
    const int P = gridDim.x;
    const double span = range[1] - range[0];
    const float* s = state + (int64_t)r * HW;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < HW; n += (int64_t)P * 256) {
        if (mask[n]) continue;
        acc += ((double)gz[n] * span) * (double)s[n];
    }
    acc = block_sum256(acc, lds);
    if (threadIdx.x == 0) part[(int64_t)r * P + blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_grad_g_final(const double* part, int P, int R, double* g)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += part[(int64_t)r * P + p];
    g[r] = s;
}

// dT_b = [sum_r (g_r - mean g)(H_rb - mean H_b) / (R - 1)] / T_b^2 (0 when T_b = 0).
__global__ __launch_bounds__(256) void k_grad_cov(const double* g, const double* Hrb, int R, int64_t B,
                                                   const float* T_blocks, double* dT)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    double gm = 0.0, hm = 0.0;
    for (int r = 0; r < R; ++r) {
        gm += g[r];
        hm += Hrb[(int64_t)r * B + b];
    }
    gm /= (double)R;
    hm /= (double)R;
    double cov = 0.0;
    for (int r = 0; r < R; ++r) cov += (g[r] - gm) * (Hrb[(int64_t)r * B + b] - hm);
    cov /= (double)(R - 1);
    const double T = (double)T_blocks[b];
    dT[b] = T > 0.0 ? cov / (T * T) : 0.0;
}

int grad_parts(int64_t HW)
{
    int64_t p = (HW + 256 * 16 - 1) / (256 * 16);
    return (int)(p < 1 ? 1 : (p > 256 ? 256 : p));
}

hipError_t launch_temperature_grad(const float* state, const double* Hrb, const float* gz, const uint8_t* mask,
                                   int64_t HW, int R, int64_t B, const double* range, const float* T_blocks,
                                   double* part, double* g, double* dT, hipStream_t s)
{
    const int P = grad_parts(HW);
    hipLaunchKernelGGL(k_grad_g_part, dim3((unsigned)P, (unsigned)R), dim3(256), 0, s, state, gz, mask, HW, range,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_g_final, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, part, P, R, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_cov, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, g, Hrb, R, B, T_blocks, dT);
    return hipGetLastError();
}

}  // namespace mpr
