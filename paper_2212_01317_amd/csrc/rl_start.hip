// The start of the chains (Sec. 3.3: samples keep their angles, gaps the block mean of the samples or a uniform
// draw) and the whole-grid energy of the start, in the realization-lane layout: a wave handles one site of one group
// of 64 realizations at a time (each lane one realization, so that the writes and reads of a site are one 256-byte
// access) and walks the sites with a grid stride.  The
// values and the per-site energy terms are those of k_init and k_energy_full.
#include <hip/hip_runtime.h>

#include "metropolis.hpp"
#include "mpr_internal.hpp"
#include "philox.hpp"
#include "rl_start.hpp"

namespace mpr {

namespace {

__device__ __forceinline__ int fix24(float x) { return __float2int_rn(x * 16777216.0f); }

__global__ __launch_bounds__(256) void k_rl_init(InitArgs a, float* __restrict__ out0, float* __restrict__ out1)
{
    const int64_t HW = a.H * a.W;
    const int g = blockIdx.y, l = threadIdx.x & 63;
    const int r = g * 64 + l;
    // the site is the same for the whole wave: its row and column on the scalar unit, in 32 bits (H W < 2^32)
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t n = (int64_t)blockIdx.x * 4 + wv; n < HW; n += (int64_t)gridDim.x * 4) {
        const uint32_t nu = (uint32_t)n, Wu = (uint32_t)a.W;
        const int64_t y = nu / Wu, x = nu - (uint32_t)y * Wu;
        float v = 0.0f;
        if (r < a.R) {
            if (a.mask[n]) {
                v = a.t[n];
            } else if (a.mode == 1) {
                const int64_t b = (y / a.lb_h) * a.nbx + (x / a.lb_w);
                v = a.No[b] > 0 ? (float)(a.Ts[b] / (double)a.No[b]) : *a.gmean;
            } else {
                const uint32_t Mw = (uint32_t)((a.W + 3) / 4);
                const uint32_t pair = (uint32_t)y * Mw + (uint32_t)(x >> 2);
                const uint32_t colour = (uint32_t)((x + y) & 1);
                const U4 w = philox4x32_10(pair, 0u, a.real_offset + (uint32_t)r,
                                           ctr_word3(a.scene, TAG_INIT, colour), a.key0, a.key1);
                v = u24(((x >> 1) & 1) ? w.z : w.x);
            }
        }
        const int64_t o = ((int64_t)g * HW + n) * 64 + l;
        out0[o] = v;
        out1[o] = v;
    }
}

// each wave walks sites (a grid stride), each lane sums its realization's terms; the four waves of a workgroup
// then add their lanes' sums
__global__ __launch_bounds__(256) void k_rl_energy_full(const float* __restrict__ lanes, int64_t H, int64_t W, int R,
                                                        float q, long long* __restrict__ partial)
{
    __shared__ long long s_red[4][64];
    const int64_t HW = H * W;
    const int g = blockIdx.y, l = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const float* st = lanes + (int64_t)g * HW * 64 + l;
    long long acc = 0;
    for (int64_t n = (int64_t)blockIdx.x * 4 + wv; n < HW; n += (int64_t)gridDim.x * 4) {
        const uint32_t nu = (uint32_t)n, Wu = (uint32_t)W;
        const int64_t y = nu / Wu, x = nu - (uint32_t)y * Wu;     // on the scalar unit, in 32 bits (H W < 2^32)
        const float tn = st[n * 64];
        float e = 0.0f;                                   // energy of the site's right and lower bonds / J
        if (x + 1 < W) e -= cos_rev(q * (tn - st[(n + 1) * 64]));
        if (y + 1 < H) e -= cos_rev(q * (tn - st[(n + W) * 64]));
        acc += fix24(e);
    }
    s_red[wv][l] = acc;
    __syncthreads();
    const int r = g * 64 + l;
    if (wv == 0 && r < R)
        partial[(int64_t)r * gridDim.x + blockIdx.x] = s_red[0][l] + s_red[1][l] + s_red[2][l] + s_red[3][l];
}

// rows 1 .. R - 1 of partial[R][nparts] from row 0
__global__ __launch_bounds__(256) void k_rows_from_first(long long* __restrict__ partial, int nparts, int R)
{
    const int64_t n = (int64_t)(R - 1) * nparts;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        partial[nparts + i] = partial[i % nparts];
}

}  // namespace

hipError_t launch_rl_init(const InitArgs& a, int Rp, float* out0, float* out1, hipStream_t s)
{
    const int64_t HW = a.H * a.W;
    const int64_t blocks = (HW + 3) / 4;          // four sites per workgroup and step, at most 8192 workgroups per group
    hipLaunchKernelGGL(k_rl_init, dim3((unsigned)(blocks < 8192 ? blocks : 8192), (unsigned)(Rp / 64)), dim3(256), 0, s,
                       a, out0, out1);
    return hipGetLastError();
}

hipError_t launch_rl_energy_full(const float* lanes, int64_t H, int64_t W, int R, float q, long long* partial,
                                 int nparts, bool same_start, hipStream_t s)
{
    const unsigned groups = same_start ? 1u : (unsigned)((R + 63) / 64);
    hipLaunchKernelGGL(k_rl_energy_full, dim3((unsigned)nparts, groups), dim3(256), 0, s, lanes, H, W, R, q, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !same_start) return e;
    return launch_rows_from_first(partial, nparts, R, s);
}

hipError_t launch_rows_from_first(long long* partial, int nparts, int R, hipStream_t s)
{
    if (R <= 1 || nparts <= 0) return hipSuccess;
    const int64_t n = (int64_t)(R - 1) * nparts;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_rows_from_first, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, partial,
                       nparts, R);
    return hipGetLastError();
}

}  // namespace mpr
