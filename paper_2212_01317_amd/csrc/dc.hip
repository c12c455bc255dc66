// Double-checkerboard sweep (Sec. 2.2.2): the grid divided into the lb_h x lb_w blocks, coloured like a
// checkerboard by (block row + block column) % 2; one sweep = four in-place phases: colour 0 then colour 1 inside
// the even blocks, then the same inside the odd blocks.  Sites of one phase share no bond, so each phase updates
// the state in place.  One thread per row pair of same-colour sites four columns apart (one Philox block, words 0-1
// for the first site and 2-3 for the second, the counter of the single-checkerboard order); the (cos, sin) of the
// neighbours are computed from the stored angles; the decision is the FP32 filter with the exact FP64 test inside its
// error band, as in the fused sweep.
#include <hip/hip_runtime.h>

#include "metropolis.hpp"
#include "mpr_internal.hpp"

namespace mpr {

namespace {

__global__ __launch_bounds__(256) void k_dc_phase(DcArgs a, uint32_t sweep, int colour, int parity)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= a.H * a.Mw) return;
    const int64_t y = p / a.Mw, m = p - y * a.Mw;
    float* const st = a.state + (int64_t)r * a.H * a.W;
    const U4 w = philox_x3((uint32_t)p, sweep, a.real_offset + (uint32_t)r, ctr_word3(a.scene, TAG_SWEEP, (uint32_t)colour),
                           a.key0, a.key1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t x = 4 * m + ((y + colour) & 1) + 2 * h;
        if (x >= a.W) continue;
        const int64_t n = y * a.W + x;
        if (a.mask[n]) continue;
        if ((int)(((y / a.lb_h) + (x / a.lb_w)) & 1) != parity) continue;
        const TBand tb = a.tb[(y / a.tb_h) * a.nbx_t + (x / a.tb_w)];
        const bool pu = y > 0, pl = x > 0, pr = x + 1 < a.W, pd = y + 1 < a.H;
        const float tu = pu ? st[n - a.W] : 0.0f, tl = pl ? st[n - 1] : 0.0f;
        const float tr = pr ? st[n + 1] : 0.0f, td = pd ? st[n + a.W] : 0.0f;
        const float to = st[n];
        float Cx = 0.0f, Sy = 0.0f;
        if (pu) { Cx += cos_rev(a.q * tu); Sy += sin_rev(a.q * tu); }
        if (pl) { Cx += cos_rev(a.q * tl); Sy += sin_rev(a.q * tl); }
        if (pr) { Cx += cos_rev(a.q * tr); Sy += sin_rev(a.q * tr); }
        if (pd) { Cx += cos_rev(a.q * td); Sy += sin_rev(a.q * td); }
        const uint32_t wp = h ? w.z : w.x, wa = h ? w.w : w.y;
        const float tp = u24(wp);
        const float ui = (float)(wa >> 8);
        const float cp = cos_rev(a.q * tp), sp = sin_rev(a.q * tp);
        const float co = cos_rev(a.q * to), so = sin_rev(a.q * to);
        const float X = fmaf(cp - co, Cx, (sp - so) * Sy);
        int dec = filter32(X, ui, tb, a.J, a.delta_e);
        if (dec < 0) {
            const unsigned present = (pu ? 1u : 0u) | (pl ? 2u : 0u) | (pr ? 4u : 0u) | (pd ? 8u : 0u);
            dec = exact64(tp, to, tu, tl, tr, td, present, a.two_pi_q, a.Jd, tb.T, ui * 5.9604644775390625e-8f) ? 1 : 0;
        }
        if (dec) st[n] = tp;
    }
}

}  // namespace

hipError_t launch_dc_sweep(const DcArgs& a, uint32_t sweep, hipStream_t s)
{
    const dim3 grid((unsigned)((a.H * a.Mw + 255) / 256), (unsigned)a.R);
    for (int parity = 0; parity < 2; ++parity) {
        for (int colour = 0; colour < 2; ++colour) {
            hipLaunchKernelGGL(k_dc_phase, grid, dim3(256), 0, s, a, sweep, colour, parity);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace mpr
