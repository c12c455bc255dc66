// Device helpers of the Metropolis update shared by the sweep kernels: the gfx950 transcendental intrinsics, the
// FP32 acceptance filter with its error band, and the exact FP64 decision.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mpr_internal.hpp"
#include "philox.hpp"

namespace mpr {

// cos / sin of 2 pi x for x in revolutions (v_cos_f32 / v_sin_f32, valid for |x| <= 256); 2^x (v_exp_f32).
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// a ^ b ^ k in one gfx950 three-input bit operation (truth table 0x96 over the inputs a = 0xF0, b = 0xCC, k = 0xAA).
// The builtin, not inline assembly: the compiler then knows the instruction and inserts no wait states for it.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k)
{
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Philox4x32-10 written with the three-input xor (the same function as philox4x32_10).  In the sweeps only c0
// differs between lanes, so in the first two rounds one of the two products and half of the xors are wave-uniform:
// those rounds are plain C and the compiler keeps the uniform parts on the scalar unit; the other eight use v_bitop3.
__device__ __forceinline__ U4 philox_x3(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    // keep the key schedule as per-call scalar adds instead of twenty loop-invariant registers
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return U4{c0, c1, c2, c3};
}

// FP32 Metropolis filter.  Returns 1 = accept, 0 = reject, -1 = inside the error band (the exact FP64 test decides).
//
// Inputs in scaled form: X = (c' - c) Cx + (s' - s) Sy, so that the energy change is dE = -J X, with
// |dE - dE_exact| <= delta; ui = (wa >> 8) as a float, so that u2 = ui 2^-24 exactly; tb = the block's
// {T, kappa = J log2(e) / T, band, kb}.  The exact test is u2 < exp(-dE/T) (T > 0) or dE <= 0 (T == 0).
//
// For T > 0, y24 = fma(X, kappa, 24) is 24 plus y = log2 of the acceptance ratio, and w24 = 2^y24 = 2^24 w.  Its
// error: |y24 - 24 - y_exact| <= delta log2(e) / T (from dE) + |y| 2^-22 (roundings of kappa and of the product)
// + 2^-20 (rounding of the sum near 24), and v_exp_f32 adds a relative 2^-22.  The relative error of w24 is then at
// most ln 2 times the first three terms plus 2^-22; the band is that bound with a 25 % margin,
// rel = |X| kb + band with kb = 1.25 ln2 2^-22 kappa and band = band_of(T, delta), plus an absolute 2^-6 (2^-30 in u2
// units) for results that flush to zero.  y24 is clamped at 25 (y >= 1 accepts: w > 1 > u2, and the clamped value
// still lies more than the band above any ui).
constexpr float kBandY = 1.25f * 0.6931472f * 2.3841858e-7f;

__device__ __forceinline__ float band_of(float T, float delta)
{
    return T > 0.0f ? 1.25f * (0.6931472f * (delta * (1.4426950f / T) + 9.5367432e-7f) + 2.3841858e-7f) : 0.0f;
}

__device__ __forceinline__ TBand make_tband(float T, float J, float delta)
{
    TBand b;
    b.T = T > 0.0f ? T : 0.0f;      // a temperature that is not > 0 (NaN included) is held as +0
    b.kappa = T > 0.0f ? (float)((double)J * 1.4426950408889634074 / (double)T) : 0.0f;
    b.band = band_of(T, delta);
    b.kb = kBandY * b.kappa;
    return b;
}

// Directional coupling: y24 = fma(X_h, kx, fma(X_v, ky, 24)) with the horizontal and vertical parts X_h, X_v of the
// field change (each within delta / J of exact).  Its error: delta log2(e) (1/Tx + 1/Ty) from the fields, two
// roundings near 24 (2^-19 together), and the roundings of kx, ky and of large intermediate sums (at most
// (|X_h| kx + |X_v| ky) 2^-22); v_exp_f32 adds a relative 2^-22.  The band is that bound with a 25 % margin, as for
// one temperature.  Both temperatures are > 0.
__device__ __forceinline__ TBandDir make_tband_directional(float Tx, float Ty, float J, float delta)
{
    TBandDir b;
    b.Tx = Tx;
    b.Ty = Ty;
    b.kx = (float)((double)J * 1.4426950408889634074 / (double)Tx);
    b.ky = (float)((double)J * 1.4426950408889634074 / (double)Ty);
    b.kbx = kBandY * b.kx;
    b.kby = kBandY * b.ky;
    b.band = 1.25f * (0.6931472f * (delta * 1.4426950f * (1.0f / Tx + 1.0f / Ty) + 1.9073486e-6f) + 2.3841858e-7f);
    b.pad = 0.0f;
    return b;
}

__device__ __forceinline__ int filter32(float X, float ui, const TBand& tb, float J, float delta)
{
    if (tb.T > 0.0f) {
        const float y24 = fminf(fmaf(X, tb.kappa, 24.0f), 25.0f);
        const float w24 = exp2_fast(y24);
        const float rel = fmaf(fabsf(X), tb.kb, tb.band);
        if (fabsf(ui - w24) <= fmaf(w24, rel, 0.015625f)) return -1;
        return ui < w24 ? 1 : 0;
    }
    const float dE = -J * X;
    if (fabsf(dE) <= delta) return -1;
    return dE <= 0.0f ? 1 : 0;
}

// The exact decision, evaluated as the published formula: dE = -J sum_j [cos 2 pi q (t' - t_j) - cos 2 pi q (t - t_j)]
// over the present neighbours in the order up, left, right, down; accept iff u2 < exp(-dE / T) (T > 0) or dE <= 0.
__device__ __noinline__ bool exact64(float tp, float to, float nu, float nl, float nr, float nd, unsigned present,
                                     double two_pi_q, double J, float T, float u2)
{
    double acc = 0.0;
    const double dtp = (double)tp, dto = (double)to;
    if (present & 1u) acc += cos(two_pi_q * (dtp - (double)nu)) - cos(two_pi_q * (dto - (double)nu));
    if (present & 2u) acc += cos(two_pi_q * (dtp - (double)nl)) - cos(two_pi_q * (dto - (double)nl));
    if (present & 4u) acc += cos(two_pi_q * (dtp - (double)nr)) - cos(two_pi_q * (dto - (double)nr));
    if (present & 8u) acc += cos(two_pi_q * (dtp - (double)nd)) - cos(two_pi_q * (dto - (double)nd));
    const double dE = -J * acc;
    if ((double)T > 0.0) return (double)u2 < exp(-dE / (double)T);
    return dE <= 0.0;
}

// The exact directional decision, evaluated as the definition writes it: ah over the left and right neighbours, av
// over the up and down neighbours (each term cos 2 pi q (t' - t_j) - cos 2 pi q (t - t_j), in the order up, left,
// right, down), accept iff u2 < exp(J ah / Tx + J av / Ty).
__device__ __noinline__ bool exact64_directional(float tp, float to, float nu, float nl, float nr, float nd,
                                                 unsigned present, double two_pi_q, double J, float Tx, float Ty,
                                                 float u2)
{
    double ah = 0.0, av = 0.0;
    const double dtp = (double)tp, dto = (double)to;
    if (present & 1u) av += cos(two_pi_q * (dtp - (double)nu)) - cos(two_pi_q * (dto - (double)nu));
    if (present & 2u) ah += cos(two_pi_q * (dtp - (double)nl)) - cos(two_pi_q * (dto - (double)nl));
    if (present & 4u) ah += cos(two_pi_q * (dtp - (double)nr)) - cos(two_pi_q * (dto - (double)nr));
    if (present & 8u) av += cos(two_pi_q * (dtp - (double)nd)) - cos(two_pi_q * (dto - (double)nd));
    const double w = J * ah / (double)Tx + J * av / (double)Ty;
    return (double)u2 < exp(w);
}

}  // namespace mpr
