// Philox4x32-10 for kernels in which a wave's 64 lanes are 64 realizations of the same site (the realization-lane
// sweeps of the plane and of the 3D lattice): the counter differs between lanes only in the realization word.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "philox.hpp"

namespace mpr {

// Philox4x32-10 of the counter (site, sweep, realization, w3) and key (k0, k1) when only the realization differs
// between lanes.  The realization enters round 0 only through M1 * realization, and the result of round 0's first
// word depends on nothing else that varies (sweep and key are fixed for a launch), so the lane parts of rounds 0 and
// 1 are three per-lane constants: lo(M1 r), and (hi, lo) of M0 * (hi(M1 r) ^ sweep ^ k0); the round-1 keys are
// folded into the first two (lc1 = lo(M1 r) ^ k0', lph = hi(...) ^ k1', with k' the keys of round 1).  A call then
// does the site's half of rounds 0 and 1 on the scalar unit (w3k1 = w3 ^ k1 folds the round-0 key into the counter
// word), and rounds 2..9 with the three-input xor and the round keys held in vector registers (the same in every
// lane), so that the rounds need no scalar key arithmetic.
struct PhiloxLane {
    uint32_t lc1, lph, lpl;
};

__device__ __forceinline__ PhiloxLane philox_lane(uint32_t real, uint32_t sweep, uint32_t k0, uint32_t k1)
{
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)real;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ sweep ^ k0;
    const uint64_t q = (uint64_t)0xD2511F53u * (uint64_t)n0;
    return PhiloxLane{(uint32_t)p1 ^ (k0 + 0x9E3779B9u), (uint32_t)(q >> 32) ^ (k1 + 0xBB67AE85u), (uint32_t)q};
}

struct RoundKeys {
    uint32_t k[16];   // (k0, k1) of rounds 2 .. 9
};

// The round keys in vector registers: the empty asm makes each key a vector value, so the rounds read it from a
// register instead of recomputing it on the scalar unit.

__device__ __forceinline__ RoundKeys round_keys(uint32_t k0, uint32_t k1)
{
    RoundKeys r;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        r.k[2 * i] = k0 + (uint32_t)(i + 2) * 0x9E3779B9u;
        r.k[2 * i + 1] = k1 + (uint32_t)(i + 2) * 0xBB67AE85u;
        asm volatile("" : "+v"(r.k[2 * i]), "+v"(r.k[2 * i + 1]));
    }
    return r;
}

// a ^ b ^ k in one v_bitop3_b32 (truth table 0x96 = 0xF0 ^ 0xCC ^ 0xAA) with the round key k in a vector register
__device__ __forceinline__ uint32_t xor3v(uint32_t a, uint32_t b, uint32_t k)
{
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

__device__ __forceinline__ U4 philox_site(uint32_t site, uint32_t w3k1, const PhiloxLane& L, const RoundKeys& RK)
{
    // round 0, the site's half (wave-uniform)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)site;
    const uint32_t n2u = (uint32_t)(p0 >> 32) ^ w3k1, c3u = (uint32_t)p0;
    // round 1: M1 * n2u is wave-uniform, M0 * (first word) is the lane constant
    const uint64_t q1 = (uint64_t)0xCD9E8D57u * (uint64_t)n2u;
    uint32_t c0 = (uint32_t)(q1 >> 32) ^ L.lc1;
    uint32_t c1 = (uint32_t)q1;
    uint32_t c2 = c3u ^ L.lph;
    uint32_t c3 = L.lpl;
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        const uint64_t a0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t a1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3v((uint32_t)(a1 >> 32), c1, RK.k[2 * (round - 2)]);
        const uint32_t n2 = xor3v((uint32_t)(a0 >> 32), c3, RK.k[2 * (round - 2) + 1]);
        c1 = (uint32_t)a1;
        c3 = (uint32_t)a0;
        c0 = n0;
        c2 = n2;
    }
    return U4{c0, c1, c2, c3};
}

}  // namespace mpr
