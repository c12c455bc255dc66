// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11), device side.
//
// Ten rounds of the Philox S-box: the two 32x32 -> 64-bit products of counter words 0 and 2 with the round
// multipliers; the high halves are xored with the other counter words and the round key; the key advances by the
// Weyl constants between rounds.  The key is a kernel argument (wave-uniform), so its schedule stays in SGPRs.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mpr {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return U4{c0, c1, c2, c3};
}

// Uniform on [0, 1) from the top 24 bits of a word; exact in FP32.
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }

// Stream tags (fourth counter word = scene << 4 | tag << 1 | colour).
enum : uint32_t { TAG_SWEEP = 0u, TAG_INIT = 1u, TAG_REFLAT = 2u };

__device__ __forceinline__ uint32_t ctr_word3(uint32_t scene, uint32_t tag, uint32_t colour)
{
    return (scene << 4) | (tag << 1) | colour;
}

}  // namespace mpr
