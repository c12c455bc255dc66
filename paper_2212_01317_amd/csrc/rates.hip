// Instruction-rate probe for the ALU roofline of the sweep: the issue cost of the instructions the Metropolis update
// is made of, measured on the device relative to a full-rate 32-bit add.  Each probe kernel runs eight independent
// dependency chains per lane (enough to cover the pipeline latency) over a fixed number of steps on a grid that fills
// every SIMD several times; the cost is the kernel time divided by the number of wave-instructions.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mpr_internal.hpp"

namespace {

constexpr int kChains = 8;
constexpr int kSteps = 2048;
constexpr int kNT = 256;

enum Probe : int {
    P_ADD = 0,      // v_add_u32
    P_MAD64,        // v_mad_u64_u32 (32 x 32 + 64 -> 64), chained through its 64-bit addend
    P_MUL_LO,       // v_mul_lo_u32
    P_MUL_HI,       // v_mul_hi_u32
    P_BITOP3,       // v_bitop3_b32 (three-input xor)
    P_SIN,          // v_sin_f32
    P_COS,          // v_cos_f32
    P_EXP,          // v_exp_f32
    P_CVT,          // v_cvt_f32_u32
    P_XOR,          // v_xor_b32
    P_MAD_ADD,      // per chain and step: one v_mad_u64_u32 and one independent v_add_u32 (do the two co-issue?)
    P_MAD_BITOP3,   // per chain and step: v_mad_u64_u32, then v_bitop3_b32 folding its high half into a word (the
                    // shape of a Philox round: the three-input xor consumes the product)
    P_COUNT
};

// wave-instructions per chain and step of each probe
__host__ __device__ constexpr int probe_width(int op) { return op == P_MAD_ADD || op == P_MAD_BITOP3 ? 2 : 1; }
static_assert(P_COUNT == mpr::kProbeCount, "probe count");

template <int OP>
__global__ __launch_bounds__(kNT) void k_probe(uint32_t* out, uint32_t seed)
{
    uint32_t a[kChains];
    uint64_t d[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        a[c] = threadIdx.x * 7919u + (uint32_t)c * 104729u + seed;
        d[c] = (uint64_t)a[c] << 17;
    }
    const uint32_t m = 0xD2511F53u;
    uint64_t carry[kChains];     // one carry-out pair per chain: no two products write the same SGPRs
#pragma unroll
    for (int c = 0; c < kChains; ++c) carry[c] = 0;
    for (int i = 0; i < kSteps; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (OP == P_ADD) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "s"(m));
            if (OP == P_MAD64)
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(d[c]), "+s"(carry[c]) : "v"(a[c]), "s"(m));
            if (OP == P_MAD_ADD) {
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(d[c]), "+s"(carry[c]) : "v"(a[c]), "s"(m));
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[(c + 4) % kChains]) : "s"(m));
            }
            if (OP == P_MAD_BITOP3) {
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(d[c]), "+s"(carry[c]) : "v"(a[c]), "s"(m));
                const uint32_t hi = (uint32_t)(d[c] >> 32);       // the high register of the pair, no instruction
                asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[c]) : "v"(hi), "s"(m));
            }
            if (OP == P_MUL_LO) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[c]) : "s"(m));
            if (OP == P_MUL_HI) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[c]) : "s"(m));
            if (OP == P_BITOP3)
                asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[c]) : "v"(a[(c + 1) % kChains]), "s"(m));
            if (OP == P_SIN) asm volatile("v_sin_f32 %0, %0" : "+v"(a[c]));
            if (OP == P_COS) asm volatile("v_cos_f32 %0, %0" : "+v"(a[c]));
            if (OP == P_EXP) asm volatile("v_exp_f32 %0, %0" : "+v"(a[c]));
            if (OP == P_CVT) asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(a[c]));
            if (OP == P_XOR) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[c]) : "v"(a[(c + 1) % kChains]));
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s ^= a[c] ^ (uint32_t)d[c] ^ (uint32_t)(d[c] >> 32) ^ (uint32_t)carry[c];
    out[(size_t)blockIdx.x * kNT + threadIdx.x] = s;
}

template <int OP>
hipError_t launch_probe(uint32_t* out, int grid, hipStream_t s, uint32_t seed)
{
    hipLaunchKernelGGL(k_probe<OP>, dim3(grid), dim3(kNT), 0, s, out, seed);
    return hipGetLastError();
}

hipError_t launch_any(int op, uint32_t* out, int grid, hipStream_t s, uint32_t seed)
{
    switch (op) {
    case P_ADD: return launch_probe<P_ADD>(out, grid, s, seed);
    case P_MAD64: return launch_probe<P_MAD64>(out, grid, s, seed);
    case P_MUL_LO: return launch_probe<P_MUL_LO>(out, grid, s, seed);
    case P_MUL_HI: return launch_probe<P_MUL_HI>(out, grid, s, seed);
    case P_BITOP3: return launch_probe<P_BITOP3>(out, grid, s, seed);
    case P_SIN: return launch_probe<P_SIN>(out, grid, s, seed);
    case P_COS: return launch_probe<P_COS>(out, grid, s, seed);
    case P_EXP: return launch_probe<P_EXP>(out, grid, s, seed);
    case P_CVT: return launch_probe<P_CVT>(out, grid, s, seed);
    case P_XOR: return launch_probe<P_XOR>(out, grid, s, seed);
    case P_MAD_ADD: return launch_probe<P_MAD_ADD>(out, grid, s, seed);
    default: return launch_probe<P_MAD_BITOP3>(out, grid, s, seed);
    }
}

}  // namespace

namespace mpr {

int probe_grid()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    return 16 * cus;     // 16 workgroups of 4 waves per CU: 16 waves per SIMD over the run
}

size_t probe_out_bytes() { return (size_t)probe_grid() * kNT * sizeof(uint32_t); }

double probe_wave_instructions() { return (double)probe_grid() * (kNT / 64) * kSteps * kChains; }

hipError_t time_probes(uint32_t* out, hipStream_t s, double* ns)
{
    const int grid = probe_grid();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    for (int op = 0; op < kProbeCount && err == hipSuccess; ++op) {
        err = launch_any(op, out, grid, s, 1u);                  // warm
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        if (err == hipSuccess) err = launch_any(op, out, grid, s, 2u);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ns[op] = (double)ms * 1e6 / probe_width(op);     // per wave-instruction of the probe
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return err;
}

}  // namespace mpr
