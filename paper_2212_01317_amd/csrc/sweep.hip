// Single-scene launch of the fused red/black sweep (the body is in sweep_body.hpp): one launch = one sweep of every
// realization; workgroup = one tile and a chunk of realizations, in an XCD-aware order (consecutive work items,
// i.e. adjacent tiles, land on the same XCD and share its L2).
#include <hip/hip_runtime.h>

#include "sweep_body.hpp"

namespace mpr {

template <int FTH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sweep_fused(SweepFusedArgs a)
{
    __shared__ LdsT<FTH> L;
    const int64_t nwork = (int64_t)a.ntiles * a.nchunks;
    const int64_t per = (nwork + 7) / 8;
    const int64_t work = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (work >= nwork) return;
    sweep_tile<FTH>(L, a, (int)(work % a.ntiles), (int)(work / a.ntiles));
}

void fused_geometry(int64_t H, int64_t W, int R, int tile_h, int* ntx, int* nty, int* rchunk, int* nchunks)
{
    *ntx = (int)((W + 63) / 64);
    *nty = (int)((H + tile_h - 1) / tile_h);
    const int64_t ntiles = (int64_t)(*ntx) * (*nty);
    // enough workgroups to fill 256 CUs several times over; longer realization chunks amortise the setup
    int64_t rc = ntiles * (int64_t)R / 4096;
    if (rc < 1) rc = 1;
    if (rc > R) rc = R;
    if (rc > 64) rc = 64;
    *rchunk = (int)rc;
    *nchunks = (int)((R + rc - 1) / rc);
}

hipError_t launch_sweep_fused(const SweepFusedArgs& a, hipStream_t s)
{
    const int64_t nwork = (int64_t)a.ntiles * a.nchunks;
    const int64_t grid = ((nwork + 7) / 8) * 8;
    if (a.tile_h == 16)
        hipLaunchKernelGGL(k_sweep_fused<16>, dim3((unsigned)grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_sweep_fused<32>, dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mpr
