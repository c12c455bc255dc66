// The start of the chains and its energy in the realization-lane layout S[g][n][64] (realization r = 64 g + l), for
// the runs that sweep with the realization-lane kernel: the start is written straight into the two lane buffers
// instead of into the [R][H][W] state and transposed.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mpr_internal.hpp"

namespace mpr {

// the start of k_init (a.state and a.state2 unused) for realizations 0 .. Rp - 1 into out0 and out1 (pad realizations
// r >= a.R get 0, as the transposition gives them)
hipError_t launch_rl_init(const InitArgs& a, int Rp, float* out0, float* out1, hipStream_t s);
// the energy partials of k_energy_full (the same per-site terms, so the same integer sums) from a lane buffer:
// partial[r][part], part < nparts
// rows 1 .. R - 1 of partial[R][nparts] from row 0: the start energy of a start that every realization shares
hipError_t launch_rows_from_first(long long* partial, int nparts, int R, hipStream_t s);
// same_start: every realization holds the same start (the block-mean start has no random part), so the partials of
// the first group of 64 realizations are computed and realization 0's row is copied to the others
hipError_t launch_rl_energy_full(const float* lanes, int64_t H, int64_t W, int R, float q, long long* partial,
                                 int nparts, bool same_start, hipStream_t s);

}  // namespace mpr
