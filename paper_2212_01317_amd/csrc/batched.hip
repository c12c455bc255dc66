// Batched conditional simulation: many scenes of different sizes and gap fractions advance together, one sweep
// per launch of a persistent kernel that takes (scene, tile, realization chunk) work items from a global queue.
//
// Every scene keeps its own random stream (its scene id), temperatures, stopping test and sampling sweeps, so its
// results are bit-identical to a single-scene run.  All per-sweep control lives on the device (sweep counter,
// queue head, per-scene phase, work-list prefix), so a chunk of sweeps is a fixed sequence of launches that can be
// captured once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include "batched.hpp"
#include "sweep_body.hpp"

namespace mpr {

namespace {

__device__ __forceinline__ SweepFusedArgs scene_args(const BatchScene& d, const BatchCfg& c, int variant, int k)
{
    SweepFusedArgs a;
    a.src = d.buf[(k - 1) & 1];
    a.dst = d.buf[k & 1];
    a.mask = d.mask;
    a.Tb = d.tp;
    a.H = d.H;
    a.W = d.W;
    a.lb_h = d.lb_h;
    a.lb_w = d.lb_w;
    a.nbx = d.nbx;
    a.ntx = d.ntx;
    a.nty = d.nty[variant];
    a.ntiles = d.ntiles[variant];
    a.Mw = d.Mw;
    a.R = c.R;
    a.rchunk = d.rchunk[variant];
    a.nchunks = d.nchunks[variant];
    a.tile_h = variant ? 32 : 16;
    a.HW = d.HW;
    a.sweep = (uint32_t)k;
    a.real_offset = c.real_offset;
    a.scene = d.scene;
    a.key0 = c.key0;
    a.key1 = c.key1;
    a.q = c.q;
    a.J = c.J;
    a.delta_e = c.delta_e;
    a.two_pi_q = c.two_pi_q;
    a.Jd = c.Jd;
    a.e_partial = nullptr;
    return a;
}

}  // namespace

// Persistent sweep: workgroups take items until the queue is empty.  Items are numbered through the work-list
// prefix of the scenes in longest-first order; item -> (scene, tile, chunk).
template <int FTH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_batch_sweep(
    const BatchScene* __restrict__ scenes, const BatchRun* __restrict__ runs, const int* __restrict__ order,
    const int64_t* __restrict__ prefix, BatchCtl* ctl, BatchCfg c, int n_scenes)
{
    __shared__ LdsT<FTH> L;
    __shared__ int64_t s_item;
    constexpr int variant = FTH == 32 ? 1 : 0;
    const int k = ctl->k;
    const int64_t n_items = prefix[n_scenes];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(&ctl->queue, 1ull);
        __syncthreads();
        // uniform: the scene descriptor is then read with scalar loads and kept in scalar registers
        const uint64_t iu = (uint64_t)s_item;
        const int64_t item = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(iu >> 32)) << 32) |
                                       (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)iu));
        __syncthreads();
        if (item >= n_items) break;
        int lo = 0, hi = n_scenes;            // largest i with prefix[i] <= item
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int s = order[lo];
        const BatchScene& d = scenes[s];
        SweepFusedArgs a = scene_args(d, c, variant, k);
        if (c.energy && runs[s].phase == 0) a.e_partial = d.epart;
        const int64_t local = item - prefix[lo];
        sweep_tile<FTH>(L, a, (int)(local % a.ntiles), (int)(local / a.ntiles));
    }
}

__global__ void k_batch_begin(BatchCtl* ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->k += 1;
        ctl->queue = 0ull;
    }
}

// e_real[r] of every equilibrating scene: one workgroup per (scene, realization), tiles summed in a fixed order.
__global__ __launch_bounds__(256) void k_batch_energy_real(const BatchScene* scenes, const BatchRun* runs,
                                                            BatchCfg c, int variant)
{
    __shared__ long long lds[4];
    const int s = blockIdx.x, r = blockIdx.y;
    if (runs[s].phase != 0) return;
    const BatchScene& d = scenes[s];
    const int nt = d.ntiles[variant];
    const long long* row = d.epart + (int64_t)r * nt;
    long long v = 0;
    for (int p = threadIdx.x; p < nt; p += 256) v += row[p];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) d.e_real[r] = ((double)(((lds[0] + lds[1]) + lds[2]) + lds[3]) * kFixUnit) * d.inv_norm;
}

__global__ __launch_bounds__(256) void k_batch_energy_mean(const BatchScene* scenes, const BatchRun* runs,
                                                            const BatchCtl* ctl, BatchCfg c, int n_scenes)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_scenes || runs[s].phase != 0) return;
    const BatchScene& d = scenes[s];
    double sum = 0.0;
    for (int r = 0; r < c.R; ++r) sum += d.e_real[r];
    d.series[ctl->k] = sum / (double)c.R;
}

// The sampling scenes of this sweep, for every workgroup of a grid that shares out their sites: the scenes are listed
// 256 at a time from one coalesced read of their phases, and body(s) runs for each listed scene.  (One workgroup per
// (share, scene) instead left almost all workgroups without work: only the few scenes that have just equilibrated
// sample in a given sweep.)  A workgroup of 256 threads; the order of the list does not matter, since each site of
// a scene is summed by one thread.
template <class Body>
__device__ __forceinline__ void for_sampling_scenes(const BatchRun* runs, int n_scenes, Body body)
{
    __shared__ int list[256];
    __shared__ int cnt;
    for (int i0 = 0; i0 < n_scenes; i0 += 256) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        const int i = i0 + (int)threadIdx.x;
        if (i < n_scenes && runs[i].phase == 1) list[atomicAdd(&cnt, 1)] = i;
        __syncthreads();
        const int m = cnt;
        for (int j = 0; j < m; ++j) body(list[j]);
        __syncthreads();   // the list and its count are rewritten for the next 256 scenes
    }
}

// The work list of the scenes still running (one workgroup of 256 threads, after the phase transitions):
// prefix[i] = the work of the running scenes among order[0 .. i), prefix[n_scenes] the total, *n_active their
// number.  An exclusive scan over 256 scenes at a time: wave scans by shuffles, then the four wave totals.
template <class WorkOf>
__device__ __forceinline__ void running_work_prefix(const BatchRun* runs, const int* order, int64_t* prefix,
                                                    int n_scenes, int* n_active, WorkOf work_of)
{
    __shared__ long long wsum[4];
    __shared__ int wcnt[4];
    const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
    long long base = 0;
    int active = 0;
    for (int i0 = 0; i0 < n_scenes; i0 += 256) {
        const int i = i0 + (int)threadIdx.x;
        long long w = 0;
        bool running = false;
        if (i < n_scenes) {
            const int s = order[i];
            if (runs[s].phase < 2) {
                w = (long long)work_of(s);
                running = true;
            }
        }
        long long x = w;                    // inclusive scan of w within the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        const int nrun = __popcll(__ballot(running));
        if (lane == 63) {
            wsum[wv] = x;
            wcnt[wv] = nrun;
        }
        __syncthreads();
        long long before = 0;
        for (int j = 0; j < wv; ++j) before += wsum[j];
        if (i < n_scenes) prefix[i] = base + before + (x - w);
        base += ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
        active += ((wcnt[0] + wcnt[1]) + wcnt[2]) + wcnt[3];
        __syncthreads();                    // the wave totals are rewritten for the next 256 scenes
    }
    if (threadIdx.x == 0) {
        prefix[n_scenes] = base;
        *n_active = active;
    }
}

// Sampling scenes: acc += sum over realizations (in order) of the state after this sweep.
__global__ __launch_bounds__(256) void k_batch_accumulate(const BatchScene* scenes, const BatchRun* runs,
                                                           const BatchCtl* ctl, BatchCfg c, int n_scenes)
{
    const int k = ctl->k;
    for_sampling_scenes(runs, n_scenes, [&](int s) {
        const BatchRun run = runs[s];
        const BatchScene& d = scenes[s];
        const float* st = d.buf[k & 1];
        for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < d.HW; n += (int64_t)gridDim.x * 256) {
            if (d.mask[n]) {
                if (run.samp == 0) d.acc[n] = 0.0;
                continue;
            }
            double acc = run.samp == 0 ? 0.0 : d.acc[n];
            for (int r = 0; r < c.R; ++r) acc += (double)st[(int64_t)r * d.HW + n];
            d.acc[n] = acc;
        }
    });
}

// Sec. 3.4 test on the device (same reading as the single-scene driver): OLS slope of the last n_fit energies,
// equilibrium when it no longer points away from the starting energy.
__device__ bool batch_equilibrium(const double* series, int k, int n_fit)
{
    const double* y = series + (k - n_fit + 1);
    double xm = 0.0, ym = 0.0;
    for (int j = 0; j < n_fit; ++j) {
        xm += (double)j;
        ym += y[j];
    }
    xm /= (double)n_fit;
    ym /= (double)n_fit;
    double sxy = 0.0, sxx = 0.0;
    for (int j = 0; j < n_fit; ++j) {
        sxy += ((double)j - xm) * (y[j] - ym);
        sxx += ((double)j - xm) * ((double)j - xm);
    }
    const double beta = sxx > 0.0 ? sxy / sxx : 0.0;
    const double d = series[k] - series[0];
    const double sigma0 = (double)((d > 0.0) - (d < 0.0));
    return beta * sigma0 <= 0.0;
}

// Phase transitions after sweep k, then the work-list prefix over the scenes still running (one workgroup).
__global__ __launch_bounds__(256) void k_batch_phase(const BatchScene* scenes, BatchRun* runs, const int* order,
                                                      int64_t* prefix, BatchCtl* ctl, BatchCfg c, int n_scenes,
                                                      int variant)
{
    const int k = ctl->k;
    for (int s = threadIdx.x; s < n_scenes; s += 256) {
        BatchRun run = runs[s];
        if (run.phase == 0) {
            bool stop = false;
            if (c.stop_mode == 1) {
                if (k >= c.n_fit + c.n_f && (k - c.n_fit) % c.n_f == 0)
                    stop = batch_equilibrium(scenes[s].series, k, c.n_fit);
                if (!stop && k >= c.n_max) {
                    stop = true;
                    run.converged = 0;
                }
            } else {
                stop = k >= c.n_eq;
            }
            if (stop) {
                run.phase = c.n_samp > 0 ? 1 : 2;
                run.k_star = k;
            }
        } else if (run.phase == 1) {
            run.samp += 1;
            if (run.samp >= c.n_samp) run.phase = 2;
        }
        runs[s] = run;
    }
    __syncthreads();
    running_work_prefix(runs, order, prefix, n_scenes, &ctl->n_active,
                        [&](int s) { return (int64_t)scenes[s].ntiles[variant] * scenes[s].nchunks[variant]; });
}

hipError_t launch_batch_sweep(const BatchDev& b, int variant, int grid, hipStream_t s)
{
    if (variant)
        hipLaunchKernelGGL(k_batch_sweep<32>, dim3(grid), dim3(256), 0, s, b.scenes, b.runs, b.order, b.prefix,
                           b.ctl, b.cfg, b.n);
    else
        hipLaunchKernelGGL(k_batch_sweep<16>, dim3(grid), dim3(256), 0, s, b.scenes, b.runs, b.order, b.prefix,
                           b.ctl, b.cfg, b.n);
    return hipGetLastError();
}

// One sweep of the batch: counter, sweep, energies of the equilibrating scenes, accumulation of the sampling
// scenes, phase transitions and the next work list.
hipError_t launch_batch_step(const BatchDev& b, int variant, int next_variant, int grid, int acc_blocks,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, s, b.ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_batch_sweep(b, variant, grid, s)) != hipSuccess) return e;
    if (b.cfg.energy) {
        hipLaunchKernelGGL(k_batch_energy_real, dim3(b.n, b.cfg.R), dim3(256), 0, s, b.scenes, b.runs, b.cfg, variant);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_batch_energy_mean, dim3((b.n + 255) / 256), dim3(256), 0, s, b.scenes, b.runs, b.ctl,
                           b.cfg, b.n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_accumulate, dim3(acc_blocks), dim3(256), 0, s, b.scenes, b.runs, b.ctl, b.cfg, b.n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_phase, dim3(1), dim3(256), 0, s, b.scenes, b.runs, b.order, b.prefix, b.ctl, b.cfg,
                       b.n, next_variant);
    return hipGetLastError();
}

// ---- the batch on the realization-lane sweep ----

__global__ void k_batchl_begin(BatchLaneCtl* ctl)
{
    if (blockIdx.x == 0 && threadIdx.x < 8) {
        ctl->queue[threadIdx.x] = 0ull;
        if (threadIdx.x == 0) ctl->k += 1;
    }
}

// e_real[r] of every equilibrating scene: one workgroup per (scene, realization), the partials summed as integers
// (order-free), as in the single-scene reduction.
__global__ __launch_bounds__(256) void k_batchl_energy_real(const BatchLaneScene* scenes, const BatchRun* runs)
{
    __shared__ long long lds[4];
    const int s = blockIdx.x, r = blockIdx.y;
    if (runs[s].phase != 0) return;
    const BatchLaneScene& d = scenes[s];
    const long long* row = d.epart + (int64_t)r * d.nparts;
    long long v = 0;
    for (int p = threadIdx.x; p < d.nparts; p += 256) v += row[p];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) d.e_real[r] = ((double)(((lds[0] + lds[1]) + lds[2]) + lds[3]) * kFixUnit) * d.inv_norm;
}

__global__ __launch_bounds__(256) void k_batchl_energy_mean(const BatchLaneScene* scenes, const BatchRun* runs,
                                                             const BatchLaneCtl* ctl, int R, int n_scenes)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n_scenes || runs[s].phase != 0) return;
    const BatchLaneScene& d = scenes[s];
    double sum = 0.0;
    for (int r = 0; r < R; ++r) sum += d.e_real[r];
    d.series[ctl->k] = sum / (double)R;
}

// Sampling scenes: acc += sum over realizations (in order) of the state after this sweep (lane layout).
__global__ __launch_bounds__(256) void k_batchl_accumulate(const BatchLaneScene* scenes, const BatchRun* runs,
                                                            const BatchLaneCtl* ctl, int R, int n_scenes)
{
    const int k = ctl->k;
    for_sampling_scenes(runs, n_scenes, [&](int s) {
        const BatchRun run = runs[s];
        const BatchLaneScene& d = scenes[s];
        const float* st = d.buf[k & 1];
        for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < d.HW; n += (int64_t)gridDim.x * 256) {
            if (d.mask[n]) {
                if (run.samp == 0) d.acc[n] = 0.0;
                continue;
            }
            double acc = run.samp == 0 ? 0.0 : d.acc[n];
            for (int r = 0; r < R; ++r) acc += (double)st[((int64_t)(r >> 6) * d.HW + n) * 64 + (r & 63)];
            d.acc[n] = acc;
        }
    });
}

// Estimated time of one sweep of a scene, relative: every site costs kSiteCost (its angle, cos, sin and energy term
// and its share of the row's loads and waits) and every gap site kGapCost more (its update), the costs per site and
// per update that fit the lane sweep's measured times on the 4096^2 input at p = 0.3, 0.6 and 0.9.
constexpr int64_t kSiteCost = 32, kGapCost = 59;

// The XCD bounds of the work list of the running scenes (one workgroup of 256 threads, after `prefix` holds the
// list's item offsets): bound[x] is the item at which x eighths of the estimated time are reached, the time of a
// scene spread evenly over its items.  Integer costs, so that the scenes' cost intervals tile [0, total) exactly
// and every eighth's boundary falls in exactly one of them.
__device__ __forceinline__ void xcd_bounds(const BatchLaneScene* scenes, const BatchRun* runs, const int* order,
                                           const int64_t* prefix, const int64_t* gaps, int n_scenes,
                                           int64_t* bound)
{
    __shared__ long long csum[4];
    const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
    auto cost_of = [&](int i) -> long long {
        if (i >= n_scenes) return 0;
        const int s = order[i];
        return runs[s].phase < 2 ? (long long)(kSiteCost * scenes[s].HW + kGapCost * gaps[s]) : 0;
    };
    // total
    long long total = 0;
    for (int i0 = 0; i0 < n_scenes; i0 += 256) {
        long long x = cost_of(i0 + (int)threadIdx.x);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) csum[wv] = x;
        __syncthreads();
        total += ((csum[0] + csum[1]) + csum[2]) + csum[3];
        __syncthreads();
    }
    const int64_t N = prefix[n_scenes];
    if (threadIdx.x == 0) {
        bound[0] = 0;
        bound[8] = N;
    }
    if (total <= 0) {
        if (threadIdx.x >= 1 && threadIdx.x < 8) bound[threadIdx.x] = N;
        return;
    }
    // the scene whose cost interval holds x eighths of the total sets bound[x]
    long long base = 0;
    for (int i0 = 0; i0 < n_scenes; i0 += 256) {
        const int i = i0 + (int)threadIdx.x;
        const long long c = cost_of(i);
        long long x = c;                    // inclusive scan of the costs within the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) csum[wv] = x;
        __syncthreads();
        long long before = base;
        for (int j = 0; j < wv; ++j) before += csum[j];
        before += x - c;
        if (c > 0) {
            const int s = order[i];
            for (int q = 1; q < 8; ++q) {
                const long long t = total / 8 * q + (total % 8) * q / 8;     // floor(total q / 8) without overflow
                if (before <= t && t < before + c)      // (a 128-bit product: cost x items can pass 2^63)
                    bound[q] = prefix[i] + (int64_t)((__int128)(t - before) * scenes[s].work / c);
            }
        }
        base += ((csum[0] + csum[1]) + csum[2]) + csum[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_batchl_bounds(const BatchLaneScene* scenes, const BatchRun* runs,
                                                        const int* order, const int64_t* prefix,
                                                        const int64_t* gaps, BatchLaneCtl* ctl, int n_scenes)
{
    xcd_bounds(scenes, runs, order, prefix, gaps, n_scenes, ctl->bound);
}

__global__ __launch_bounds__(256) void k_count_gaps(const uint8_t* __restrict__ mask, int64_t HW,
                                                     unsigned long long* out)
{
    __shared__ unsigned long long wsum[4];
    unsigned long long c = 0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < HW; n += (int64_t)gridDim.x * 256)
        c += mask[n] ? 0u : 1u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3]);
}

// Phase transitions after sweep k (the test of the single-scene driver), then the work list of the scenes still
// running (one workgroup).
__global__ __launch_bounds__(256) void k_batchl_phase(const BatchLaneScene* scenes, BatchRun* runs, const int* order,
                                                       int64_t* prefix, const int64_t* gaps, BatchLaneCtl* ctl,
                                                       BatchCfg c, int n_scenes)
{
    const int k = ctl->k;
    for (int s = threadIdx.x; s < n_scenes; s += 256) {
        BatchRun run = runs[s];
        if (run.phase == 0) {
            bool stop = false;
            if (c.stop_mode == 1) {
                if (k >= c.n_fit + c.n_f && (k - c.n_fit) % c.n_f == 0)
                    stop = batch_equilibrium(scenes[s].series, k, c.n_fit);
                if (!stop && k >= c.n_max) {
                    stop = true;
                    run.converged = 0;
                }
            } else {
                stop = k >= c.n_eq;
            }
            if (stop) {
                run.phase = c.n_samp > 0 ? 1 : 2;
                run.k_star = k;
            }
        } else if (run.phase == 1) {
            run.samp += 1;
            if (run.samp >= c.n_samp) run.phase = 2;
        }
        runs[s] = run;
    }
    __syncthreads();
    running_work_prefix(runs, order, prefix, n_scenes, &ctl->n_active, [&](int s) { return scenes[s].work; });
    __syncthreads();
    xcd_bounds(scenes, runs, order, prefix, gaps, n_scenes, ctl->bound);
}

hipError_t launch_batchl_step(const BatchLaneDev& b, int grid, int acc_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_batchl_begin, dim3(1), dim3(64), 0, s, b.ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_batchl_sweep(b, grid, s)) != hipSuccess) return e;
    if (b.cfg.energy) {
        hipLaunchKernelGGL(k_batchl_energy_real, dim3(b.n, b.cfg.R), dim3(256), 0, s, b.scenes, b.runs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_batchl_energy_mean, dim3((b.n + 255) / 256), dim3(256), 0, s, b.scenes, b.runs, b.ctl,
                           b.cfg.R, b.n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batchl_accumulate, dim3(acc_blocks), dim3(256), 0, s, b.scenes, b.runs, b.ctl, b.cfg.R, b.n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_batchl_phase, dim3(1), dim3(256), 0, s, b.scenes, b.runs, b.order, b.prefix, b.gaps, b.ctl,
                       b.cfg, b.n);
    return hipGetLastError();
}

hipError_t launch_batchl_bounds(const BatchLaneDev& b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batchl_bounds, dim3(1), dim3(256), 0, s, b.scenes, b.runs, b.order, b.prefix, b.gaps, b.ctl,
                       b.n);
    return hipGetLastError();
}

hipError_t launch_count_gaps(const uint8_t* mask, int64_t HW, int64_t* out, hipStream_t s)
{
    const int64_t blocks = (HW + 255) / 256;
    hipLaunchKernelGGL(k_count_gaps, dim3((unsigned)(blocks < 256 ? (blocks > 0 ? blocks : 1) : 256)), dim3(256), 0, s,
                       mask, HW, reinterpret_cast<unsigned long long*>(out));
    return hipGetLastError();
}

}  // namespace mpr
