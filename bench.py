"""Throughput benchmark of the SV-MPR hot path on one MI355X.

One step = one whole gap-filling pass over the 4096 x 4096 headline workload with inputs resident in HBM:
map to angles -> block temperatures (32 x 32 blocks) -> conditional simulation of 256 realizations with the
automatic equilibrium test and one sampling sweep -> prediction -> validation error (AAE/RASE) on the removed pixels.
value = gap-site updates per second = sum over steps of R * (gap sites) * (sweeps) / wall time of the steps.

Prints one JSON line.  --profile-sweeps N runs only N sweeps of the sweep kernel (plus a 1 GiB device copy used to
calibrate the HBM byte counters) and prints nothing else; it is the command the counter profiles are taken with.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU work, in lane-operations (one full-rate VALU lane-instruction = 1; quarter-rate = 4):
# per gap-site update: half a Philox4x32-10 block (10 rounds x (2 mad_u64_u32 x 4 + 2 xor3)) / 2 = 50, two
# uniforms 6, proposal angle and its sin/cos 9, local field from 4 neighbours 6, energy change 5, Boltzmann test
# with exp 6, select/store 2  -> 84;  per site and sweep: sin/cos of its angle as a neighbour 9.
A_UPD = 84.0
A_SITE_SWEEP = 9.0
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
PEAK_LANE_OPS = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--p", type=float, default=0.6, help="gap fraction of the 4096^2 workload")
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--n-real", type=int, default=256)
    ap.add_argument("--roofline-sweeps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-sweeps", type=int, default=0)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the realizations would shard over "
              f"GPUs with a single all-reduce of the accumulator, which this build does not run.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2212_01317_amd as mpr
    from paper_2212_01317_amd import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    L = args.size
    R = args.n_real
    lb = (32, 32)
    t0 = time.time()
    sc = synth.config3(args.p, L, L)
    log(f"[bench] workload generated in {time.time() - t0:.1f}s: {L}x{L}, p={args.p}, gaps={int((sc.mask == 0).sum())}")
    z = torch.from_numpy(sc.z_obs).to(dev)
    mask = torch.from_numpy(sc.mask).to(dev)
    truth = torch.from_numpy(sc.z_true).to(dev)
    evm = torch.from_numpy(sc.eval_mask).to(dev)
    n_gap = int((sc.mask == 0).sum())
    state = torch.empty((R, L, L), dtype=torch.float32, device=dev)
    cfg = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_AUTO, n_samp=1, n_fit=20,
                        n_f=5, n_max=1000, seed=synth.seed_for(3, synth.ROLE_PHILOX))
    fixed = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_FIXED, n_eq=0, n_samp=0,
                          seed=cfg.seed)

    if args.profile_sweeps > 0:
        # counter runs: a small matching curve (T values do not change the traffic), the start, an even number of
        # sweeps, and a 1 GiB elementwise copy (read 1 GiB, write 1 GiB) that calibrates the byte counters
        small = dict(L=16, n_therm=20, n_meas=20, seed=1, decades=(-3, 2), per_decade=4)
        cT, ce = mpr.reference_curve(0.5, dev, spec=small)
        t, rng = mpr.mpr_map_angles(z, mask)
        T, _, _ = mpr.mpr_calibrate_temperature(t, mask, lb[0], lb[1], cT, ce)
        mpr.mpr_simulate(t, mask, T, lb[0], lb[1], fixed, state=state, want_energy=False)
        alt = state.clone()
        n = args.profile_sweeps + (args.profile_sweeps & 1)
        mpr.mpr_sweep(state, mask, T, lb[0], lb[1], fixed, 1, n, state_alt=alt)
        del alt
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log(f"[bench] profile run done: {n} sweeps, then a 1 GiB elementwise copy")
        return

    cT, ce = mpr.reference_curve(0.5, dev)          # a constant of the method, computed once per process
    ws_need = mpr.lib().mpr_simulate_workspace_bytes(L, L, lb[0], lb[1], ctypes.byref(cfg.to_c()))
    ws = torch.empty(ws_need, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        t, rng = mpr.mpr_map_angles(z, mask)
        T, _, _ = mpr.mpr_calibrate_temperature(t, mask, lb[0], lb[1], cT, ce)
        sim = mpr.mpr_simulate(t, mask, T, lb[0], lb[1], cfg, state=state, workspace=ws)
        zhat = mpr.mpr_predict(sim.acc, z, mask, R * cfg.n_samp, rng)
        err = mpr.mpr_validate(zhat, truth, evm)
        return sim, err, T

    for i in range(args.warmup):
        sim, err, T = step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i}: k*={sim.sweeps} converged={sim.converged}")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    updates = 0
    sweeps = []
    for i in range(args.steps):
        sim, err, T = step()
        sweeps.append(sim.sweeps + cfg.n_samp)
        updates += R * n_gap * (sim.sweeps + cfg.n_samp)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    errs = err.cpu().numpy()
    log(f"[bench] {args.steps} steps in {elapsed:.3f}s, sweeps/step {sweeps}, AAE {errs[0]:.5f} RASE {errs[1]:.5f}")

    # roofline of the dominant kernel (one fused sweep over all R realizations), timed with HIP events
    # on the stream the library launches on (torch's current stream)
    ns = args.roofline_sweeps + (args.roofline_sweeps & 1)        # even: the result ends in `state`
    k0 = sim.sweeps + cfg.n_samp + 1
    del ws
    alt = state.clone()
    mpr.mpr_sweep(state, mask, T, lb[0], lb[1], fixed, k0, 2, state_alt=alt)        # warm
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    mpr.mpr_sweep(state, mask, T, lb[0], lb[1], fixed, k0 + 2, ns, state_alt=alt)
    ev1.record()
    torch.cuda.synchronize()
    t_launch = ev0.elapsed_time(ev1) / 1e3 / ns
    upd_launch = float(R) * n_gap
    ops_launch = upd_launch * A_UPD + float(R) * L * L * A_SITE_SWEEP
    achieved = ops_launch / t_launch
    sweep_upd_rate = upd_launch / t_launch
    log(f"[bench] sweep launch {t_launch * 1e3:.3f} ms -> {sweep_upd_rate:.3e} upd/s in the sweep kernel")

    value = updates / elapsed
    out = {
        "metric": "SV-MPR gap-site updates/s at 4096^2 (C3)",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"SV-MPR {L}x{L} non-stationary field NS(8,[2,64]), p={args.p} blob-dominated gaps, "
                               f"32x32 T-blocks, {R} realizations, automatic equilibrium test (n_fit=20, n_f=5), "
                               f"1 sampling sweep; step = map+calibrate+simulate+predict+validate",
                   "H": L, "W": L, "p": args.p, "gap_sites": n_gap, "n_real": R, "block": list(lb),
                   "sweeps_per_step": sweeps},
        "roofline": {"bound": "alu", "kernel": "k_sweep_fused", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T lane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                     "launch_ms": t_launch * 1e3, "ops_per_launch": ops_launch,
                     "sweep_kernel_updates_per_s": sweep_upd_rate},
        "validation": {"aae": float(errs[0]), "rase": float(errs[1])},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, lb)
    print(json.dumps(out), flush=True)


def cpu_baseline(sc, lb):
    """The CPU oracle, single-threaded, on a bounded sample of the same workload: map + calibration + one realization
    of 2 realizations x (3 equilibration sweeps + 1 sampling sweep)."""
    import numpy as np

    import oracle
    Tg = np.geomspace(1e-3, 1e2, 31).astype(np.float32)
    e = oracle.reference_curve(Tg, L=24, n_therm=200, n_meas=300, seed=21)
    n_gap = int((sc.mask == 0).sum())
    t0 = time.perf_counter()
    t, rng = oracle.map_angles(sc.z_obs, sc.mask)
    T, _, _ = oracle.calibrate_temperature(t, sc.mask, lb[0], lb[1], Tg.astype(np.float64), e)
    res = oracle.simulate(t, sc.mask, T, lb[0], lb[1],
                          oracle.SimConfig(n_real=2, init_mode=1, stop_mode=0, n_eq=3, n_samp=1, seed=1))
    el = time.perf_counter() - t0
    upd = n_gap * 2 * 4
    log(f"[bench] cpu oracle: {upd} updates in {el:.1f}s")
    return {"value": upd / el, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"same 4096^2 input; map + calibration + 2 realizations x 4 sweeps ({upd} updates), "
                      f"{el:.1f} s single-threaded FP64"}


if __name__ == "__main__":
    main()
