"""Throughput benchmark of the SV-MPR hot path on one MI355X.

One step = one whole gap-filling pass over the 4096 x 4096 headline workload with inputs resident in HBM:
map to angles -> block temperatures (32 x 32 blocks) -> conditional simulation of 256 realizations with the
automatic equilibrium test and one sampling sweep -> prediction -> validation error (AAE/RASE) on the removed pixels.
value = gap-site updates per second = sum over steps of R * (gap sites) * (sweeps) / wall time of the steps.

Prints one JSON line.  --profile-sweeps N runs only the start and N sweeps (energy of each sweep, as in the
automatic stop) of the simulation, plus a 1 GiB device copy used to calibrate the HBM byte counters, and prints
nothing else; it is the command the counter profiles are taken with.
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

# Algorithmic VALU work of one gap-site update, in lane-operations priced by the issue cost of each instruction
# relative to a full-rate 32-bit add, as measured on the device (mpr_probe_instruction_rates):
#   half a Philox4x32-10 block (the two sites of a pair share one): 10 rounds x (2 v_mad_u64_u32 + 2 v_bitop3), each
#     instruction priced by the probe of a 64-bit product feeding a three-input xor (the round's own shape, so that a
#     product and an xor that issue together are priced together)
#   two uniforms: shift + v_cvt_f32_u32 each, plus the scale of the proposal
#   proposal angle, v_cos_f32, v_sin_f32
#   local field from four neighbours' (cos, sin): 6 adds;  energy change: 2 sub, mul, fma
#   Boltzmann test: fma (log2 of the ratio), v_exp_f32, compare;  select / store of t, cos, sin: 3
# and per site and sweep (every site of a realization, as a neighbour): its angle, v_cos_f32, v_sin_f32, and its share
# of the whole-grid energy that the stopping test reads after every sweep (6 lane-operations: the bond terms of the
# site and the fixed-point partial sum).
A_SITE_ENERGY = 6.0


def algorithmic_costs(r):
    pair = r["v_mad_u64_u32+v_bitop3_b32"]
    parts = {
        "philox_half_block": 10 * (2 * pair + 2 * pair) / 2,
        "uniforms": 2 * (1 + r["v_cvt_f32_u32"]) + 1,
        "proposal_sincos": 1 + r["v_sin_f32"] + r["v_cos_f32"],
        "local_field": 6.0,
        "energy_change": 4.0,
        "boltzmann_test": 2 + r["v_exp_f32"],
        "select_store": 3.0,
    }
    site = {"angle_sincos": 1 + r["v_sin_f32"] + r["v_cos_f32"], "energy": A_SITE_ENERGY}
    return sum(parts.values()), sum(site.values()), dict(parts, **{"site_" + k: v for k, v in site.items()})


# The pricing written before any measurement (quarter-rate 64-bit products and transcendentals): 82 lane-cycles per
# update plus 15 per site and sweep; reported beside the measured pricing for comparison.
A_UPDATE_NOMINAL, A_SITE_NOMINAL = 82.0, 15.0


# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
PEAK_LANE_OPS = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0


# The simulation sweeps with the realization-lane kernel when R >= 64 (one realization per lane), else with the
# fused tile kernel; the sources each kernel is built from, for matching a committed counter summary.
SWEEP_SOURCES = {
    "k_sweep_rl": ("rl_sweep.hip", "batched.hpp", "metropolis.hpp", "philox.hpp", "philox_lane.hpp", "mpr_internal.hpp"),
    "k_sweep_fused": ("sweep_body.hpp", "sweep.hip", "metropolis.hpp", "philox.hpp", "mpr_internal.hpp"),
}


def sweep_kernel(R: int, choice: str = "auto") -> str:
    """The kernel mpr_simulate sweeps with (at the 4096^2 workload the automatic choice is the realization-lane
    kernel exactly when R >= 64)."""
    if choice == "tiles":
        return "k_sweep_fused"
    if choice == "lanes":
        return "k_sweep_rl"
    return "k_sweep_rl" if R >= 64 else "k_sweep_fused"


def hbm_profile(kernel: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_c3_p0.6_hbm.txt")


def code_text(src: str) -> str:
    """C++ source without comments, trailing blanks and blank lines (what a counter summary's hash covers, so that
    editing a comment does not invalidate a measurement)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def sweep_sources_sha256(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2212_01317_amd", "csrc", name)) as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()


def measured_traffic(kernel: str, L: int, R: int, p: float):
    """HBM bytes per sweep launch from the committed counter summary (FETCH_SIZE and WRITE_SIZE, scaled by the
    counters' reading of a 1 GiB copy), if it was taken on this workload with the current sweep sources; else None."""
    path = hbm_profile(kernel)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        same = (kv.get("sources_sha256") == sweep_sources_sha256(kernel) and int(kv["size"]) == L
                and int(kv["n_real"]) == R and float(kv["p"]) == p)
        return float(kv["hbm_bytes_per_launch"]) if same else None
    except (KeyError, ValueError):
        return None


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
    ap.add_argument("--other-p", default="0.3,0.9",
                    help="further gap fractions of the 4096^2 workload, each timed and priced on its own ('' = none)")
    ap.add_argument("--other-p-steps", type=int, default=2)
    ap.add_argument("--profile-sweeps", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and gradient measurements")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched 256-scene measurement (for kernel traces of the batched sweep)")
    ap.add_argument("--lattice3d-only", action="store_true",
                    help="run only the 3D-lattice leg and print its object (for profiling its kernels)")
    ap.add_argument("--batch-scenes", type=int, default=256)
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes generating the batched scenes (1: in this process, e.g. under a profiler)")
    ap.add_argument("--sweep-kernel", choices=("auto", "tiles", "lanes"), default="auto",
                    help="sweep kernel of the simulation (auto: the library's choice)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def c3_leg(sc, p, R, lb, cT, ce, dev, steps, warmup, kchoice, kernel, roofline_sweeps, state):
    """The 4096^2 workload at gap fraction p: `warmup` untimed and `steps` timed steps (map -> calibrate -> simulate
    with the automatic stop -> predict -> validate, inputs resident in HBM), then the roofline of the sweep kernel at
    that p.  Returns the measured quantities and the step objects the extra legs reuse."""
    import torch

    import paper_2212_01317_amd as mpr
    from paper_2212_01317_amd import synth
    L = sc.z_obs.shape[0]
    z = torch.from_numpy(sc.z_obs).to(dev)
    mask = torch.from_numpy(sc.mask).to(dev)
    truth = torch.from_numpy(sc.z_true).to(dev)
    evm = torch.from_numpy(sc.eval_mask).to(dev)
    n_gap = int((sc.mask == 0).sum())
    cfg = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_AUTO, n_samp=1, n_fit=20,
                        n_f=5, n_max=1000, seed=synth.seed_for(3, synth.ROLE_PHILOX), sweep_kernel=kchoice)
    fixed = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_FIXED, n_eq=0, n_samp=0,
                          seed=cfg.seed, sweep_kernel=kchoice)
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

    for i in range(warmup):
        sim, err, T = step()
        torch.cuda.synchronize()
        log(f"[bench] p={p} warmup {i}: k*={sim.sweeps} converged={sim.converged}")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    updates = 0
    sweeps = []
    for i in range(steps):
        sim, err, T = step()
        sweeps.append(sim.sweeps + cfg.n_samp)
        updates += R * n_gap * (sim.sweeps + cfg.n_samp)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    errs = err.cpu().numpy()
    log(f"[bench] p={p}: {steps} steps in {elapsed:.3f}s, sweeps/step {sweeps}, AAE {errs[0]:.5f} RASE {errs[1]:.5f}")

    # Roofline of the dominant kernel: one sweep of all R realizations as the simulation runs it (with the energy
    # of the sweep, as under the automatic stop).  HIP events on the stream the library launches on (torch's
    # current stream) bracket two fixed-length simulations of the same start, n1 and n1 + ns sweeps; their
    # difference is ns sweeps, each one sweep launch plus the two small launches that reduce its energy.
    ns = roofline_sweeps
    n1 = 4

    def timed_simulation(n):
        c = mpr.SimConfig(**{**fixed.__dict__, "n_eq": n})
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        mpr.mpr_simulate(t, mask, T, lb[0], lb[1], c, state=state, workspace=ws, want_energy=True)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    t, _ = mpr.mpr_map_angles(z, mask)
    timed_simulation(n1)                                                          # warm
    t_launch = (timed_simulation(n1 + ns) - timed_simulation(n1)) / ns
    del ws
    upd_launch = float(R) * n_gap
    rates, add_ns = mpr.mpr_probe_instruction_rates(dev)
    a_upd, a_site, a_parts = algorithmic_costs(rates)
    log(f"[bench] instruction costs (v_add_u32 = 1): {rates}; A_update {a_upd:.2f}, A_site {a_site:.2f}")
    ops_launch = upd_launch * a_upd + float(R) * L * L * a_site
    achieved = ops_launch / t_launch
    sweep_upd_rate = upd_launch / t_launch
    log(f"[bench] p={p}: sweep launch {t_launch * 1e3:.3f} ms -> {sweep_upd_rate:.3e} upd/s in the sweep kernel, "
        f"ALU roofline fraction {achieved / PEAK_LANE_OPS:.3f}")
    traffic = measured_traffic(kernel, L, R, p)
    alg_bytes = float(R) * n_gap * 8.0              # 4 B read + 4 B written per gap site and realization
    roofline = {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "T lane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                "frac_nominal_pricing": (upd_launch * A_UPDATE_NOMINAL + float(R) * L * L * A_SITE_NOMINAL)
                / t_launch / PEAK_LANE_OPS,
                "traffic_gbs": traffic / t_launch / 1e9 if traffic else None,
                "algorithmic_bytes_per_launch": alg_bytes,
                "launch_ms": t_launch * 1e3, "ops_per_launch": ops_launch,
                "a_update": a_upd, "a_site": a_site, "a_parts": a_parts,
                "instruction_cost_vs_add": rates, "add_ns_per_wave_instruction": add_ns,
                "sweep_kernel_updates_per_s": sweep_upd_rate}
    return {"value": updates / elapsed, "ms_per_step": elapsed / steps * 1e3, "steps": steps, "sweeps": sweeps,
            "gap_sites": n_gap, "roofline": roofline, "aae": float(errs[0]), "rase": float(errs[1]),
            "cfg": cfg, "errs": errs}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the realizations would shard over "
              f"GPUs with a single all-reduce of the accumulator, which this build does not run.", file=sys.stderr)
        sys.exit(2)
    import numpy as np  # noqa: F401
    import torch

    import paper_2212_01317_amd as mpr
    from paper_2212_01317_amd import synth

    L = args.size
    R = args.n_real
    lb = (32, 32)
    t0 = time.time()
    sc = synth.config3(args.p, L, L)
    log(f"[bench] workload generated in {time.time() - t0:.1f}s: {L}x{L}, p={args.p}, gaps={int((sc.mask == 0).sum())}")
    extras_inputs = None
    other_p = [float(x) for x in args.other_p.split(",") if x.strip()] if args.profile_sweeps == 0 else []
    if (not args.no_extras or args.batched_only) and args.profile_sweeps == 0 and not args.lattice3d_only:
        # generated before the GPU is touched (worker processes are started from a process without a GPU context)
        t0 = time.time()
        scenes4 = synth.config4_scenes(args.batch_scenes, workers=max(1, min(args.gen_workers, os.cpu_count() or 1)))
        sc5 = synth.config5()
        extras_inputs = (scenes4, sc5)
        log(f"[bench] batched and gradient workloads generated in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.lattice3d_only:
        print(json.dumps({"lattice3d": bench_lattice3d(dev, R, float("nan"), L * L)}), flush=True)
        return
    if args.batched_only:
        cT, ce = mpr.reference_curve(0.5, dev)
        rates, _ = mpr.mpr_probe_instruction_rates(dev)
        a_upd, a_site, _ = algorithmic_costs(rates)
        print(json.dumps({"batched": bench_batched(extras_inputs[0], cT, ce, dev, a_upd, a_site)}), flush=True)
        return
    state = torch.empty((R, L, L), dtype=torch.float32, device=dev)
    kchoice = {"auto": mpr.SWEEP_AUTO, "tiles": mpr.SWEEP_TILES, "lanes": mpr.SWEEP_LANES}[args.sweep_kernel]
    kernel = sweep_kernel(R, args.sweep_kernel)

    if args.profile_sweeps > 0:
        # counter runs: a small matching curve (T values do not change the traffic), the start, an even number of
        # sweeps, and a 1 GiB elementwise copy (read 1 GiB, write 1 GiB) that calibrates the byte counters
        z = torch.from_numpy(sc.z_obs).to(dev)
        mask = torch.from_numpy(sc.mask).to(dev)
        small = dict(L=16, n_therm=20, n_meas=20, seed=1, decades=(-3, 2), per_decade=4)
        cT, ce = mpr.reference_curve(0.5, dev, spec=small)
        t, rng = mpr.mpr_map_angles(z, mask)
        T, _, _ = mpr.mpr_calibrate_temperature(t, mask, lb[0], lb[1], cT, ce)
        n = args.profile_sweeps
        prof = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_FIXED, n_eq=n, n_samp=0,
                             seed=synth.seed_for(3, synth.ROLE_PHILOX), sweep_kernel=kchoice)
        mpr.mpr_simulate(t, mask, T, lb[0], lb[1], prof, state=state, want_energy=True)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log(f"[bench] profile run done: {n} sweeps, then a 1 GiB elementwise copy")
        return

    cT, ce = mpr.reference_curve(0.5, dev)          # a constant of the method, computed once per process
    head = c3_leg(sc, args.p, R, lb, cT, ce, dev, args.steps, args.warmup, kchoice, kernel, args.roofline_sweeps,
                  state)
    n_gap, cfg, errs = head["gap_sites"], head["cfg"], head["errs"]
    out = {
        "metric": "SV-MPR gap-site updates/s at 4096^2 (C3)",
        "value": head["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"SV-MPR {L}x{L} non-stationary field NS(8,[2,64]), p={args.p} blob-dominated gaps, "
                               f"32x32 T-blocks, {R} realizations, automatic equilibrium test (n_fit=20, n_f=5), "
                               f"1 sampling sweep; step = map+calibrate+simulate+predict+validate",
                   "H": L, "W": L, "p": args.p, "gap_sites": n_gap, "n_real": R, "block": list(lb),
                   "sweep_kernel": kernel,
                   "sweeps_per_step": head["sweeps"]},
        "roofline": head["roofline"],
        "validation": {"aae": head["aae"], "rase": head["rase"]},
    }
    if other_p:
        # the other gap fractions of the same configuration: each its own step timing and its own roofline
        legs = {}
        for p in other_p:
            t0 = time.time()
            scp = synth.config3(p, L, L)
            log(f"[bench] workload generated in {time.time() - t0:.1f}s: {L}x{L}, p={p}")
            leg = c3_leg(scp, p, R, lb, cT, ce, dev, args.other_p_steps, 1, kchoice, kernel, args.roofline_sweeps,
                         state)
            legs[f"{p:g}"] = {k: v for k, v in leg.items() if k not in ("cfg", "errs")}
            del scp
        out["other_gap_fractions"] = legs
    if extras_inputs is not None:
        out["sst"] = bench_sst(sc, cT, ce, dev, state, R, lb, cfg, n_gap, errs)
        out["directional"] = bench_directional(sc, cT, ce, dev, state, R, lb, cfg, n_gap, errs)
        del state
        torch.cuda.empty_cache()
        out["lattice3d"] = bench_lattice3d(dev, R, head["roofline"]["launch_ms"], L * L)
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(extras_inputs[0], cT, ce, dev, head["roofline"]["a_update"],
                                       head["roofline"]["a_site"])
        torch.cuda.empty_cache()
        out["gradient"] = bench_gradient(extras_inputs[1], cT, ce, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, lb)
    print(json.dumps(out), flush=True)


def bench_directional(sc, cT, ce, dev, state, R, lb, cfg, n_gap, bst_errs):
    """The directional coupling (the extension suggested in Sec. 4) on the headline input: per block a temperature
    for the horizontal and one for the vertical sample bonds, the same simulation otherwise (AUTO, 1 sampling sweep);
    one warm-up and one timed step (map, directional calibration, simulate, predict, validate)."""
    import dataclasses

    import torch

    import paper_2212_01317_amd as mpr
    L = sc.z_obs.shape[0]
    z = torch.from_numpy(sc.z_obs).to(dev)
    mask = torch.from_numpy(sc.mask).to(dev)
    truth = torch.from_numpy(sc.z_true).to(dev)
    evm = torch.from_numpy(sc.eval_mask).to(dev)
    c_dir = dataclasses.replace(cfg, coupling=mpr.COUPLING_DIRECTIONAL, sweep_kernel=mpr.SWEEP_AUTO)
    ws = torch.empty(mpr.lib().mpr_simulate_workspace_bytes(L, L, lb[0], lb[1], ctypes.byref(c_dir.to_c())),
                     dtype=torch.uint8, device=dev)

    def step():
        t, rng = mpr.mpr_map_angles(z, mask)
        Tx, Ty = mpr.mpr_calibrate_directional(t, mask, lb[0], lb[1], cT, ce)
        sim = mpr.mpr_simulate(t, mask, torch.stack([Tx, Ty]), lb[0], lb[1], c_dir, state=state, workspace=ws)
        zhat = mpr.mpr_predict(sim.acc, z, mask, R * c_dir.n_samp, rng)
        return sim, mpr.mpr_validate(zhat, truth, evm)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim, err = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    e = err.cpu().numpy()
    upd = R * n_gap * (sim.sweeps + c_dir.n_samp)
    log(f"[bench] directional: {sim.sweeps} + 1 sweeps in {el:.3f}s ({upd / el:.3e} upd/s), AAE {e[0]:.5f} "
        f"RASE {e[1]:.5f} (BST {bst_errs[0]:.5f} / {bst_errs[1]:.5f})")
    return {"workload": "headline input, directional coupling (Tx, Ty per block), AUTO, 1 sampling sweep",
            "seconds_per_step": el, "sweeps": sim.sweeps + c_dir.n_samp, "updates_per_s": upd / el,
            "aae": float(e[0]), "rase": float(e[1]), "bst_aae": float(bst_errs[0]), "bst_rase": float(bst_errs[1])}


def bench_sst(sc, cT, ce, dev, state, R, lb, cfg, n_gap, bst_errs):
    """The SST variant (Sec. 2.2.3) on the headline input: the block temperatures smoothed by n_s = 5 passes of the
    radius-1 window mean into one temperature per site, the same simulation otherwise (AUTO, 1 sampling sweep);
    one warm-up and one timed step (map, calibrate, smooth, simulate, predict, validate)."""
    import dataclasses

    import torch

    import paper_2212_01317_amd as mpr
    L = sc.z_obs.shape[0]
    z = torch.from_numpy(sc.z_obs).to(dev)
    mask = torch.from_numpy(sc.mask).to(dev)
    truth = torch.from_numpy(sc.z_true).to(dev)
    evm = torch.from_numpy(sc.eval_mask).to(dev)
    c_sst = dataclasses.replace(cfg, t_mode=mpr.T_SITE)
    ws = torch.empty(mpr.lib().mpr_simulate_workspace_bytes(L, L, lb[0], lb[1], ctypes.byref(c_sst.to_c())),
                     dtype=torch.uint8, device=dev)

    def step():
        t, rng = mpr.mpr_map_angles(z, mask)
        T, _, _ = mpr.mpr_calibrate_temperature(t, mask, lb[0], lb[1], cT, ce)
        Ts = mpr.mpr_sst_temperatures(T, L, L, lb[0], lb[1], 1, 5)
        sim = mpr.mpr_simulate(t, mask, Ts, lb[0], lb[1], c_sst, state=state, workspace=ws)
        zhat = mpr.mpr_predict(sim.acc, z, mask, R * c_sst.n_samp, rng)
        return sim, mpr.mpr_validate(zhat, truth, evm)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim, err = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    e = err.cpu().numpy()
    upd = R * n_gap * (sim.sweeps + c_sst.n_samp)
    log(f"[bench] SST: {sim.sweeps} + 1 sweeps in {el:.3f}s ({upd / el:.3e} upd/s), AAE {e[0]:.5f} RASE {e[1]:.5f} "
        f"(BST {bst_errs[0]:.5f} / {bst_errs[1]:.5f})")
    return {"workload": "headline input, SST with r_s = 1, n_s = 5 (one temperature per site), AUTO, 1 sampling sweep",
            "seconds_per_step": el, "sweeps": sim.sweeps + c_sst.n_samp, "updates_per_s": upd / el,
            "aae": float(e[0]), "rase": float(e[1]), "bst_aae": float(bst_errs[0]), "bst_rase": float(bst_errs[1])}


def bench_lattice3d(dev, R, plane_sweep_ms, plane_sites):
    """The 3D lattice (the extension to three dimensions of Sec. 4) at the plane's site count: 256^3 GRF stand-in,
    60 % of the sites removed uniformly, 32^3 temperature blocks calibrated on a matching curve of the cubic
    lattice, R realizations.  Time of one sweep with its energy (as under the automatic stop), by HIP events around
    two fixed-length simulations of the same start, against the plane's sweep at the same site count."""
    import numpy as np
    import torch

    import paper_2212_01317_amd as mpr
    from paper_2212_01317_amd import synth
    L, lb = 256, (32, 32, 32)
    t0 = time.time()
    f, m = synth.config3d(L, 0.6)
    log(f"[bench] 3D workload generated in {time.time() - t0:.1f}s")
    z = torch.from_numpy(f * m).to(dev)
    mask = torch.from_numpy(m).to(dev)
    t2, _ = mpr.mpr_map_angles(z.view(L * L, L), mask.view(L * L, L))
    t = t2.view(L, L, L)
    cT = torch.from_numpy(np.geomspace(1e-3, 1e2, 41).astype(np.float32)).to(dev)
    ce = mpr.mpr_reference_curve3d(cT, L=32, n_therm=300, n_meas=300, seed=1)
    T, _, _ = mpr.mpr_calibrate_temperature3d(t, mask, *lb, cT.double(), ce)
    n_gap = int((m == 0).sum())
    state = torch.empty((R, L, L, L), dtype=torch.float32, device=dev)

    def timed(n):
        c = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_FIXED, n_eq=n, n_samp=0,
                          seed=synth.seed_for(7, synth.ROLE_PHILOX))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        mpr.mpr_simulate3d(t, mask, T, *lb, c, state=state, want_energy=True)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    timed(2)
    ns = 10
    t_sweep = (timed(2 + ns) - timed(2)) / ns
    del state
    torch.cuda.empty_cache()
    log(f"[bench] 3D: {L}^3 R={R}: sweep {t_sweep * 1e3:.3f} ms -> {R * n_gap / t_sweep:.3e} upd/s, "
        f"{t_sweep * 1e3 / plane_sweep_ms:.2f}x the plane's sweep at {plane_sites} sites")
    return {"workload": f"{L}^3 GRF (xi=8), p=0.6 uniform gaps, {lb[0]}^3 T-blocks, {R} realizations, six neighbours",
            "sites": L ** 3, "gap_sites": n_gap, "sweep_ms": t_sweep * 1e3, "updates_per_s": R * n_gap / t_sweep,
            "plane_sweep_ms_same_sites": plane_sweep_ms, "plane_sites": plane_sites,
            "time_ratio_vs_plane": t_sweep * 1e3 / plane_sweep_ms,
            "mean_T": float(T.double().mean())}


def bench_batched(scenes, cT, ce, dev, a_upd, a_site):
    """Config 4: 256 scenes of uneven size and gap fraction, 64 realizations each, automatic stopping, in one
    batched call (timed after one untimed call); then the same scenes through one single-scene call each
    (bit-identical results, so equal MAE).
    The ALU fraction of each is the sweeps' lane-operations (A_update per update, A_site per site and sweep, priced
    as for the headline kernel) over the whole call's time: a lower bound on the sweep kernel's own fraction, since
    the call also holds the per-sweep energy, test and sampling kernels and the host's reads between chunks."""
    import numpy as np
    import torch

    import paper_2212_01317_amd as mpr
    R = 64
    cfg = mpr.SimConfig(n_real=R, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_AUTO, n_samp=1, n_max=1000,
                        seed=2212013170 + 402)
    items, gaps = [], []
    for i, sc in enumerate(scenes):
        z, m = torch.from_numpy(sc.z_obs).to(dev), torch.from_numpy(sc.mask).to(dev)
        t, rng = mpr.mpr_map_angles(z, m)
        T, _, _ = mpr.mpr_calibrate_temperature(t, m, 16, 16, cT, ce)
        items.append(dict(t=t, mask=m, T_blocks=T, block=(16, 16), scene_id=i, z=z, rng=rng,
                          truth=torch.from_numpy(sc.z_true).to(dev), ev=torch.from_numpy(sc.eval_mask).to(dev)))
        gaps.append(int((sc.mask == 0).sum()))
    # one untimed call first, as for the headline step: the library's streams, the allocator's blocks for the
    # outputs and the workspace exist from then on
    warm = mpr.mpr_simulate_batched(items, cfg, tile_h=0)
    del warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = mpr.mpr_simulate_batched(items, cfg, tile_h=0)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    upd = sum(R * g * (o.sweeps + cfg.n_samp) for g, o in zip(gaps, b.outputs))
    ops = sum(R * (o.sweeps + cfg.n_samp) * (g * a_upd + sc.z_true.size * a_site)
              for g, o, sc in zip(gaps, b.outputs, scenes))
    maes = []
    for it, o in zip(items, b.outputs):
        zh = mpr.mpr_predict(o.acc, it["z"], it["mask"], R, it["rng"])
        maes.append(float(mpr.mpr_validate(zh, it["truth"], it["ev"])[0]))
    del b
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    accs = []
    for i, it in enumerate(items):
        c1 = mpr.SimConfig(**{**cfg.__dict__, "scene_id": i})
        accs.append(mpr.mpr_simulate(it["t"], it["mask"], it["T_blocks"], 16, 16, c1, want_energy=False).acc)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    maes1 = []
    for it, acc in zip(items, accs):
        zh = mpr.mpr_predict(acc, it["z"], it["mask"], R, it["rng"])
        maes1.append(float(mpr.mpr_validate(zh, it["truth"], it["ev"])[0]))
    del accs
    sites = sum(sc.z_true.size for sc in scenes)
    log(f"[bench] batched: {len(scenes)} scenes, {sites} sites, {upd:.3e} updates: {t_batch:.2f}s batched, "
        f"{t_single:.2f}s as single-scene calls")
    return {"workload": f"{len(scenes)} scenes, sides log-uniform in [64, 2048], p ~ U[0.1, 0.9], NS(4,[2,32]), "
                        f"16x16 T-blocks, {R} realizations each, automatic stopping, 1 sampling sweep",
            "sites": sites, "updates": upd, "seconds": t_batch, "updates_per_s": upd / t_batch,
            "single_scene_seconds": t_single, "single_scene_updates_per_s": upd / t_single,
            "speedup_vs_single_scene": t_single / t_batch,
            "alu_frac_of_call": ops / t_batch / PEAK_LANE_OPS,
            "alu_frac_of_call_single_scene": ops / t_single / PEAK_LANE_OPS,
            "mean_validation_mae": float(np.mean(maes)),
            "mean_validation_mae_single_scene": float(np.mean(maes1)),
            "max_abs_mae_difference_vs_single_scene": float(np.max(np.abs(np.array(maes) - np.array(maes1))))}


def bench_gradient(sc, cT, ce, dev):
    """Config 5: 512^2, 16 x 16 temperature map, 1024 realizations, 60 + 1 sweeps.  Times the plain form (simulate +
    predict), the autograd forward (the same plus the block energies) and the backward (d validation MAE / dT by the
    covariance estimator); the three share the chains, so the validation MAE is the same.  Then the estimator against
    central differences with common random numbers (dT = 1e-3 T_b, 4 seeds) where the derivative is measurable:
    block temperatures U[0.3, 1.2] and a loss confined to one block (the mean over its gap sites of
    sign(1/2 - tbar) zhat), on the six partially gapped blocks with the highest T."""
    import numpy as np
    import torch

    import paper_2212_01317_amd as mpr
    lb = sc.block
    z, m = torch.from_numpy(sc.z_obs).to(dev), torch.from_numpy(sc.mask).to(dev)
    truth = torch.from_numpy(sc.z_true).to(dev)
    ev = torch.from_numpy(sc.eval_mask.astype(bool)).to(dev)
    t, rng = mpr.mpr_map_angles(z, m)
    T, _, _ = mpr.mpr_calibrate_temperature(t, m, lb[0], lb[1], cT, ce)

    def cfg_for(seed):
        return mpr.SimConfig(n_real=1024, init_mode=mpr.INIT_BLOCK_MEAN, stop_mode=mpr.STOP_FIXED, n_eq=60, n_samp=1,
                             seed=seed)
    cfg = cfg_for(2212013170 + 502)
    loss = lambda zh: (zh.double() - truth.double()).abs()[ev].mean()     # FP64: FD steps move it by ~1e-7
    Tm = T.clone().requires_grad_(True)
    loss(mpr.MPRFunction.apply(Tm, t, m, z, rng, lb, cfg)).backward()      # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = mpr.mpr_simulate(t, m, T, lb[0], lb[1], cfg, want_energy=False)
    L_plain = loss(mpr.mpr_predict(sim.acc, z, m, cfg.n_real, rng))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Tm = T.clone().requires_grad_(True)
    L0 = loss(mpr.MPRFunction.apply(Tm, t, m, z, rng, lb, cfg))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    L0.backward()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    gaps = int((sc.mask == 0).sum())
    log(f"[bench] gradient: plain {t1 - t0:.3f}s forward {t2 - t1:.3f}s backward {t3 - t2:.4f}s, "
        f"MAE {float(L_plain):.6f} / {float(L0):.6f}")

    # derivative check where it is measurable
    T_host = np.random.default_rng(7).uniform(0.3, 1.2, 256).astype(np.float32).reshape(16, 16)
    gapn = (sc.mask == 0).astype(np.int64).reshape(16, 32, 16, 32).sum(axis=(1, 3)).ravel()
    cand = np.flatnonzero((gapn >= 200) & (gapn <= 800))
    blocks = cand[np.argsort(-T_host.ravel()[cand], kind="stable")[:6]]
    Th = torch.from_numpy(T_host).to(dev)
    tbar = mpr.mpr_simulate(t, m, Th, lb[0], lb[1], cfg_for(99), want_energy=False).state.double().mean(0)
    gap = m == 0
    Cs = {}
    for bidx in blocks:
        by, bx = divmod(int(bidx), 16)
        C = torch.zeros_like(tbar)
        sl = (slice(by * 32, by * 32 + 32), slice(bx * 32, bx * 32 + 32))
        C[sl] = torch.sign(0.5 - tbar[sl]) * gap[sl] / float(gapn[bidx])
        Cs[int(bidx)] = C
    seeds = [1000 + i for i in range(4)]
    est = np.zeros((len(seeds), len(blocks)))
    fd = np.zeros_like(est)
    for i, seed in enumerate(seeds):
        c = cfg_for(seed)
        Tg = Th.clone().requires_grad_(True)
        zh = mpr.MPRFunction.apply(Tg, t, m, z, rng, lb, c)
        for j, bidx in enumerate(blocks):
            C = Cs[int(bidx)]
            (g,) = torch.autograd.grad((zh.double() * C).sum(), Tg, retain_graph=j + 1 < len(blocks))
            est[i, j] = float(g.double().ravel()[bidx])
            v = []
            for sgn in (1, -1):
                Tp = T_host.copy().ravel()
                Tp[bidx] *= 1 + sgn * 1e-3
                s2 = mpr.mpr_simulate(t, m, torch.from_numpy(Tp.reshape(16, 16)).to(dev), lb[0], lb[1], c,
                                      want_energy=False)
                v.append(float((mpr.mpr_predict(s2.acc, z, m, c.n_real, rng).double() * C).sum()))
            fd[i, j] = (v[0] - v[1]) / (2e-3 * T_host.ravel()[bidx])
    n = len(seeds)
    me, mf = est.mean(0), fd.mean(0)
    se_e, se_f = est.std(0, ddof=1) / np.sqrt(n), fd.std(0, ddof=1) / np.sqrt(n)
    zs = (me - mf) / np.sqrt(se_e ** 2 + se_f ** 2)
    ratio = float(me.sum() / mf.sum())
    log(f"[bench] gradient check: estimator {np.round(me, 4)} FD {np.round(mf, 4)} z {np.round(zs, 2)} "
        f"ratio {ratio:.3f}")
    return {"workload": "512x512 NS(4,[2,32]), 50% missing + 5% held out, 16x16 T-map, 1024 realizations, 60 + 1 "
                        "sweeps",
            "plain_s": t1 - t0, "forward_s": t2 - t1, "backward_s": t3 - t2,
            "plain_updates_per_s": 1024 * gaps * 61 / (t1 - t0),
            "forward_backward_over_plain": (t3 - t1) / (t1 - t0),
            "validation_mae_plain": float(L_plain), "validation_mae_forward": float(L0),
            "fd_check": {"temperatures": "U[0.3, 1.2] per block", "loss": "block-confined sign(1/2 - tbar) zhat",
                         "seeds": n, "dT": "1e-3 T_b", "blocks": [int(x) for x in blocks],
                         "estimator": [float(x) for x in me], "estimator_se": [float(x) for x in se_e],
                         "central_differences": [float(x) for x in mf], "central_differences_se": [float(x) for x in se_f],
                         "z": [float(x) for x in zs], "sum_ratio": ratio}}


def host_cpu():
    """CPU model and logical CPU count of this host (lscpu, else /proc/cpuinfo), and the CPUs this process may use."""
    import subprocess
    model, ncpu = None, None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name" and model is None:
                model = v.strip()
            if k.strip() == "CPU(s)" and ncpu is None:
                ncpu = int(v.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, ncpu, usable


def cpu_baseline(sc, lb):
    """The CPU oracle on this host's cores, on bounded samples of the benchmark's workloads (about 25 s):
    the 4096^2 input (map + calibration + 4 sweeps of 2 realizations single-threaded, and of 2 realizations per thread
    with the OpenMP build, realizations spread over threads), and the 128^2 plain-MPR configuration (10 realizations,
    100 + 100 sweeps) in full, both builds.  value = the OpenMP rate on the 4096^2 sample."""
    import numpy as np

    import oracle
    from paper_2212_01317_amd import synth
    model, ncpu, usable = host_cpu()
    nthr = oracle.threads(parallel=True)
    Tg = np.geomspace(1e-3, 1e2, 31).astype(np.float32)
    e = oracle.reference_curve(Tg, L=24, n_therm=200, n_meas=300, seed=21)
    n_gap = int((sc.mask == 0).sum())

    def c3(parallel, R):
        t0 = time.perf_counter()
        t, rng = oracle.map_angles(sc.z_obs, sc.mask)
        T, _, _ = oracle.calibrate_temperature(t, sc.mask, lb[0], lb[1], Tg.astype(np.float64), e)
        oracle.simulate(t, sc.mask, T, lb[0], lb[1],
                        oracle.SimConfig(n_real=R, init_mode=1, stop_mode=0, n_eq=3, n_samp=1, seed=1),
                        parallel=parallel)
        el = time.perf_counter() - t0
        return n_gap * R * 4 / el, el

    one, el1 = c3(False, 2)
    par, elp = c3(True, 2 * nthr)
    c1 = synth.config1()
    n1 = int((c1.mask == 0).sum())

    def c1_full(parallel):
        t0 = time.perf_counter()
        t, rng = oracle.map_angles(c1.z_obs, c1.mask)
        T, _, _ = oracle.calibrate_temperature(t, c1.mask, 128, 128, Tg.astype(np.float64), e)
        res = oracle.simulate(t, c1.mask, T, 128, 128,
                              oracle.SimConfig(n_real=10, init_mode=0, stop_mode=0, n_eq=100, n_samp=100, seed=1),
                              parallel=parallel)
        oracle.predict(res.acc, c1.z_obs, c1.mask, 1000, rng)
        return time.perf_counter() - t0

    c1_one, c1_par = c1_full(False), c1_full(True)
    log(f"[bench] cpu oracle on {model} ({usable} usable CPUs): 4096^2 sample {one:.3e} upd/s on 1 thread, "
        f"{par:.3e} on {nthr}; 128^2 in full {c1_one:.2f}s / {c1_par:.2f}s")
    return {"value": par, "unit": "site-updates/s", "cores": nthr, "kind": "oracle",
            "cpu_model": model, "host_logical_cpus": ncpu, "usable_cpus": usable,
            "sample": f"4096^2 input of the benchmark; map + calibration + {2 * nthr} realizations x 4 sweeps "
                      f"({n_gap * 2 * nthr * 4} updates) in {elp:.1f}s with the OpenMP build of the FP64 oracle "
                      f"(realizations over {nthr} threads)",
            "single_thread": {"value": one, "sample": f"2 realizations x 4 sweeps, {el1:.1f}s"},
            "config1_full": {"workload": "128^2 GRF(8), 33% gaps, global T, 10 realizations, 100 + 100 sweeps",
                             "updates": n1 * 10 * 200, "seconds_1_thread": c1_one, "seconds_openmp": c1_par,
                             "openmp_threads": nthr, "updates_per_s_1_thread": n1 * 2000 / c1_one,
                             "updates_per_s_openmp": n1 * 2000 / c1_par}}


if __name__ == "__main__":
    main()
