"""SV-MPR gap filling on MI355X (gfx950): conditional Monte Carlo simulation of the modified planar rotator model
with block-specific temperatures (Lach & Zukovic, arXiv 2212.01317).

The compute runs in libmpr.so (HIP kernels behind the C ABI of include/mpr.h); this package is its thin binding.
``predict`` chains the ABI calls of one gap-filling run: map -> calibrate -> simulate -> predict.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from .autograd import MPRFunction
from ._lib import (INIT_BLOCK_MEAN, INIT_RANDOM, STOP_AUTO, STOP_AUTO_CHAIN, STOP_FIXED, T_BLOCK, T_SITE, ORDER_SC, ORDER_DC, SWEEP_AUTO, SWEEP_TILES, SWEEP_LANES, COUPLING_ISOTROPIC, COUPLING_DIRECTIONAL, MprError, SimConfig, SimOutput, lib,
                   mpr_block_stats, mpr_calibrate_temperature, mpr_calibrate_temperature_noalloc, mpr_calibrate_directional, mpr_map_angles, mpr_predict, mpr_reference_curve,
                   mpr_simulate, mpr_sweep, mpr_validate, mpr_block_energy, mpr_temperature_grad,
                   mpr_simulate_batched, BatchOutput, mpr_probe_instruction_rates, mpr_sst_temperatures,
                   mpr_calibrate_temperature3d, mpr_reference_curve3d, mpr_simulate3d)

__all__ = ["INIT_BLOCK_MEAN", "INIT_RANDOM", "STOP_AUTO", "STOP_AUTO_CHAIN", "STOP_FIXED", "T_BLOCK", "T_SITE", "ORDER_SC", "ORDER_DC", "SWEEP_AUTO", "SWEEP_TILES", "SWEEP_LANES", "COUPLING_ISOTROPIC", "COUPLING_DIRECTIONAL", "MprError", "SimConfig", "SimOutput",
           "lib", "mpr_block_stats", "mpr_calibrate_temperature", "mpr_calibrate_temperature_noalloc",
           "mpr_calibrate_directional", "mpr_map_angles",
           "mpr_predict",
           "mpr_reference_curve", "mpr_simulate", "mpr_sweep", "mpr_validate", "default_T_grid", "reference_curve", "predict",
           "Prediction", "CURVE_SPEC", "MPRFunction", "mpr_block_energy", "mpr_temperature_grad",
           "mpr_simulate_batched", "BatchOutput", "mpr_probe_instruction_rates", "mpr_sst_temperatures",
           "mpr_calibrate_temperature3d", "mpr_reference_curve3d", "mpr_simulate3d", "predict3d", "reference_curve3d",
           "CURVE3_SPEC"]

# The matching curve used by default: 121 temperatures log-spaced over [1e-3, 1e2] (24 per decade), periodic
# 128 x 128 lattice, 1000 sweeps to equilibrate and 2000 to average, fixed seed.
CURVE_SPEC = dict(L=128, n_therm=1000, n_meas=2000, seed=2212013170, decades=(-3, 2), per_decade=24)

_curve_cache: dict = {}


def default_T_grid(device="cuda") -> torch.Tensor:
    lo, hi = CURVE_SPEC["decades"]
    n = (hi - lo) * CURVE_SPEC["per_decade"] + 1
    T = [10.0 ** (lo + i / CURVE_SPEC["per_decade"]) for i in range(n)]
    return torch.tensor(T, dtype=torch.float32, device=device)


def reference_curve(q: float = 0.5, device="cuda", spec: dict | None = None):
    """(curve_T float64, curve_e float64) on the device, computed once per (q, spec) by mpr_reference_curve."""
    sp = dict(CURVE_SPEC if spec is None else spec)
    key = (float(q), str(torch.device(device)), tuple(sorted((k, str(v)) for k, v in sp.items())))
    if key not in _curve_cache:
        Tg = default_T_grid(device) if spec is None or "T_grid" not in sp else sp["T_grid"]
        e = mpr_reference_curve(Tg, L=sp["L"], n_therm=sp["n_therm"], n_meas=sp["n_meas"], seed=sp["seed"], q=q)
        _curve_cache[key] = (Tg.to(torch.float64), e)
    return _curve_cache[key]


# The matching curve of the cubic lattice used by predict3d by default: 41 temperatures log-spaced over [1e-3, 1e2]
# (8 per decade), periodic 32^3 lattice, 500 sweeps to equilibrate and 1000 to average, fixed seed.
CURVE3_SPEC = dict(L=32, n_therm=500, n_meas=1000, seed=2212013170, decades=(-3, 2), per_decade=8)


def reference_curve3d(q: float = 0.5, device="cuda", spec: dict | None = None):
    """(curve_T float64, curve_e float64) of the cubic lattice on the device, computed once per (q, spec) by
    mpr_reference_curve3d."""
    sp = dict(CURVE3_SPEC if spec is None else spec)
    key = ("3d", float(q), str(torch.device(device)), tuple(sorted((k, str(v)) for k, v in sp.items())))
    if key not in _curve_cache:
        lo, hi = sp["decades"]
        n = (hi - lo) * sp["per_decade"] + 1
        Tg = torch.tensor([10.0 ** (lo + i / sp["per_decade"]) for i in range(n)], dtype=torch.float32,
                          device=device)
        e = mpr_reference_curve3d(Tg, L=sp["L"], n_therm=sp["n_therm"], n_meas=sp["n_meas"], seed=sp["seed"], q=q)
        _curve_cache[key] = (Tg.to(torch.float64), e)
    return _curve_cache[key]


@dataclass
class Prediction:
    zhat: torch.Tensor         # [H, W] float32
    T: torch.Tensor            # [nby, nbx] float32 block temperatures
    sim: SimOutput
    range: torch.Tensor        # [2] float64 (zmin, zmax)


def predict(z: torch.Tensor, mask: torch.Tensor, block=(32, 32), n_real: int = 100, *, q: float = 0.5,
            J: float = 1.0, init_mode: int = INIT_BLOCK_MEAN, stop_mode: int = STOP_AUTO, n_eq: int = 50,
            n_samp: int = 1, n_fit: int = 20, n_f: int = 5, n_max: int = 1000, seed: int = 0, scene_id: int = 0,
            curve=None, T_blocks: torch.Tensor | None = None, sst: tuple | None = None,
            order: int = ORDER_SC, directional: bool = False) -> Prediction:
    """Fill the gaps (mask == 0) of z: Sec. 2.1 map, Sec. 2.2.2 block temperatures (block = (lb_h, lb_w); a block
    as large as the grid gives the plain MPR method), conditional simulation with the Sec. 3.4 stopping rule, and
    the conditional mean over n_real realizations x n_samp sampling sweeps.  sst = (r_s, n_s) gives the SST variant
    (Sec. 2.2.3): the block temperatures smoothed into one temperature per site; `T` is then that [H, W] map.
    order = ORDER_DC sweeps in the double-checkerboard order over the blocks (Sec. 2.2.2).  directional = True uses
    the directional coupling (one temperature per bond direction and block, the extension suggested in Sec. 4);
    `T` is then the [2, nby, nbx] stack (Tx, Ty)."""
    lb_h, lb_w = int(block[0]), int(block[1])
    t, rng = mpr_map_angles(z, mask)
    if T_blocks is None:
        cT, ce = reference_curve(q, z.device) if curve is None else curve
        if directional:
            T_blocks = torch.stack(mpr_calibrate_directional(t, mask, lb_h, lb_w, cT, ce, q, J))
        else:
            T_blocks, _, _ = mpr_calibrate_temperature(t, mask, lb_h, lb_w, cT, ce, q, J)
    t_mode = T_BLOCK
    if sst is not None:
        H, W = int(z.shape[-2]), int(z.shape[-1])
        T_blocks = mpr_sst_temperatures(T_blocks, H, W, lb_h, lb_w, int(sst[0]), int(sst[1]))
        t_mode = T_SITE
    cfg = SimConfig(q=q, J=J, n_real=n_real, init_mode=init_mode, stop_mode=stop_mode, n_eq=n_eq, n_samp=n_samp,
                    n_fit=n_fit, n_f=n_f, n_max=n_max, seed=seed, scene_id=scene_id, t_mode=t_mode, order=order,
                    coupling=COUPLING_DIRECTIONAL if directional else COUPLING_ISOTROPIC)
    sim = mpr_simulate(t, mask, T_blocks, lb_h, lb_w, cfg)
    zhat = mpr_predict(sim.acc, z, mask, n_real * n_samp, rng)
    return Prediction(zhat=zhat, T=T_blocks, sim=sim, range=rng)


def predict3d(z: torch.Tensor, mask: torch.Tensor, block=(32, 32, 32), n_real: int = 100, *, q: float = 0.5,
              J: float = 1.0, init_mode: int = INIT_BLOCK_MEAN, stop_mode: int = STOP_AUTO, n_eq: int = 50,
              n_samp: int = 1, n_fit: int = 20, n_f: int = 5, n_max: int = 1000, seed: int = 0, scene_id: int = 0,
              curve=None, T_blocks: torch.Tensor | None = None) -> Prediction:
    """Fill the gaps (mask == 0) of a [D, H, W] grid on the 3D lattice (the extension to three dimensions named in
    Sec. 4): the Sec. 2.1 map over the whole grid, temperatures per lb_d x lb_h x lb_w block from the cubic lattice's
    matching curve, the conditional simulation and the conditional mean.  The map, the prediction and their range
    are those of the plane, applied to the flattened grid."""
    D, H, W = (int(v) for v in z.shape)
    lb = tuple(int(v) for v in block)
    t2, rng = mpr_map_angles(z.reshape(D * H, W), mask.reshape(D * H, W))
    t = t2.view(D, H, W)
    if T_blocks is None:
        cT, ce = reference_curve3d(q, z.device) if curve is None else curve
        T_blocks, _, _ = mpr_calibrate_temperature3d(t, mask, *lb, cT, ce, q, J)
    cfg = SimConfig(q=q, J=J, n_real=n_real, init_mode=init_mode, stop_mode=stop_mode, n_eq=n_eq, n_samp=n_samp,
                    n_fit=n_fit, n_f=n_f, n_max=n_max, seed=seed, scene_id=scene_id)
    sim = mpr_simulate3d(t, mask, T_blocks, *lb, cfg)
    zhat = mpr_predict(sim.acc.view(D * H, W), z.reshape(D * H, W), mask.reshape(D * H, W), n_real * n_samp, rng)
    return Prediction(zhat=zhat.view(D, H, W), T=T_blocks, sim=sim, range=rng)
