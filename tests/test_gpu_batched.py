"""Batched simulation on the GPU: every scene of one persistent batched call equals its own single-scene call bit
for bit (states, accumulators, stopping sweep, energy series), whatever tile height the sweep kernel uses."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2212_01317_amd import _lib as M
from paper_2212_01317_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(70, 130, 0.5, 0), (200, 64, 0.3, 1), (33, 257, 0.8, 2), (128, 128, 0.6, 3), (16, 300, 0.4, 4),
          (5, 5, 0.5, 5), (1, 40, 0.5, 6), (97, 97, 0.9, 7)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _scenes(lb=(16, 16)):
    out = []
    for i, (H, W, p, seed) in enumerate(SHAPES):
        sc = synth.random_small(H, W, p, seed=100 + seed)
        sc.mask.ravel()[0] = 1
        t, _ = oracle.map_angles(sc.z_obs, sc.mask)
        B = (-(-H // lb[0])) * (-(-W // lb[1]))
        T = np.random.default_rng(seed).uniform(0.02, 0.5, B).astype(np.float32)
        out.append(dict(t=dev(t), mask=dev(sc.mask), T_blocks=dev(T), block=lb, scene_id=1000 + i))
    return out


@pytest.mark.parametrize("stop_mode", [M.STOP_AUTO, M.STOP_FIXED])
def test_lane_batch_with_few_realizations_equals_single_scene(stop_mode):
    """sweep_kernel = LANES sends a batch of 6 realizations (lanes 6 .. 63 idle) to the lane batch: every scene, down to
    1 x 40 and 5 x 5, equals its single-scene call (which sweeps on the tile kernel)."""
    scenes = _scenes()
    cfg = M.SimConfig(n_real=6, init_mode=M.INIT_BLOCK_MEAN, stop_mode=stop_mode, n_eq=13, n_samp=2, n_max=150,
                      seed=78, sweep_kernel=M.SWEEP_LANES)
    print(f"[batched] lane batch, 6 realizations, stop_mode {stop_mode}", flush=True)
    b = M.mpr_simulate_batched(scenes, cfg, want_energy=True)
    assert b.tile_h == 0
    for sc, out in zip(scenes, b.outputs):
        c1 = M.SimConfig(**{**cfg.__dict__, "scene_id": sc["scene_id"], "sweep_kernel": M.SWEEP_AUTO})
        single = M.mpr_simulate(sc["t"], sc["mask"], sc["T_blocks"], *sc["block"], c1)
        assert out.sweeps == single.sweeps
        assert out.converged == single.converged
        assert np.array_equal(host(out.state), host(single.state))
        assert np.array_equal(host(out.acc), host(single.acc))
        assert np.array_equal(host(out.energy), host(single.energy))


@pytest.mark.parametrize("stop_mode,tile_h", [(M.STOP_AUTO, 0), (M.STOP_AUTO, 16), (M.STOP_FIXED, 32)])
def test_batched_equals_single_scene(stop_mode, tile_h):
    scenes = _scenes()
    cfg = M.SimConfig(n_real=6, init_mode=M.INIT_BLOCK_MEAN, stop_mode=stop_mode, n_eq=13, n_samp=2, n_max=150,
                      seed=77)
    b = M.mpr_simulate_batched(scenes, cfg, tile_h=tile_h, want_energy=True)
    assert b.tile_h in (16, 32) and (tile_h == 0 or b.tile_h == tile_h)
    for sc, out in zip(scenes, b.outputs):
        c1 = M.SimConfig(**{**cfg.__dict__, "scene_id": sc["scene_id"]})
        single = M.mpr_simulate(sc["t"], sc["mask"], sc["T_blocks"], *sc["block"], c1)
        assert out.sweeps == single.sweeps
        assert np.array_equal(host(out.state), host(single.state))
        assert np.array_equal(host(out.acc), host(single.acc))
        assert np.array_equal(host(out.energy), host(single.energy))


def test_batched_lane_and_tile_batches_equal_single_scene():
    """With 64 realizations every scene, large or small, runs in the persistent lane batch (one launch per sweep for
    all scenes); sweep_kernel = TILES puts every scene in the persistent tile batch; every scene of either equals its
    single-scene call."""
    shapes = [(1024, 800, 0.6, 11), (70, 130, 0.5, 12), (33, 57, 0.7, 13)]
    scenes = []
    for i, (H, W, p, seed) in enumerate(shapes):
        sc = synth.random_small(H, W, p, seed=seed)
        t, _ = oracle.map_angles(sc.z_obs, sc.mask)
        B = (-(-H // 16)) * (-(-W // 16))
        T = np.random.default_rng(seed).uniform(0.02, 0.5, B).astype(np.float32)
        scenes.append(dict(t=dev(t), mask=dev(sc.mask), T_blocks=dev(T), block=(16, 16), scene_id=2000 + i))
    cfg = M.SimConfig(n_real=64, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_AUTO, n_samp=1, n_max=200, seed=5)
    print("[batched] lane batch and tile batch", flush=True)
    b = M.mpr_simulate_batched(scenes, cfg, want_energy=True)
    tiles = M.mpr_simulate_batched(scenes, M.SimConfig(**{**cfg.__dict__, "sweep_kernel": M.SWEEP_TILES}),
                                   want_energy=True)
    assert b.tile_h == 0 and tiles.tile_h in (16, 32)
    for sc, out, out_t in zip(scenes, b.outputs, tiles.outputs):
        single = M.mpr_simulate(sc["t"], sc["mask"], sc["T_blocks"], *sc["block"],
                                M.SimConfig(**{**cfg.__dict__, "scene_id": sc["scene_id"]}))
        for o in (out, out_t):
            assert o.sweeps == single.sweeps
            assert np.array_equal(host(o.state), host(single.state))
            assert np.array_equal(host(o.acc), host(single.acc))
            assert np.array_equal(host(o.energy), host(single.energy))
    L = M.lib()
    c_auto, c_tiles = cfg.to_c(), M.SimConfig(**{**cfg.__dict__, "sweep_kernel": M.SWEEP_TILES}).to_c()
    assert (L.mpr_simulate_workspace_bytes(1024, 800, 16, 16, ctypes.byref(c_auto))
            != L.mpr_simulate_workspace_bytes(1024, 800, 16, 16, ctypes.byref(c_tiles)))   # the lane sweep takes it
    only_lanes = M.mpr_simulate_batched(scenes[:1], cfg)
    assert only_lanes.tile_h == 0
    assert np.array_equal(host(only_lanes.outputs[0].state), host(b.outputs[0].state))


ORACLE_SHAPES = [(40, 52, 0.5, 21), (23, 70, 0.3, 22), (64, 31, 0.8, 23), (1, 45, 0.5, 24), (33, 33, 0.9, 25),
                 (9, 9, 0.4, 26)]


@pytest.mark.parametrize("kernel", ["auto", "lanes"])
def test_batched_matches_oracle(kernel):
    """Every scene of a batched call with the automatic stop against the oracle run of that scene (its own scene_id,
    all 64 realizations): the same stopping sweep (or a marginal slope where they differ), the energy series within
    1e-5 per bond, states equal at >= 99.99 % of (realization, site), the prediction's mean |dphi| <= 1e-3 rad.
    Both 'auto' (64 realizations) and 'lanes' run them in the persistent lane batch."""
    lb = (16, 16)
    R = 64
    host_scenes, scenes = [], []
    for i, (H, W, p, seed) in enumerate(ORACLE_SHAPES):
        sc = synth.random_small(H, W, p, seed=seed)
        sc.mask.ravel()[0] = 1
        t, _ = oracle.map_angles(sc.z_obs, sc.mask)
        B = (-(-H // lb[0])) * (-(-W // lb[1]))
        T = np.random.default_rng(seed).uniform(0.02, 0.5, B).astype(np.float32)
        host_scenes.append((t, sc.mask, T))
        scenes.append(dict(t=dev(t), mask=dev(sc.mask), T_blocks=dev(T), block=lb, scene_id=3000 + i))
    sk = M.SWEEP_LANES if kernel == "lanes" else M.SWEEP_AUTO
    cfg = M.SimConfig(n_real=R, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_AUTO, n_samp=1, n_max=150, seed=91,
                      sweep_kernel=sk)
    print(f"[batched vs oracle] {kernel}", flush=True)
    b = M.mpr_simulate_batched(scenes, cfg, want_energy=True)
    for i, ((t, mask, T), out) in enumerate(zip(host_scenes, b.outputs)):
        o = oracle.simulate(t, mask, T, *lb, oracle.SimConfig(n_real=R, init_mode=1, stop_mode=1, n_samp=1, n_max=150,
                                                              seed=91, scene=3000 + i), parallel=True)
        eg = host(out.energy)
        n = min(len(eg), len(o.energy))
        assert np.max(np.abs(eg[:n] - o.energy[:n])) <= 1e-5, i
        assert out.converged == o.converged, i
        if out.sweeps != o.k_star:
            k = min(out.sweeps, o.k_star)
            assert abs(oracle.ols_slope(o.energy[k - 19: k + 1])) < 1e-5, (i, out.sweeps, o.k_star)
            continue
        gs = host(out.state)
        assert float(np.mean(gs == o.state)) >= 0.9999, i
        gap = mask == 0
        dphi = 2 * np.pi * np.abs(host(out.acc)[gap] - o.acc[gap]) / R
        assert dphi.size == 0 or dphi.mean() <= 1e-3, i


def test_lane_batch_waits_for_inputs_on_the_callers_stream():
    """The lane batch spreads the scenes' starts over private streams forked from the caller's stream: inputs that a
    non-default caller stream is still producing (behind a ~20 ms spin kernel) must be complete before any start
    reads them, so the results equal those of the same call on inputs made ready beforehand."""
    scenes = _scenes()
    cfg = M.SimConfig(n_real=64, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_AUTO, n_samp=1, n_max=120, seed=91)
    ref = M.mpr_simulate_batched(scenes, cfg, want_energy=True)
    assert ref.tile_h == 0
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    print("[batched] lane batch on a side stream behind a spin kernel", flush=True)
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)
        late = [dict(sc, t=sc["t"].clone(), mask=sc["mask"].clone(), T_blocks=sc["T_blocks"].clone()) for sc in scenes]
        b = M.mpr_simulate_batched(late, cfg, want_energy=True)
    torch.cuda.synchronize()
    for o, r in zip(b.outputs, ref.outputs):
        assert o.sweeps == r.sweeps
        assert np.array_equal(host(o.state), host(r.state))
        assert np.array_equal(host(o.acc), host(r.acc))
        assert np.array_equal(host(o.energy), host(r.energy))
