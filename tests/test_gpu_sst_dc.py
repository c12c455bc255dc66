"""SST (Sec. 2.2.3, site-specific temperatures) and the double-checkerboard order (Sec. 2.2.2) on the GPU against the
oracle: the smoothed temperature plane bit for bit; conditional simulations with one temperature per site and in
the double-checkerboard order (same chains, same predictions), on ragged grids and on sampled realizations of the
1024^2 configuration."""
import numpy as np
import pytest
import torch

import oracle
from oracle import SimConfig as OCfg
from paper_2212_01317_amd import _lib as M
from paper_2212_01317_amd import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("H,W,lb,r_s,n_s", [(37, 53, (8, 8), 1, 5), (37, 53, (8, 8), 2, 3), (64, 96, (16, 32), 1, 0),
                                            (5, 7, (3, 2), 3, 4), (1, 40, (1, 8), 1, 2)])
def test_sst_plane_matches_oracle(H, W, lb, r_s, n_s):
    nb = ((H + lb[0] - 1) // lb[0], (W + lb[1] - 1) // lb[1])
    T = np.random.default_rng(H * W + r_s).uniform(0.0, 0.6, nb).astype(np.float32)
    T.ravel()[0] = 0.0
    g = host(M.mpr_sst_temperatures(dev(T), H, W, lb[0], lb[1], r_s, n_s))
    o = oracle.sst_temperatures(T, H, W, lb[0], lb[1], r_s=r_s, n_s=n_s)
    assert np.array_equal(g, o)


@pytest.mark.parametrize("stop", ["fixed", "auto"])
def test_sst_simulation_matches_oracle(stop):
    sc = synth.random_small(45, 70, 0.55, seed=31)
    lb = (16, 16)
    t, rg = oracle.map_angles(sc.z_obs, sc.mask)
    T = np.random.default_rng(3).uniform(0.02, 0.3, (3, 5)).astype(np.float32)
    Ts = oracle.sst_temperatures(T, 45, 70, *lb, r_s=1, n_s=5)
    if stop == "fixed":
        oc = OCfg(n_real=6, init_mode=1, stop_mode=0, n_eq=25, n_samp=3, seed=12, t_mode=1)
        cfg = M.SimConfig(n_real=6, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=25, n_samp=3, seed=12,
                          t_mode=M.T_SITE)
    else:
        oc = OCfg(n_real=4, init_mode=1, stop_mode=1, n_samp=2, n_max=200, seed=13, t_mode=1)
        cfg = M.SimConfig(n_real=4, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_AUTO, n_samp=2, n_max=200, seed=13,
                          t_mode=M.T_SITE)
    o = oracle.simulate(t, sc.mask, Ts, *lb, oc)
    g = M.mpr_simulate(dev(t), dev(sc.mask), dev(Ts), *lb, cfg)
    assert g.sweeps == o.k_star
    assert np.array_equal(host(g.state), o.state)
    assert np.array_equal(host(g.acc), o.acc)
    assert np.allclose(host(g.energy), o.energy, rtol=0, atol=1e-5)
    n = cfg.n_real * cfg.n_samp
    zo = oracle.predict(o.acc, sc.z_obs, sc.mask, n, rg)
    zg = host(M.mpr_predict(g.acc, dev(sc.z_obs), dev(sc.mask), n, dev(rg)))
    assert np.array_equal(zg, zo)


def test_sst_fullsize_sampled_realizations():
    """1024^2 (C2 field and mask, 16^2 blocks, T map from the library's calibration smoothed with r_s = 1,
    n_s = 5), 100 realizations on the GPU; realizations 0 and 57 recomputed by the oracle one by one."""
    sc = synth.config2()
    lb = (16, 16)
    z, m = dev(sc.z_obs), dev(sc.mask)
    t, rg = M.mpr_map_angles(z, m)
    T_curve = np.geomspace(1e-3, 1e2, 31).astype(np.float32)
    e_curve = oracle.reference_curve(T_curve, L=16, n_therm=40, n_meas=40, seed=5)
    T, _, _ = M.mpr_calibrate_temperature(t, m, *lb, dev(T_curve.astype(np.float64)), dev(e_curve))
    Ts = M.mpr_sst_temperatures(T, 1024, 1024, *lb, 1, 5)
    cfg = M.SimConfig(n_real=100, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=2, n_samp=1, seed=77,
                      t_mode=M.T_SITE)
    g = M.mpr_simulate(t, m, Ts, *lb, cfg, want_energy=False)
    gs, t_h, Ts_h = host(g.state), host(t), host(Ts)
    assert np.array_equal(Ts_h, oracle.sst_temperatures(host(T), 1024, 1024, *lb, r_s=1, n_s=5))
    for r in (0, 57):
        o = oracle.simulate(t_h, sc.mask, Ts_h, *lb, OCfg(n_real=1, real_offset=r, init_mode=1, stop_mode=0, n_eq=2,
                                                          n_samp=1, seed=77, t_mode=1))
        agree = float(np.mean(gs[r] == o.state[0]))
        print(f"realization {r}: agreement {agree:.7f}", flush=True)
        assert agree >= 0.9999


def test_sst_error_paths():
    sc = synth.random_small(20, 24, 0.5, seed=2)
    t, m = dev(sc.z_obs * 0 + 0.5), dev(sc.mask)
    T = dev(np.full((2, 2), 0.1, np.float32))
    cfg = M.SimConfig(n_real=2, stop_mode=M.STOP_FIXED, n_eq=1, t_mode=M.T_SITE)
    with pytest.raises(ValueError):
        M.mpr_simulate(t, m, T, 16, 16, cfg)           # a block map where one temperature per site is needed
    with pytest.raises(ValueError):
        M.mpr_sst_temperatures(T, 20, 24, 8, 8)       # 3 x 3 blocks expected
    with pytest.raises(M.MprError):
        M.mpr_sst_temperatures(T, 20, 24, 16, 16, -1, 2)
    scene = dict(t=t, mask=m, T_blocks=dev(np.full(20 * 24, 0.1, np.float32)), block=(16, 16), scene_id=0)
    with pytest.raises(M.MprError):
        M.mpr_simulate_batched([scene], cfg, tile_h=0)


@pytest.mark.parametrize("lb,stop,sst", [((8, 8), "fixed", False), ((16, 12), "auto", False), ((10, 14), "fixed", True)])
def test_double_checkerboard_matches_oracle(lb, stop, sst):
    sc = synth.random_small(47, 61, 0.5, seed=37)
    t, rg = oracle.map_angles(sc.z_obs, sc.mask)
    nb = ((47 + lb[0] - 1) // lb[0], (61 + lb[1] - 1) // lb[1])
    T = np.random.default_rng(lb[0]).uniform(0.02, 0.3, nb).astype(np.float32)
    t_mode = 0
    if sst:
        T = oracle.sst_temperatures(T, 47, 61, *lb, r_s=1, n_s=3)
        t_mode = 1
    if stop == "fixed":
        oc = OCfg(n_real=5, init_mode=1, stop_mode=0, n_eq=20, n_samp=2, seed=21, t_mode=t_mode, order=1)
        cfg = M.SimConfig(n_real=5, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=20, n_samp=2, seed=21,
                          t_mode=t_mode, order=M.ORDER_DC)
    else:
        oc = OCfg(n_real=4, init_mode=1, stop_mode=1, n_samp=1, n_max=150, seed=22, t_mode=t_mode, order=1)
        cfg = M.SimConfig(n_real=4, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_AUTO, n_samp=1, n_max=150, seed=22,
                          t_mode=t_mode, order=M.ORDER_DC)
    o = oracle.simulate(t, sc.mask, T, *lb, oc)
    g = M.mpr_simulate(dev(t), dev(sc.mask), dev(T), *lb, cfg)
    assert g.sweeps == o.k_star
    assert np.array_equal(host(g.state), o.state)
    assert np.array_equal(host(g.acc), o.acc)
    assert np.allclose(host(g.energy), o.energy, rtol=0, atol=1e-5)


def test_double_checkerboard_only_where_supported():
    sc = synth.random_small(20, 24, 0.5, seed=2)
    t, m = dev(sc.z_obs * 0 + 0.5), dev(sc.mask)
    T = dev(np.full((2, 2), 0.1, np.float32))
    cfg = M.SimConfig(n_real=2, stop_mode=M.STOP_FIXED, n_eq=1, order=M.ORDER_DC)
    state = torch.zeros((2, 20, 24), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MprError):
        M.mpr_sweep(state, m, T, 16, 16, cfg, 1, 2)
    with pytest.raises(M.MprError):
        M.mpr_simulate_batched([dict(t=t, mask=m, T_blocks=T, block=(16, 16), scene_id=0)], cfg, tile_h=0)
