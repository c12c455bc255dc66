"""Pins of the oracle's SST (Sec. 2.2.3, site-specific temperatures) and double-checkerboard order (Sec. 2.2.2):
the smoothing against hand-computed values and an independent library box filter, the per-site simulation against
the block simulation when the per-site map is the block map, and the double-checkerboard sweep against the single
checkerboard in the two layouts where they visit the sites in the same order."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import SimConfig
from paper_2212_01317_amd import synth


def _box_mean(a, r):
    # independent: scipy's box sum of the zero-padded map divided by the box sum of the in-grid indicator
    k = 2 * r + 1
    s = ndimage.uniform_filter(a, size=k, mode="constant", cval=0.0) * k * k
    c = ndimage.uniform_filter(np.ones_like(a), size=k, mode="constant", cval=0.0) * k * k
    return s / np.rint(c)


def test_zero_passes_is_the_block_map():
    T = np.array([[0.1, 0.2, 0.3], [0.4, 0.5, 0.6]], np.float32)
    Ts = oracle.sst_temperatures(T, 7, 11, 4, 4, r_s=1, n_s=0)
    expect = np.repeat(np.repeat(T, 4, axis=0), 4, axis=1)[:7, :11]
    assert np.array_equal(Ts, expect)


def test_constant_map_is_invariant():
    T = np.full((3, 3), 0.375, np.float32)
    Ts = oracle.sst_temperatures(T, 20, 17, 8, 6, r_s=2, n_s=5)
    assert np.all(Ts == np.float32(0.375))


def test_hand_computed_row():
    # one row, 1 x 1 blocks, T = (0, 0, 3), radius 1, one pass: (0, 0) -> 0, (0, 0, 3) -> 1, (0, 3) -> 1.5
    Ts = oracle.sst_temperatures(np.array([[0.0, 0.0, 3.0]], np.float32), 1, 3, 1, 1, r_s=1, n_s=1)
    assert np.array_equal(Ts, np.array([[0.0, 1.0, 1.5]], np.float32))
    # two passes: (0, 1) -> 0.5, (0, 1, 1.5) -> 2.5 / 3, (1, 1.5) -> 1.25
    Ts = oracle.sst_temperatures(np.array([[0.0, 0.0, 3.0]], np.float32), 1, 3, 1, 1, r_s=1, n_s=2)
    assert np.allclose(Ts, np.array([[0.5, 2.5 / 3.0, 1.25]]), rtol=1e-7)


@pytest.mark.parametrize("r_s,n_s", [(1, 1), (1, 5), (2, 3)])
def test_matches_library_box_filter(r_s, n_s):
    rng = np.random.default_rng(4)
    H, W, lb = 37, 53, (8, 8)
    T = rng.uniform(0.01, 0.5, ((H + 7) // 8, (W + 7) // 8)).astype(np.float32)
    a = np.repeat(np.repeat(T.astype(np.float64), 8, axis=0), 8, axis=1)[:H, :W]
    for _ in range(n_s):
        a = _box_mean(a, r_s)
    Ts = oracle.sst_temperatures(T, H, W, *lb, r_s=r_s, n_s=n_s)
    assert np.allclose(Ts, a, rtol=2e-7, atol=0.0)
    assert np.mean(Ts == a.astype(np.float32)) > 0.99


def test_per_site_simulation_of_the_block_map_is_the_block_simulation():
    sc = synth.random_small(40, 56, 0.5, seed=23)
    lb = (16, 16)
    t, _ = oracle.map_angles(sc.z_obs, sc.mask)
    T = np.random.default_rng(6).uniform(0.02, 0.4, (3, 4)).astype(np.float32)
    cfg = SimConfig(n_real=3, init_mode=1, stop_mode=0, n_eq=12, n_samp=2, seed=9)
    blk = oracle.simulate(t, sc.mask, T, *lb, cfg)
    Ts = oracle.sst_temperatures(T, 40, 56, *lb, r_s=1, n_s=0)
    site = oracle.simulate(t, sc.mask, Ts, *lb, SimConfig(**{**cfg.__dict__, "t_mode": 1}))
    assert np.array_equal(site.state, blk.state)
    assert np.array_equal(site.acc, blk.acc)
    # and a smoothed map changes the chains (the per-site values are used)
    Ts5 = oracle.sst_temperatures(T, 40, 56, *lb, r_s=1, n_s=5)
    sm = oracle.simulate(t, sc.mask, Ts5, *lb, SimConfig(**{**cfg.__dict__, "t_mode": 1}))
    assert not np.array_equal(sm.state, blk.state)


def _dc_case(lb, seed=5):
    sc = synth.random_small(30, 42, 0.5, seed=seed)
    t, _ = oracle.map_angles(sc.z_obs, sc.mask)
    nb = ((30 + lb[0] - 1) // lb[0], (42 + lb[1] - 1) // lb[1])
    T = np.random.default_rng(8).uniform(0.02, 0.4, nb).astype(np.float32)
    return sc, t, T


@pytest.mark.parametrize("lb", [(30, 42), (1, 1)])
def test_double_checkerboard_reduces_to_single(lb):
    """Sec. 2.2.2 orders: with one block covering the grid, or with 1 x 1 blocks (block parity = site colour), the
    double-checkerboard sweep visits the sites in the single-checkerboard order: the chains are identical."""
    sc, t, T = _dc_case(lb)
    cfg = SimConfig(n_real=2, init_mode=1, stop_mode=0, n_eq=10, n_samp=1, seed=3)
    sc_run = oracle.simulate(t, sc.mask, T, *lb, cfg)
    dc_run = oracle.simulate(t, sc.mask, T, *lb, SimConfig(**{**cfg.__dict__, "order": 1}))
    assert np.array_equal(dc_run.state, sc_run.state)


def test_double_checkerboard_is_another_chain():
    sc, t, T = _dc_case((8, 8))
    cfg = SimConfig(n_real=2, init_mode=1, stop_mode=0, n_eq=10, n_samp=1, seed=3)
    a = oracle.simulate(t, sc.mask, T, 8, 8, cfg)
    b = oracle.simulate(t, sc.mask, T, 8, 8, SimConfig(**{**cfg.__dict__, "order": 1}))
    assert not np.array_equal(a.state, b.state)
    # observed sites untouched and every gap state a proposal value in [0, 1)
    obs = sc.mask == 1
    assert np.array_equal(b.state[:, obs], np.broadcast_to(t[obs], b.state[:, obs].shape))
    assert np.all((b.state[:, ~obs] >= 0) & (b.state[:, ~obs] < 1))


def test_double_checkerboard_zero_temperature_energy_never_increases():
    """At T = 0 every accepted update lowers (or keeps) the energy, in any visiting order."""
    sc, t, _ = _dc_case((8, 8), seed=9)
    T0 = np.zeros((4, 6), np.float32)
    e = [oracle.simulate(t, sc.mask, T0, 8, 8, SimConfig(n_real=1, init_mode=0, stop_mode=0, n_eq=k, n_samp=0,
                                                            seed=2, order=1)).energy[-1] for k in range(0, 6)]
    assert all(b <= a + 1e-12 for a, b in zip(e, e[1:]))
