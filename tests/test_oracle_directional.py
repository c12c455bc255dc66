"""Pins of the oracle's directional-coupling extension (Sec. 4: exchange interactions distinguished by direction,
parameters kept local to blocks): each block has a temperature Tx for its horizontal bonds and Ty for its vertical
bonds.  Pinned against the exact conditional density of a single gap, against the isotropic chain when Tx = Ty,
by the decoupling of the rows when Ty is huge, and by the calibration's response to geometric anisotropy."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from oracle import SimConfig
from paper_2212_01317_amd import synth


def test_single_gap_histogram_matches_directional_boltzmann():
    """A centre gap in a 3 x 3 grid: the conditional density of its angle is proportional to
    exp(J/Tx (cos pi(t - t_l) + cos pi(t - t_r)) + J/Ty (cos pi(t - t_u) + cos pi(t - t_d))) (q = 1/2)."""
    Tx, Ty = 0.2, 0.7
    g = np.array([[0.2, 0.9, 0.4], [0.1, 0.0, 0.7], [0.3, 0.6, 0.5]], np.float32)
    m = np.ones((3, 3), np.uint8)
    m[1, 1] = 0
    R = 20000
    cfg = SimConfig(n_real=R, init_mode=0, stop_mode=0, n_eq=60, n_samp=0, seed=777, directional=1)
    res = oracle.simulate(g, m, np.array([Tx, Ty], np.float32), 3, 3, cfg)
    samp = res.state[:, 1, 1].astype(np.float64)
    assert np.all(res.state[:, m.astype(bool)] == g[m.astype(bool)])
    c = lambda d: math.cos(math.pi * d)
    f = lambda t: math.exp((c(t - 0.1) + c(t - 0.7)) / Tx + (c(t - 0.9) + c(t - 0.6)) / Ty)
    Z = integrate.quad(f, 0, 1, limit=200)[0]
    edges = np.linspace(0, 1, 41)
    probs = np.array([integrate.quad(f, a, b)[0] / Z for a, b in zip(edges[:-1], edges[1:])])
    cnt, _ = np.histogram(samp, edges)
    chi2 = np.sum((cnt - R * probs) ** 2 / (R * probs))
    assert stats.chi2.sf(chi2, len(probs) - 1) > 1e-4
    mean = integrate.quad(lambda t: t * f(t), 0, 1, limit=200)[0] / Z
    assert abs(samp.mean() - mean) < 5 * samp.std() / math.sqrt(R)
    # the isotropic density at either temperature is rejected
    for T in (Tx, Ty):
        fi = lambda t, T=T: math.exp((c(t - 0.1) + c(t - 0.7) + c(t - 0.9) + c(t - 0.6)) / T)
        Zi = integrate.quad(fi, 0, 1, limit=200)[0]
        pi = np.array([integrate.quad(fi, a, b)[0] / Zi for a, b in zip(edges[:-1], edges[1:])])
        assert stats.chi2.sf(np.sum((cnt - R * pi) ** 2 / (R * pi)), len(pi) - 1) < 1e-6


def _case(H=20, W=26, lb=(8, 8), seed=5):
    sc = synth.random_small(H, W, 0.55, seed=seed)
    t, _ = oracle.map_angles(sc.z_obs, sc.mask)
    nb = ((H + lb[0] - 1) // lb[0], (W + lb[1] - 1) // lb[1])
    T = np.random.default_rng(seed).uniform(0.05, 0.5, nb).astype(np.float32)
    return sc, t, T


def test_equal_temperatures_give_the_isotropic_chain():
    sc, t, T = _case()
    cfg = SimConfig(n_real=3, init_mode=1, stop_mode=0, n_eq=12, n_samp=2, seed=9)
    iso = oracle.simulate(t, sc.mask, T, 8, 8, cfg)
    dirc = oracle.simulate(t, sc.mask, np.concatenate([T.ravel(), T.ravel()]), 8, 8,
                           SimConfig(**{**cfg.__dict__, "directional": 1}))
    assert np.array_equal(dirc.state, iso.state)
    assert np.array_equal(dirc.acc, iso.acc)


def test_rows_decouple_when_the_vertical_temperature_is_huge():
    """Ty = 1e30: the vertical terms of the Boltzmann exponent vanish, so a row's chain cannot depend on the other
    rows; with Ty = Tx it does."""
    sc, t, T = _case(seed=11)
    H, W = t.shape
    r0 = 9
    other = t.copy()
    rng = np.random.default_rng(3)
    rows = [y for y in range(H) if y != r0]
    other[rows] = rng.uniform(0, 1, (len(rows), W)).astype(np.float32)
    mask2 = sc.mask.copy()
    mask2[rows] = rng.integers(0, 2, (len(rows), W)).astype(np.uint8)
    cfg = SimConfig(n_real=2, init_mode=0, stop_mode=0, n_eq=10, n_samp=0, seed=21, directional=1)
    huge = np.concatenate([T.ravel(), np.full(T.size, 1e30, np.float32)])
    a = oracle.simulate(t, sc.mask, huge, 8, 8, cfg)
    b = oracle.simulate(other, mask2, huge, 8, 8, cfg)
    assert np.array_equal(a.state[:, r0], b.state[:, r0])
    same = np.concatenate([T.ravel(), T.ravel()])
    c = oracle.simulate(t, sc.mask, same, 8, 8, cfg)
    d = oracle.simulate(other, mask2, same, 8, 8, cfg)
    assert not np.array_equal(c.state[:, r0], d.state[:, r0])


@pytest.fixture(scope="module")
def curve():
    cT = np.logspace(-3, 1, 17).astype(np.float32)
    ce = oracle.reference_curve(cT, L=16, n_therm=60, n_meas=60, seed=5)
    return cT.astype(np.float64), ce


def test_directional_calibration_follows_the_anisotropy(curve):
    """A field correlated along x (xi_x = 12) and rough along y (xi_y = 1.5) has smoother horizontal sample bonds:
    Tx < Ty in almost every block; an isotropic field gives no systematic difference."""
    cT, ce = curve
    H = W = 128
    lb = (16, 16)
    aniso = synth.grf_aniso(H, W, 12.0, 1.5, np.random.default_rng(1))
    iso = synth.grf(H, W, 4.0, np.random.default_rng(2))
    mask = synth.uniform_mask(H, W, int(0.3 * H * W), np.random.default_rng(3))
    for field, expect in ((aniso, "x"), (iso, None)):
        t, _ = oracle.map_angles(field.astype(np.float32), mask)
        Tx, Ty = oracle.calibrate_directional(t, mask, *lb, cT, ce)
        assert np.all(Tx >= np.float32(1e-3)) and np.all(Ty >= np.float32(1e-3))
        r = np.log(Tx / Ty)
        if expect == "x":
            assert np.mean(Tx < Ty) >= 0.95
        else:
            assert abs(np.mean(r)) < 0.15
    # each direction alone is the isotropic calibration of that direction's bonds
    t, _ = oracle.map_angles(aniso.astype(np.float32), mask)
    Sh, Nh, Sv, Nv = oracle.block_stats_directional(t, mask, *lb)
    S, N, _, _ = oracle.block_stats(t, mask, *lb)
    assert np.array_equal(Nh + Nv, N)
    assert np.allclose(Sh + Sv, S, rtol=1e-12, atol=1e-12)


def test_temperatures_below_the_floor_run_the_floor_chain():
    """Reading of the directional extension (the paper gives no parameters for it): both direction temperatures are
    raised to at least fl32(1e-3 J), so that J a_h / Tx + J a_v / Ty stays finite.  A temperature below the floor
    (0, a denormal, 1e-5 J) gives exactly the chain of the floor value, for either direction and for J != 1; a value
    above the floor gives another chain."""
    sc, t, T = _case(seed=13)
    nb = T.size
    for J in (1.0, 2.0):
        floor = np.float32(1e-3 * J)
        cfg = SimConfig(n_real=2, init_mode=0, stop_mode=0, n_eq=8, n_samp=1, seed=31, directional=1, J=J)
        Ty = np.full(nb, 0.2, np.float32)
        at_floor = oracle.simulate(t, sc.mask, np.concatenate([np.full(nb, floor, np.float32), Ty]), 8, 8, cfg)
        for below in (0.0, 1e-40, 1e-5 * J, float(np.nextafter(floor, np.float32(0)))):
            low = oracle.simulate(t, sc.mask, np.concatenate([np.full(nb, below, np.float32), Ty]), 8, 8, cfg)
            assert np.array_equal(low.state, at_floor.state), (J, below)
            assert np.array_equal(low.acc, at_floor.acc)
        # the floor acts on Ty the same way
        a = oracle.simulate(t, sc.mask, np.concatenate([Ty, np.zeros(nb, np.float32)]), 8, 8, cfg)
        b = oracle.simulate(t, sc.mask, np.concatenate([Ty, np.full(nb, floor, np.float32)]), 8, 8, cfg)
        assert np.array_equal(a.state, b.state)
        above = oracle.simulate(t, sc.mask, np.concatenate([np.full(nb, 0.05 * J, np.float32), Ty]), 8, 8, cfg)
        assert not np.array_equal(above.state, at_floor.state)
