"""Pins of the oracle's three-dimensional lattice (the 3D extension named in Sec. 4; no GPU needed).

On one plane (D = 1) every 3D function must be the independently pinned 2D function, bit for bit; the third axis is
pinned by hand values and the bond count of the open cubic grid, the invariance of the energy under a permutation of
the axes, brute force on tiny grids, the exact conditional density of one gap with six, five, four and three
neighbours (numerical quadrature), the monotone energy at T = 0, and the exact low- and high-temperature limits of
the matching curve of the cubic lattice.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import SimConfig

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _limits():
    vals = {}
    with open(os.path.join(GOLDEN, "mpr_limits.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _scene3(D, H, W, p, seed):
    rng = np.random.default_rng(seed)
    t = rng.random((D, H, W)).astype(np.float32)
    m = (rng.random((D, H, W)) >= p).astype(np.uint8)
    t[m == 0] = 0.0
    return t, m


def test_site_uniforms3_on_plane_zero_are_the_plane_stream(orc):
    for (x, y) in [(0, 0), (5, 3), (6, 2), (11, 7)]:
        a = orc.site_uniforms3(123456789, 3, 0, 7, 42, 8, 13, x, y, 0)
        b = orc.site_uniforms(123456789, 3, 0, 7, 42, 13, x, y)
        assert np.array_equal(a, b)
    # on plane z the row index is z H + y and the colour (x + y + z) & 1: a site of plane 1 draws what the plane
    # stream gives at row H + y when H + y has the parity of y + 1
    H, W = 7, 10
    for (x, y) in [(0, 0), (3, 2), (4, 5)]:
        a = orc.site_uniforms3(99, 0, 0, 3, 5, H, W, x, y, 1)
        b = orc.site_uniforms(99, 0, 0, 3, 5, W, x, H + y)     # H odd: (x + H + y) & 1 == (x + y + 1) & 1
        assert np.array_equal(a, b)


def test_one_plane_is_the_plane_model(orc):
    """D = 1: block statistics, energy, sweeps and the whole simulation equal the 2D oracle bit for bit."""
    H, W = 13, 17
    t, m = _scene3(1, H, W, 0.45, 5)
    S3, N3, T3, O3 = orc.block_stats3(t, m, 1, 4, 5)
    S2, N2, T2, O2 = orc.block_stats(t[0], m[0], 4, 5)
    assert np.array_equal(N3, N2) and np.array_equal(O3, O2)
    assert np.array_equal(S3, S2) and np.array_equal(T3, T2)
    assert orc.energy3(t) == orc.energy(t[0])
    rng = np.random.default_rng(1)
    Tb = rng.uniform(0.05, 0.8, S2.size).astype(np.float32)
    s3, s2 = t.copy(), t[0].copy()
    for k in range(1, 6):
        orc.sweep3(s3, m, Tb, 1, 4, 5, k, seed=77, scene=2, real=9)
        orc.sweep(s2, m[0], Tb, 4, 5, k, seed=77, scene=2, real=9)
        assert np.array_equal(s3[0], s2)
    for stop in (0, 1):
        cfg = SimConfig(n_real=3, init_mode=1, stop_mode=stop, n_eq=12, n_samp=2, n_max=60, seed=31, scene=1)
        r3 = orc.simulate3(t, m, Tb, 1, 4, 5, cfg)
        r2 = orc.simulate(t[0], m[0], Tb, 4, 5, cfg)
        assert r3.k_star == r2.k_star
        assert np.array_equal(r3.state[:, 0], r2.state)
        assert np.array_equal(r3.acc[0], r2.acc)
        assert np.array_equal(r3.energy, r2.energy)


def test_energy3_hand_values_and_bond_count(orc):
    D, H, W = 3, 4, 5
    nb = (W - 1) * H * D + W * (H - 1) * D + W * H * (D - 1)
    assert orc.energy3(np.zeros((D, H, W), np.float32)) == -1.0
    z, y, x = np.indices((D, H, W))
    cb = ((x + y + z) & 1).astype(np.float32)          # neighbours 1 turn apart: cos(pi) = -1 on every bond
    assert orc.energy3(cb) == pytest.approx(1.0, abs=1e-15)
    # one interior site at 1/2 turn: its six bonds give -cos(pi/2) = 0, every other bond -1
    s = np.zeros((D, H, W), np.float32)
    s[1, 2, 2] = 0.5
    assert orc.energy3(s) == pytest.approx(-(nb - 6) / nb, abs=1e-15)
    # a corner site has three bonds
    s = np.zeros((D, H, W), np.float32)
    s[0, 0, 0] = 0.5
    assert orc.energy3(s) == pytest.approx(-(nb - 3) / nb, abs=1e-15)


def test_energy3_is_invariant_under_axis_permutations(orc):
    rng = np.random.default_rng(3)
    s = rng.random((4, 6, 5)).astype(np.float32)
    e = orc.energy3(s)
    for perm in [(2, 1, 0), (1, 0, 2), (0, 2, 1), (1, 2, 0)]:
        assert orc.energy3(np.ascontiguousarray(s.transpose(perm))) == pytest.approx(e, rel=1e-13)


def test_block_stats3_brute_force(orc):
    D, H, W = 5, 6, 7
    t, m = _scene3(D, H, W, 0.4, 11)
    lb = (2, 3, 4)
    S, N, Ts, No = orc.block_stats3(t, m, *lb)
    nbz, nby, nbx = -(-D // lb[0]), -(-H // lb[1]), -(-W // lb[2])
    S_ref = np.zeros(nbz * nby * nbx)
    N_ref = np.zeros(nbz * nby * nbx, int)
    Ts_ref = np.zeros(nbz * nby * nbx)
    No_ref = np.zeros(nbz * nby * nbx, int)
    for z in range(D):
        for y in range(H):
            for x in range(W):
                if not m[z, y, x]:
                    continue
                b = ((z // lb[0]) * nby + y // lb[1]) * nbx + x // lb[2]
                Ts_ref[b] += float(t[z, y, x])
                No_ref[b] += 1
                for dz, dy, dx in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
                    zz, yy, xx = z + dz, y + dy, x + dx
                    if zz < D and yy < H and xx < W and m[zz, yy, xx]:
                        S_ref[b] += -math.cos(math.pi * (float(t[z, y, x]) - float(t[zz, yy, xx])))
                        N_ref[b] += 1
    assert np.array_equal(N, N_ref) and np.array_equal(No, No_ref)
    assert np.allclose(S, S_ref, rtol=1e-13, atol=1e-13) and np.allclose(Ts, Ts_ref, rtol=1e-13)


def _one_gap_density(nbr, T):
    f = lambda t: math.exp((1.0 / T) * sum(math.cos(math.pi * (t - tj)) for tj in nbr))
    return f, integrate.quad(f, 0.0, 1.0, limit=200)[0]


@pytest.mark.parametrize("where", ["centre", "face", "edge", "corner"])
def test_single_gap3_histogram_matches_boltzmann(orc, where):
    T = 0.5
    rng = np.random.default_rng(17)
    g = rng.random((3, 3, 3)).astype(np.float32)
    pos = {"centre": (1, 1, 1), "face": (0, 1, 1), "edge": (0, 0, 1), "corner": (0, 0, 0)}[where]
    m = np.ones((3, 3, 3), np.uint8)
    m[pos] = 0
    z, y, x = pos
    nbr = [float(g[zz, yy, xx]) for (zz, yy, xx) in ((z - 1, y, x), (z, y - 1, x), (z, y, x - 1), (z, y, x + 1),
                                                    (z, y + 1, x), (z + 1, y, x))
           if 0 <= zz < 3 and 0 <= yy < 3 and 0 <= xx < 3]
    assert len(nbr) == {"centre": 6, "face": 5, "edge": 4, "corner": 3}[where]
    R = 20000
    cfg = SimConfig(n_real=R, init_mode=0, stop_mode=0, n_eq=40, n_samp=0, seed=4243)
    res = orc.simulate3(g, m, np.array([T], np.float32), 3, 3, 3, cfg)
    obs = m.astype(bool)
    assert np.all(res.state[:, obs] == g[obs])
    samp = res.state[:, z, y, x].astype(np.float64)
    f, Z = _one_gap_density(nbr, T)
    edges = np.linspace(0, 1, 41)
    probs = np.array([integrate.quad(f, a, b)[0] / Z for a, b in zip(edges[:-1], edges[1:])])
    cnt, _ = np.histogram(samp, edges)
    chi2 = np.sum((cnt - R * probs) ** 2 / (R * probs))
    assert stats.chi2.sf(chi2, len(probs) - 1) > 1e-4
    mean = integrate.quad(lambda t: t * f(t), 0, 1)[0] / Z
    assert abs(samp.mean() - mean) < 5 * samp.std() / math.sqrt(R)


def test_zero_temperature_energy3_non_increasing(orc):
    t, m = _scene3(6, 7, 8, 0.6, 21)
    rng = np.random.default_rng(2)
    s = t.copy()
    s[m == 0] = rng.random(int((m == 0).sum())).astype(np.float32)
    e_prev = orc.energy3(s)
    T0 = np.zeros(1, np.float32)
    for k in range(1, 15):
        orc.sweep3(s, m, T0, 6, 7, 8, k, seed=5)
        e = orc.energy3(s)
        assert e <= e_prev + 1e-12
        e_prev = e
    assert np.all(s[m == 1] == t[m == 1])


def test_reference_curve3_exact_limits(orc):
    lim = _limits()
    T = np.array([0.005, 0.02], np.float32)
    e = orc.reference_curve3(T, L=12, n_therm=200, n_meas=300, seed=13)
    for i in range(2):
        assert abs(e[i] - (-1.0 + lim["lowT_slope_3d"] * T[i])) < 0.02 * T[i] + 2e-5
    # the 2D slope 1/4 is ruled out
    assert abs(e[1] - (-1.0 + 0.25 * T[1])) > 0.5 * T[1] * (0.25 - 1.0 / 6.0)
    Th = np.array([100.0, 400.0], np.float32)
    eh = orc.reference_curve3(Th, L=16, n_therm=20, n_meas=400, seed=13)
    for i in range(2):
        assert abs(eh[i] - (lim["e_inf_q05"] - lim["c1_q05_3d"] / Th[i])) < 1e-3


def test_calibration3_recovers_temperature_on_complete_field(orc):
    """A fully observed cubic field from the unconditional model at T0 (all sites free, open grid) calibrates back
    to about T0 with the cubic matching curve and one block."""
    Tg = np.geomspace(1e-3, 1e2, 31).astype(np.float32)
    ce = orc.reference_curve3(Tg, L=10, n_therm=150, n_meas=150, seed=21)
    D = H = W = 14
    for T0 in (0.08, 0.4):
        free = np.zeros((D, H, W), np.uint8)
        cfg = SimConfig(n_real=1, init_mode=0, stop_mode=0, n_eq=300, n_samp=0, seed=7)
        s = orc.simulate3(np.zeros((D, H, W), np.float32), free, np.array([T0], np.float32), D, H, W, cfg).state[0]
        T, _, _ = orc.calibrate_temperature3(s, np.ones((D, H, W), np.uint8), D, H, W, Tg.astype(np.float64), ce)
        assert abs(T.ravel()[0] / T0 - 1.0) < 0.15


def test_simulate3_per_chain_stop_is_the_latest_chain(orc):
    """The per-chain test on the 3D grid: the scene stops at the latest of the chains' own sweeps (each chain run
    alone with the plain test), and a chain's state equals that chain run alone for as many sweeps."""
    t, m = _scene3(6, 7, 8, 0.5, 21)
    T = np.full((1, 1, 1), 0.1, np.float32)
    ks = [orc.simulate3(t, m, T, 6, 7, 8, SimConfig(n_real=1, real_offset=r, init_mode=0, stop_mode=1, n_fit=6,
                                                     n_f=2, n_max=200, n_samp=0, seed=2)).k_star for r in range(4)]
    both = orc.simulate3(t, m, T, 6, 7, 8, SimConfig(n_real=4, init_mode=0, stop_mode=2, n_fit=6, n_f=2, n_max=200,
                                                      n_samp=1, seed=2))
    assert len(set(ks)) > 1 and both.k_star == max(ks)
    for r in (0, 3):
        alone = orc.simulate3(t, m, T, 6, 7, 8, SimConfig(n_real=1, real_offset=r, init_mode=0, stop_mode=0,
                                                           n_eq=both.k_star, n_samp=1, seed=2))
        assert np.array_equal(alone.state[0], both.state[r])
