"""Pins of the oracle's temperature-gradient functions (block energies H_b and the score-function estimator)."""
import math

import numpy as np
import pytest
from scipy import integrate


def test_block_energy_hand_values(orc):
    # 1 x 3, middle gap: both bonds touch the gap and the samples -> full weight
    t = np.array([[0.0, 0.25, 0.75]], np.float32)
    m = np.array([[1, 0, 1]], np.uint8)
    Hb = orc.block_energy(t, m, 1, 3)
    assert Hb.shape == (1,)
    assert abs(Hb[0] - (-math.cos(math.pi * 0.25) - math.cos(math.pi * 0.5))) < 1e-15
    # 1 x 2, two gaps in different blocks: the bond counts one half in each
    t2 = np.array([[0.1, 0.6]], np.float32)
    m2 = np.zeros((1, 2), np.uint8)
    Hb2 = orc.block_energy(t2, m2, 1, 1)
    e = -math.cos(math.pi * (np.float64(np.float32(0.1)) - np.float64(np.float32(0.6))))
    assert np.allclose(Hb2, [0.5 * e, 0.5 * e], atol=1e-15)
    # same two gaps in one block: the bond counts once in full
    assert abs(orc.block_energy(t2, m2, 1, 2)[0] - e) < 1e-15
    # samples only: no state-dependent bond
    assert np.all(orc.block_energy(t2, np.ones((1, 2), np.uint8), 1, 1) == 0)


def test_block_energy_brute_force(orc):
    rng = np.random.default_rng(7)
    H, W, lb_h, lb_w = 11, 9, 4, 3
    t = rng.random((H, W)).astype(np.float32)
    m = (rng.random((H, W)) < 0.5).astype(np.uint8)
    Hb = orc.block_energy(t, m, lb_h, lb_w)
    nbx = -(-W // lb_w)
    ref = np.zeros_like(Hb)
    # every bond once: attribute to the block(s) of its gap end(s)
    for y in range(H):
        for x in range(W):
            for (yy, xx) in ((y, x + 1), (y + 1, x)):
                if yy >= H or xx >= W:
                    continue
                e = -math.cos(math.pi * (float(t[y, x]) - float(t[yy, xx])))
                gaps = [(a, b) for (a, b) in ((y, x), (yy, xx)) if not m[a, b]]
                for (a, b) in gaps:
                    ref[(a // lb_h) * nbx + b // lb_w] += e / len(gaps)
    assert np.allclose(Hb, ref, atol=1e-12)


def test_gradient_estimator_single_gap_exact(orc):
    """3 x 3 with one gap and one block: the conditional law of the gap is exactly exp(-H/T) / Z, so the
    derivative of its mean with respect to T (central difference of quadratures) pins the estimator."""
    from oracle import SimConfig
    T0 = 0.3
    g3 = np.array([[0.2, 0.85, 0.4], [0.8, 0.0, 0.9], [0.3, 0.95, 0.5]], np.float32)
    m = np.ones((3, 3), np.uint8)
    m[1, 1] = 0
    nbr = [float(np.float32(v)) for v in (0.85, 0.8, 0.9, 0.95)]

    def mean_t(T):
        f = lambda x: math.exp(sum(math.cos(math.pi * (x - v)) for v in nbr) / T)
        Z = integrate.quad(f, 0, 1, epsabs=1e-13, epsrel=1e-13)[0]
        return integrate.quad(lambda x: x * f(x), 0, 1, epsabs=1e-13, epsrel=1e-13)[0] / Z

    h = 1e-4
    exact = (mean_t(T0 + h) - mean_t(T0 - h)) / (2 * h)
    R = 60000
    res = orc.simulate(g3, m, np.array([T0], np.float32), 3, 3,
                       SimConfig(n_real=R, init_mode=0, stop_mode=0, n_eq=60, n_samp=0, seed=31))
    Hrb = np.stack([orc.block_energy(res.state[r], m, 3, 3) for r in range(R)])
    w = np.zeros((3, 3))
    w[1, 1] = 1.0
    est = orc.temperature_grad(res.state, Hrb, w, np.array([T0], np.float32))[0]
    t = res.state[:, 1, 1].astype(np.float64)
    Hc = Hrb[:, 0] - Hrb[:, 0].mean()
    se = np.std((t - t.mean()) * Hc) / math.sqrt(R) / T0 ** 2
    print(f"exact {exact:.6f} estimate {est:.6f} se {se:.6f}")
    assert abs(est - exact) < 4 * se
    assert abs(exact) > 10 * se           # the pin is informative


def test_gradient_estimator_is_covariance(orc):
    """With R = 2 the estimator is (g_0 - g_1)(H_0 - H_1) / 2 / T^2 exactly."""
    rng = np.random.default_rng(1)
    st = rng.random((2, 4, 5)).astype(np.float32)
    Hrb = rng.standard_normal((2, 3))
    w = rng.standard_normal((4, 5))
    T = np.array([0.5, 0.0, 2.0], np.float32)
    d = orc.temperature_grad(st, Hrb, w, T)
    g = [float(np.sum(w * st[r].astype(np.float64))) for r in range(2)]
    for b in range(3):
        exp = 0.0 if T[b] == 0 else (g[0] - g[1]) * (Hrb[0, b] - Hrb[1, b]) / 2 / float(T[b]) ** 2
        assert d[b] == pytest.approx(exp, rel=1e-12, abs=1e-15)
