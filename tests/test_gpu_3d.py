"""The 3D lattice on the GPU (the extension to three dimensions named in Sec. 4) against the oracle's 3D functions.

Bars as for the plane: block counts bit-exact, temperatures within one FP32 ulp, the matching curve within 1e-6 per
bond, chain states, accumulators and the stopping sweep equal (the accept/reject decision is exact in FP64 on both
sides), energies within 1e-5 per bond (the kernel sums FP32 bond terms in fixed point).  Shapes span several
8-column bands with a ragged last band, several 64-plane segments with a ragged last one, odd and even rows,
temperature blocks that straddle bands and segments, zero-temperature blocks, two groups of realizations with idle
lanes, and the degenerate grids (one site, one column along each axis).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import SimConfig as OCfg
from paper_2212_01317_amd import _lib as M

pytestmark = pytest.mark.gpu

E_TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _scene3(D, H, W, p, seed):
    rng = np.random.default_rng(seed)
    t = rng.random((D, H, W)).astype(np.float32)
    m = (rng.random((D, H, W)) >= p).astype(np.uint8)
    t[m == 0] = 0.0
    return t, m


def _temps3(D, H, W, lb, seed, zero=False):
    nb = (-(-D // lb[0]), -(-H // lb[1]), -(-W // lb[2]))
    T = np.random.default_rng(seed).uniform(0.02, 0.5, nb).astype(np.float32)
    if zero:
        T.ravel()[::3] = 0.0
    return T


def _gcfg(o: OCfg) -> M.SimConfig:
    return M.SimConfig(q=o.q, J=o.J, n_real=o.n_real, real_offset=o.real_offset, init_mode=o.init_mode,
                       stop_mode=o.stop_mode, n_eq=o.n_eq, n_samp=o.n_samp, n_fit=o.n_fit, n_f=o.n_f, n_max=o.n_max,
                       seed=o.seed, scene_id=o.scene)


@pytest.fixture(scope="module")
def curve3():
    T = np.geomspace(1e-3, 1e2, 25).astype(np.float32)
    e = oracle.reference_curve3(T, L=8, n_therm=60, n_meas=80, seed=5)
    return T.astype(np.float64), e


@pytest.mark.parametrize("D,H,W,lb", [(9, 13, 17, (4, 5, 6)), (70, 6, 11, (64, 6, 11)), (5, 4, 3, (1, 1, 1))])
def test_calibrate3d_parity(curve3, D, H, W, lb):
    cT, ce = curve3
    t, m = _scene3(D, H, W, 0.4, D * H + W)
    To, So, No = oracle.calibrate_temperature3(t, m, *lb, cT, ce)
    Tg, eg, ng = M.mpr_calibrate_temperature3d(dev(t), dev(m), *lb, dev(cT), dev(ce))
    assert np.array_equal(host(ng), No)
    a, b = host(Tg).ravel(), np.asarray(To, np.float32).ravel()
    d = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
    assert np.all(d <= 1) and np.mean(d == 0) >= 0.99


def test_calibrate3d_without_bonds_fails(curve3):
    cT, ce = curve3
    m = np.zeros((4, 4, 4), np.uint8)
    m[::2, ::2, ::2] = 1
    t = np.random.default_rng(0).random((4, 4, 4)).astype(np.float32)
    with pytest.raises(M.MprError) as e:
        M.mpr_calibrate_temperature3d(dev(t), dev(m), 2, 2, 2, dev(cT), dev(ce))
    assert e.value.status == 4


def test_reference_curve3d_parity():
    Tg = np.array([0.003, 0.05, 0.4, 3.0, 60.0], np.float32)
    eo = oracle.reference_curve3(Tg, L=8, n_therm=15, n_meas=20, seed=31)
    eg = host(M.mpr_reference_curve3d(dev(Tg), L=8, n_therm=15, n_meas=20, seed=31))
    print("ref curve 3d", eo, eg, flush=True)
    assert np.max(np.abs(eg - eo)) <= 1e-6


@pytest.mark.parametrize("D,H,W,lb,R,p,zero,init", [
    (70, 9, 19, (16, 4, 6), 70, 0.6, False, 1),    # two plane segments (the last ragged), ragged band, 58 idle lanes
    (12, 10, 16, (5, 5, 8), 64, 0.5, True, 0),     # zero-temperature blocks, random start, blocks on the bands
    (8, 7, 9, (3, 3, 3), 20, 0.7, False, 1),       # odd sides, small blocks across bands and rows
    (1, 13, 21, (1, 4, 5), 64, 0.5, False, 1),     # one plane
    (9, 1, 1, (2, 1, 1), 64, 0.5, False, 0),       # one column along z
    (1, 1, 9, (1, 1, 4), 64, 0.5, False, 0),       # one row along x
    (2, 2, 2, (2, 2, 2), 64, 0.5, False, 0),
    (6, 11, 13, (2, 3, 1), 64, 0.5, False, 1),     # one-column blocks (every column its own temperature)
])
def test_simulate3d_fixed_matches_oracle(D, H, W, lb, R, p, zero, init):
    t, m = _scene3(D, H, W, p, seed=D * 100 + H * 10 + W)
    T = _temps3(D, H, W, lb, seed=D + H + W, zero=zero)
    oc = OCfg(n_real=R, init_mode=init, stop_mode=0, n_eq=5, n_samp=2, seed=17, scene=3)
    print(f"[3d] fixed D={D} H={H} W={W} lb={lb} R={R}", flush=True)
    o = oracle.simulate3(t, m, T, *lb, oc, parallel=True)
    g = M.mpr_simulate3d(dev(t), dev(m), dev(T), *lb, _gcfg(oc))
    assert g.sweeps == o.k_star
    gs = host(g.state)
    print("state agreement", float(np.mean(gs == o.state)), flush=True)
    assert np.array_equal(gs, o.state)
    assert np.array_equal(host(g.acc), o.acc)
    assert np.allclose(host(g.energy), o.energy, rtol=0, atol=E_TOL)


def test_simulate3d_single_site():
    t = np.zeros((1, 1, 1), np.float32)
    m = np.zeros((1, 1, 1), np.uint8)
    T = np.full((1, 1, 1), 0.3, np.float32)
    oc = OCfg(n_real=64, init_mode=0, stop_mode=0, n_eq=3, n_samp=1, seed=2)
    o = oracle.simulate3(t, m, T, 1, 1, 1, oc)
    g = M.mpr_simulate3d(dev(t), dev(m), dev(T), 1, 1, 1, _gcfg(oc))
    assert np.array_equal(host(g.state), o.state)
    assert np.array_equal(host(g.acc), o.acc)


def test_simulate3d_auto_matches_oracle():
    D, H, W, lb = (20, 12, 18, (10, 6, 9))
    t, m = _scene3(D, H, W, 0.55, seed=77)
    T = _temps3(D, H, W, lb, seed=4)
    oc = OCfg(n_real=64, init_mode=1, stop_mode=1, n_fit=6, n_f=3, n_max=60, n_samp=3, seed=8)
    o = oracle.simulate3(t, m, T, *lb, oc, parallel=True)
    g = M.mpr_simulate3d(dev(t), dev(m), dev(T), *lb, _gcfg(oc))
    print("k*", o.k_star, g.sweeps, o.converged, g.converged, flush=True)
    assert g.sweeps == o.k_star and g.converged == o.converged
    assert np.array_equal(host(g.state), o.state)
    assert np.array_equal(host(g.acc), o.acc)
    assert np.allclose(host(g.energy), o.energy, rtol=0, atol=E_TOL)


def test_one_plane_equals_the_plane_path():
    """D = 1 is the plane model: the 3D GPU path equals the plane's GPU path bit for bit."""
    H, W, lb = 33, 45, (8, 9)
    t, m = _scene3(1, H, W, 0.5, seed=3)
    T = np.random.default_rng(1).uniform(0.05, 0.4, (-(-H // lb[0]), -(-W // lb[1]))).astype(np.float32)
    cfg = M.SimConfig(n_real=64, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=7, n_samp=2, seed=9,
                      sweep_kernel=M.SWEEP_LANES)
    g3 = M.mpr_simulate3d(dev(t), dev(m), dev(T.reshape(1, *T.shape)), 1, *lb, cfg)
    g2 = M.mpr_simulate(dev(t[0]), dev(m[0]), dev(T), *lb, cfg)
    assert np.array_equal(host(g3.state)[:, 0], host(g2.state))
    assert np.array_equal(host(g3.acc)[0], host(g2.acc))
    assert np.allclose(host(g3.energy), host(g2.energy), rtol=0, atol=E_TOL)


def test_simulate3d_deterministic_and_errors():
    D, H, W, lb = (6, 8, 10, (3, 4, 5))
    t, m = _scene3(D, H, W, 0.5, seed=12)
    T = _temps3(D, H, W, lb, seed=6)
    cfg = M.SimConfig(n_real=64, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=4, n_samp=1, seed=1)
    a = M.mpr_simulate3d(dev(t), dev(m), dev(T), *lb, cfg)
    b = M.mpr_simulate3d(dev(t), dev(m), dev(T), *lb, cfg)
    assert np.array_equal(host(a.state), host(b.state)) and np.array_equal(host(a.acc), host(b.acc))
    for bad in (dict(t_mode=M.T_SITE), dict(order=M.ORDER_DC), dict(coupling=M.COUPLING_DIRECTIONAL)):
        c = M.SimConfig(n_real=64, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=4, n_samp=1, seed=1,
                        **bad)
        with pytest.raises(M.MprError) as e:
            M.mpr_simulate3d(dev(t), dev(m), dev(T), *lb, c)
        assert e.value.status == 1
    with pytest.raises(ValueError):
        M.mpr_simulate3d(dev(t), dev(m), dev(T[:1]), *lb, cfg)


def test_fullsize_3d_sampled_realizations():
    """The 3D leg as the benchmark runs it (256^3 stand-in, p = 0.6, 32^3 blocks, R = 256 on the GPU): realizations 0
    and 255, recomputed one by one by the oracle (the stream is keyed by the global realization index), have the same
    chains after 3 sweeps and one sampling sweep, and e(0) of the block-mean start is the same."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2212_01317_amd import synth
    L, R, lb, n_eq = 256, 256, (32, 32, 32), 3
    f, m = synth.config3d(L, 0.6)
    z = dev(f * m)
    md = dev(m)
    t2, _ = M.mpr_map_angles(z.view(L * L, L), md.view(L * L, L))
    t = t2.view(L, L, L)
    T = np.random.default_rng(3).uniform(0.03, 0.3, (L // 32,) * 3).astype(np.float32)
    seed = synth.seed_for(7, synth.ROLE_PHILOX)
    cfg = M.SimConfig(n_real=R, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=n_eq, n_samp=1, seed=seed)
    g = M.mpr_simulate3d(t, md, dev(T), *lb, cfg)
    torch.cuda.synchronize()
    t_h = host(t)
    e0 = float(host(g.energy)[0])
    picks = (0, R - 1)
    gs = {r: host(g.state[r]) for r in picks}
    del g
    torch.cuda.empty_cache()

    def one(r):
        return oracle.simulate3(t_h, m, T, *lb, OCfg(n_real=1, real_offset=r, init_mode=1, stop_mode=0, n_eq=n_eq,
                                                     n_samp=1, seed=seed))

    with ThreadPoolExecutor(2) as ex:
        outs = list(ex.map(one, picks))
    for r, o in zip(picks, outs):
        frac = float(np.mean(gs[r] == o.state[0]))
        print(f"3D realization {r}: state agreement {frac:.7f}", flush=True)
        assert frac >= 0.9999
        assert abs(e0 - o.energy[0]) <= 1e-5


def test_predict3d_matches_the_oracle_pipeline():
    """predict3d (map, 3D calibration, simulation, conditional mean) against the oracle's steps on the same inputs:
    temperatures equal or one ulp apart, and, on the GPU's temperatures, the same stopping sweep and prediction bit
    for bit."""
    import paper_2212_01317_amd as P
    D, H, W, lb = 10, 12, 14, (5, 6, 7)
    rng = np.random.default_rng(31)
    z = (rng.standard_normal((D, H, W)) * 3 + 10).astype(np.float32)
    m = (rng.random((D, H, W)) >= 0.5).astype(np.uint8)
    zi = z.copy()
    zi[m == 0] = np.nan
    Tc = np.geomspace(1e-3, 1e2, 21).astype(np.float32)
    ec = oracle.reference_curve3(Tc, L=8, n_therm=30, n_meas=40, seed=3)
    cT, ce = Tc.astype(np.float64), ec
    pr = P.predict3d(dev(zi), dev(m), block=lb, n_real=64, stop_mode=M.STOP_AUTO, n_fit=6, n_f=3, n_max=60, n_samp=2,
                     seed=11, curve=(dev(cT), dev(ce)))
    t2, rg = oracle.map_angles(zi.reshape(D * H, W), m.reshape(D * H, W))
    t = t2.reshape(D, H, W)
    To, _, _ = oracle.calibrate_temperature3(t, m, *lb, cT, ce)
    Tg = host(pr.T)
    d = np.abs(Tg.ravel().view(np.int32).astype(np.int64) - np.asarray(To, np.float32).ravel().view(np.int32))
    assert np.all(d <= 1)                       # the block sums are FP64 in another order: equal or one ulp apart
    o = oracle.simulate3(t, m, Tg, *lb, OCfg(n_real=64, init_mode=1, stop_mode=1, n_fit=6, n_f=3, n_max=60,
                                                 n_samp=2, seed=11))
    assert pr.sim.sweeps == o.k_star
    zo = oracle.predict(o.acc.reshape(D * H, W), zi.reshape(D * H, W), m.reshape(D * H, W), 128, rg)
    assert np.array_equal(host(pr.zhat).reshape(D * H, W), zo)
