"""Temperature gradient on the GPU: parity of H_b and of the score-function estimate with the oracle (same chains),
and agreement with central finite differences under common random numbers (the method's own check)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import SimConfig as OCfg
from paper_2212_01317_amd import _lib as M
from paper_2212_01317_amd import synth
from paper_2212_01317_amd.autograd import MPRFunction

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_block_energy_and_gradient_parity():
    sc = synth.random_small(48, 70, 0.5, seed=41)
    lb = (16, 16)
    t, rg = oracle.map_angles(sc.z_obs, sc.mask)
    B = 3 * 5
    T = np.random.default_rng(2).uniform(0.03, 0.4, B).astype(np.float32)
    R = 24
    oc = OCfg(n_real=R, init_mode=1, stop_mode=0, n_eq=20, n_samp=1, seed=8)
    o = oracle.simulate(t, sc.mask, T, lb[0], lb[1], oc)
    Ho = np.stack([oracle.block_energy(o.state[r], sc.mask, *lb) for r in range(R)])
    gz = np.random.default_rng(3).standard_normal(sc.mask.shape).astype(np.float32)
    w = np.where(sc.mask == 0, gz.astype(np.float64) * (rg[1] - rg[0]), 0.0)
    do = oracle.temperature_grad(o.state, Ho, w, T)

    T_map = dev(T.reshape(3, 5)).requires_grad_(True)
    cfg = M.SimConfig(n_real=R, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=20, n_samp=1, seed=8)
    zhat = MPRFunction.apply(T_map, dev(t), dev(sc.mask), dev(sc.z_obs), dev(rg), lb, cfg)
    (zhat * dev(gz)).sum().backward()
    g_state = M.mpr_simulate(dev(t), dev(sc.mask), dev(T), lb[0], lb[1], cfg).state
    assert np.array_equal(host(g_state), o.state)
    Hg = host(M.mpr_block_energy(g_state, dev(sc.mask), *lb))
    assert np.allclose(Hg, Ho, rtol=1e-12, atol=1e-12)
    d64 = host(M.mpr_temperature_grad(g_state, M.mpr_block_energy(g_state, dev(sc.mask), *lb), dev(gz),
                                      dev(sc.mask), dev(rg), dev(T)))
    assert np.allclose(d64, do, rtol=1e-9, atol=1e-12 * np.abs(do).max())
    # the autograd result is the same estimate in the dtype of T_map (float32 here)
    dg = host(T_map.grad).ravel()
    assert np.allclose(dg, do, rtol=1e-6, atol=1e-7 * np.abs(do).max())


def test_perturbed_temperature_pair_matches_oracle():
    """The +-1e-3 relative temperature pair of the finite-difference check, small size: both GPU runs equal the
    oracle's, and the loss difference is the oracle's."""
    sc = synth.config5(128, 128)
    t, rg = oracle.map_angles(sc.z_obs, sc.mask)
    T = np.full(16, 0.06, np.float32)
    R = 64
    counts = sc.eval_mask.astype(np.int64).reshape(4, 32, 4, 32).sum(axis=(1, 3)).ravel()
    b = int(np.argmax(counts))
    oc = OCfg(n_real=R, init_mode=1, stop_mode=0, n_eq=20, n_samp=1, seed=5)
    cfg = M.SimConfig(n_real=R, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=20, n_samp=1, seed=5)
    Lo, Lg = [], []
    for sgn in (1, -1):
        Tp = T.copy()
        Tp[b] = T[b] * (1 + sgn * 1e-3)
        o = oracle.simulate(t, sc.mask, Tp, 32, 32, oc)
        g = M.mpr_simulate(dev(t), dev(sc.mask), dev(Tp), 32, 32, cfg, want_energy=False)
        assert np.array_equal(host(g.state), o.state)
        assert np.array_equal(host(g.acc), o.acc)
        zo = oracle.predict(o.acc, sc.z_obs, sc.mask, R, rg)
        zg = host(M.mpr_predict(g.acc, dev(sc.z_obs), dev(sc.mask), R, dev(rg)))
        assert np.array_equal(zg, zo)
        Lo.append(np.abs(zo.astype(np.float64) - sc.z_true)[sc.eval_mask == 1].mean())
        Lg.append(float(_loss(dev(zg), dev(sc.z_true), dev(sc.eval_mask.astype(bool)))))
    print(f"oracle L+ - L- = {Lo[0] - Lo[1]:.3e}, gpu {Lg[0] - Lg[1]:.3e}")
    assert Lo[0] != Lo[1]
    assert abs((Lg[0] - Lg[1]) - (Lo[0] - Lo[1])) <= 1e-12


@pytest.fixture(scope="module")
def c5():
    sc = synth.config5()
    lb = sc.block
    z, m = dev(sc.z_obs), dev(sc.mask)
    t, rg = M.mpr_map_angles(z, m)
    import paper_2212_01317_amd as P
    cT, ce = P.reference_curve(0.5)
    T, _, _ = M.mpr_calibrate_temperature(t, m, lb[0], lb[1], cT, ce)
    return sc, lb, z, m, t, rg, T


def _loss(zhat, truth, ev):
    # FP64: a 1e-3 relative change of one block temperature moves the MAE by ~1e-7, below FP32 resolution
    return (zhat.double() - truth.double()).abs()[ev].mean()


def test_gradient_matches_central_differences_with_crn(c5):
    """Config 5 (512^2, 16 x 16 temperature map, R = 1024): d(validation MAE)/dT_b by the estimator against central
    differences with dT = 1e-3 T_b and the same random numbers, on the 8 blocks with the most held-out pixels."""
    sc, lb, z, m, t, rg, T = c5
    truth = dev(sc.z_true)
    ev = dev(sc.eval_mask.astype(bool))
    cfg = M.SimConfig(n_real=1024, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=60, n_samp=1,
                      seed=synth.seed_for(5, synth.ROLE_PHILOX))
    T_map = T.clone().requires_grad_(True)
    zhat = MPRFunction.apply(T_map, t, m, z, rg, lb, cfg)
    L0 = _loss(zhat, truth, ev)
    L0.backward()
    est = host(T_map.grad).ravel()
    counts = sc.eval_mask.astype(np.int64).reshape(16, 32, 16, 32).sum(axis=(1, 3)).ravel()
    blocks = np.argsort(-counts, kind="stable")[:8]
    fd = []
    Tf = host(T).ravel()
    for b in blocks:
        vals = []
        for sgn in (1, -1):
            Tp = Tf.copy()
            Tp[b] = Tf[b] * (1 + sgn * 1e-3)
            sim = M.mpr_simulate(t, m, dev(Tp.reshape(16, 16)), lb[0], lb[1], cfg, want_energy=False)
            zh = M.mpr_predict(sim.acc, z, m, cfg.n_real, rg)
            vals.append(float(_loss(zh, truth, ev)))
            if sgn == 1:
                st_plus, acc_plus, zh_plus = sim.state, sim.acc, zh
            else:
                print(f"block {b}: T = {Tf[b]:.5g}, differing states {int((st_plus != sim.state).sum())}, "
                      f"acc {int((acc_plus != sim.acc).sum())}, zhat {int((zh_plus != zh).sum())}, "
                      f"zhat at scored sites {int(((zh_plus != zh) & ev).sum())}, L+ - L- = {vals[0] - vals[1]:.3e}",
                      flush=True)
        fd.append((vals[0] - vals[1]) / (2e-3 * Tf[b]))
    fd = np.array(fd)
    e = est[blocks]
    cos = float(np.dot(e, fd) / (np.linalg.norm(e) * np.linalg.norm(fd)))
    ratio = float(np.linalg.norm(e) / np.linalg.norm(fd))
    print("estimator", e, "\nfinite differences", fd, f"\ncosine {cos:.3f} norm ratio {ratio:.3f}")
    assert cos > 0.8
    assert 0.5 < ratio < 2.0
