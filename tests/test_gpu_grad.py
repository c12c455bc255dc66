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
    lb = (32, 32)
    z, m = dev(sc.z_obs), dev(sc.mask)
    t, rg = M.mpr_map_angles(z, m)
    import paper_2212_01317_amd as P
    cT, ce = P.reference_curve(0.5)
    T, _, _ = M.mpr_calibrate_temperature(t, m, lb[0], lb[1], cT, ce)
    return sc, lb, z, m, t, rg, T


def _loss(zhat, truth, ev):
    # FP64: a 1e-3 relative change of one block temperature moves the MAE by ~1e-7, below FP32 resolution
    return (zhat.double() - truth.double()).abs()[ev].mean()


def _cfg(seed, R=1024):
    return M.SimConfig(n_real=R, init_mode=M.INIT_BLOCK_MEAN, stop_mode=M.STOP_FIXED, n_eq=60, n_samp=1, seed=seed)


def _fd_and_estimate(t, m, z, rg, T_host, blocks, losses, seeds, rel=1e-3):
    """Per seed: the estimator dL_b/dT_b (autograd, one forward) and the central difference with common random
    numbers (dT = rel * T_b, same seed for both sides), for the loss losses[b](zhat) of each block b."""
    nb = len(blocks)
    est = np.zeros((len(seeds), nb))
    fd = np.zeros((len(seeds), nb))
    shape = T_host.shape
    for i, seed in enumerate(seeds):
        cfg = _cfg(seed)
        T_map = dev(T_host).requires_grad_(True)
        zhat = MPRFunction.apply(T_map, t, m, z, rg, (32, 32), cfg)
        for j, b in enumerate(blocks):
            (g,) = torch.autograd.grad(losses[b](zhat), T_map, retain_graph=j + 1 < nb)
            est[i, j] = float(g.double().ravel()[b])
            vals = []
            for sgn in (1, -1):
                Tp = T_host.copy().ravel()
                Tp[b] = T_host.ravel()[b] * (1 + sgn * rel)
                sim = M.mpr_simulate(t, m, dev(Tp.reshape(shape)), 32, 32, cfg, want_energy=False)
                vals.append(float(losses[b](M.mpr_predict(sim.acc, z, m, cfg.n_real, rg))))
            fd[i, j] = (vals[0] - vals[1]) / (2 * rel * T_host.ravel()[b])
    return est, fd


def _summary(est, fd):
    n = est.shape[0]
    me, mf = est.mean(0), fd.mean(0)
    se_e, se_f = est.std(0, ddof=1) / np.sqrt(n), fd.std(0, ddof=1) / np.sqrt(n)
    z = (me - mf) / np.sqrt(se_e ** 2 + se_f ** 2)
    print("estimator ", np.array2string(me, precision=4), "\n  +-       ", np.array2string(se_e, precision=4),
          "\nfinite diff", np.array2string(mf, precision=4), "\n  +-       ", np.array2string(se_f, precision=4),
          "\nz          ", np.array2string(z, precision=2), flush=True)
    return me, mf, se_e, se_f, z


def test_gradient_matches_central_differences_with_crn(c5):
    """The method's check, where the derivative is measurable.  Config 5 field (512^2, 16 x 16 blocks of 32^2,
    R = 1024, 60 sweeps + 1 sample) at block temperatures U[0.3, 1.2]: there the conditional mean of a gap site moves
    with T (the pull towards mid-range grows), so a loss confined to block b, L_b = mean over its gap sites of
    c_v zhat_v with c_v = sign(1/2 - tbar_v), has a clearly positive dL_b/dT_b.  On the six partially gapped blocks
    with the highest T, 8 independent seeds: the estimator Cov(g, H_b)/T_b^2 and the central difference with
    common random numbers (dT = 1e-3 T_b) agree within their standard errors, both are significantly positive, and
    their ratio is near one (the per-block chain is not exactly the Gibbs law the estimator assumes at block
    boundaries, so a small bias is allowed)."""
    sc, lb, z, m, t, rg, _ = c5
    T_host = np.random.default_rng(7).uniform(0.3, 1.2, 256).astype(np.float32).reshape(16, 16)
    gapn = (sc.mask == 0).astype(np.int64).reshape(16, 32, 16, 32).sum(axis=(1, 3)).ravel()
    cand = np.flatnonzero((gapn >= 200) & (gapn <= 800))
    blocks = cand[np.argsort(-T_host.ravel()[cand], kind="stable")[:6]]
    base = M.mpr_simulate(t, m, dev(T_host), 32, 32, _cfg(99), want_energy=False)
    tbar = base.state.double().mean(0)
    gap = m == 0
    losses = {}
    for b in blocks:
        by, bx = divmod(int(b), 16)
        C = torch.zeros_like(tbar)
        sl = (slice(by * 32, by * 32 + 32), slice(bx * 32, bx * 32 + 32))
        C[sl] = torch.sign(0.5 - tbar[sl]) * gap[sl] / float(gapn[b])
        losses[b] = lambda zh, C=C: (zh.double() * C).sum()
    print("blocks", blocks, "T", T_host.ravel()[blocks], "gap sites", gapn[blocks], flush=True)
    est, fd = _fd_and_estimate(t, m, z, rg, T_host, blocks, losses, seeds=[1000 + i for i in range(8)])
    me, mf, se_e, se_f, zs = _summary(est, fd)
    assert np.all(np.abs(zs) < 4.0)
    assert np.sum(me > 3 * se_e) >= 4 and np.sum(mf > 3 * se_f) >= 4
    ratio = me.sum() / mf.sum()
    print(f"sum ratio estimator / finite differences {ratio:.3f}")
    assert 0.6 < ratio < 1.6


def test_validation_mae_gradient_consistent_with_crn_differences(c5):
    """Config 5 as specified: d(validation MAE)/dT_b at the calibrated temperatures on the 8 blocks with the most
    held-out pixels.  There the realization mean barely depends on a single block's temperature (first-order
    insensitivity at low T), and both estimates are dominated by their noise at R = 1024; the check is that they
    agree within it (4 seeds)."""
    sc, lb, z, m, t, rg, T = c5
    truth = dev(sc.z_true)
    ev = dev(sc.eval_mask.astype(bool))
    counts = sc.eval_mask.astype(np.int64).reshape(16, 32, 16, 32).sum(axis=(1, 3)).ravel()
    blocks = np.argsort(-counts, kind="stable")[:8]
    losses = {b: (lambda zh: _loss(zh, truth, ev)) for b in blocks}
    est, fd = _fd_and_estimate(t, m, z, rg, host(T), blocks, losses, seeds=[2000 + i for i in range(4)])
    _, _, _, _, zs = _summary(est, fd)
    assert np.all(np.isfinite(est)) and np.all(np.isfinite(fd))
    assert np.all(np.abs(zs) < 5.0)
