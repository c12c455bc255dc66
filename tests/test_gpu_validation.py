"""The validation harness (Sec. 3.2) against the oracle: for every method and mask the oracle recomputes the whole
prediction (map, temperatures, SST smoothing, simulation with the Sec. 3.4 test, conditional mean) and the MAAE and
MRASE the harness reports."""
import numpy as np
import pytest

import oracle
from oracle import SimConfig as OCfg
from paper_2212_01317_amd import reference_curve, synth
from paper_2212_01317_amd import validation as V

pytestmark = pytest.mark.gpu


def _oracle_errors(field, mask, method, s, cT, ce, scene):
    H, W = field.shape
    z = (field * mask).astype(np.float32)
    t, rg = oracle.map_angles(z, mask)
    if method == "MPR":
        lb, init = (H, W), 0
    else:
        lb, init = (s.block, s.block), 1
    T, _, _ = oracle.calibrate_temperature(t, mask, lb[0], lb[1], cT, ce)
    t_mode, order, directional = 0, 1 if method == "BST-DC" else 0, 0
    if method == "BST-DIR":
        T = np.concatenate([x.ravel() for x in oracle.calibrate_directional(t, mask, lb[0], lb[1], cT, ce)])
        directional = 1
    if method == "SST":
        T = oracle.sst_temperatures(T, H, W, lb[0], lb[1], r_s=s.r_s, n_s=s.n_s)
        t_mode = 1
    cfg = OCfg(n_real=s.n_real, init_mode=init, stop_mode=1, n_samp=s.n_samp, n_max=s.n_max, seed=s.seed,
               scene=scene, t_mode=t_mode, order=order, directional=directional)
    r = oracle.simulate(t, mask, T, lb[0], lb[1], cfg)
    zhat = oracle.predict(r.acc, z, mask, s.n_real * s.n_samp, rg)
    return oracle.validate(zhat, field, (1 - mask).astype(np.uint8))


def test_harness_matches_oracle():
    field = synth.skewed_field(48, 3)[:48, :40].copy()
    s = V.Setting(n_real=2, n_samp=1, block=16, n_max=80, seed=4)
    rows = V.run(field, [0.4], 2, V.ALL_METHODS, s)
    cT, ce = (x.cpu().numpy() for x in reference_curve(0.5))
    masks = V.masks_for(48, 40, 0.4, 2, s.seed)
    for row in rows:
        errs = [_oracle_errors(field, mk, row["method"], s, cT, ce, m) for m, mk in enumerate(masks)]
        maae, mrase = np.mean([e[0] for e in errs]), np.mean([e[1] for e in errs])
        print(row, f"oracle MAAE {maae:.6f} MRASE {mrase:.6f}", flush=True)
        assert abs(row["MAAE"] - maae) <= 1e-9 * abs(maae)
        assert abs(row["MRASE"] - mrase) <= 1e-9 * abs(mrase)
