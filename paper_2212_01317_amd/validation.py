"""Validation of the gap-filling methods in the manner of Sec. 3.2 (Tables 2 and 3, Fig. 10).

For a complete field and each missing-data ratio p, M masks remove round(p H W) pixels uniformly at random; every
method predicts the removed pixels from the rest; AAE and RASE (Eq. 3, Eq. 4) over the removed pixels are averaged
over the masks (MAAE, MRASE), next to the mean time of one prediction (map, temperatures, simulation, conditional
mean) on the device.  Methods: MPR (one global temperature, uniform random start), SV-MPR with block temperatures
(BST, Sec. 2.2.2; BST-DC: the same in the double-checkerboard order; BST-DIR: one temperature per bond direction
and block, the directional coupling suggested in Sec. 4) and with site temperatures (SST, Sec. 2.2.3);
for the SV-MPR methods every block size of `blocks`, and for SST every smoothing count of `ns` (the l_b and n_s
studies of Fig. 11).  Every step runs in the library; this module only draws the masks and orders the calls.

    python -m paper_2212_01317_amd.validation --L 256 --M 100 --p 0.1,0.3,0.5,0.7,0.9
    python -m paper_2212_01317_amd.validation --L 1024 --M 10 --p 0.3,0.8 --field ns --blocks 8,16,32,64

prints one JSON object per (p, method, block, n_s).  The paper's data sets are not available; the fields are seeded
stand-ins: `synth.skewed_field` (default), the plain non-stationary field `synth.ns_field` (--field ns), or a field
with geometric anisotropy `synth.grf_aniso` (--field aniso: correlation lengths 16 along x and 2 along y).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import INIT_BLOCK_MEAN, INIT_RANDOM, ORDER_DC, STOP_AUTO, STOP_AUTO_CHAIN, mpr_validate, predict, reference_curve
from . import synth

METHODS = ("MPR", "BST", "SST")
ALL_METHODS = ("MPR", "BST", "SST", "BST-DC", "BST-DIR")


@dataclass
class Setting:
    n_real: int = 10            # realizations per prediction
    n_samp: int = 1             # sampling sweeps per realization
    block: int = 32             # l_b of BST and SST
    r_s: int = 1                # SST smoothing radius
    n_s: int = 5                # SST smoothing passes (the paper's tables use 5)
    n_max: int = 1000
    seed: int = 0
    stop_mode: int = STOP_AUTO  # STOP_AUTO: the test on the realization-averaged energy; STOP_AUTO_CHAIN: per chain


def masks_for(H: int, W: int, p: float, M: int, seed: int, progress=None):
    """M masks (1 = sample) removing round(p H W) pixels uniformly; mask m depends only on (seed, p, m).
    progress(m), if given, is called after each mask (large grids take seconds per mask)."""
    out = []
    for m in range(M):
        rng = np.random.default_rng([seed, int(round(p * 1000)), m])
        out.append(synth.uniform_mask(H, W, int(round(p * H * W)), rng))
        if progress is not None:
            progress(m)
    return out


def predict_method(method: str, z: torch.Tensor, mask: torch.Tensor, s: Setting, curve, scene_id: int):
    H, W = int(z.shape[0]), int(z.shape[1])
    common = dict(n_real=s.n_real, n_samp=s.n_samp, n_max=s.n_max, seed=s.seed, scene_id=scene_id, curve=curve,
                  stop_mode=s.stop_mode)
    if method == "MPR":
        return predict(z, mask, block=(H, W), init_mode=INIT_RANDOM, **common)
    if method == "BST":
        return predict(z, mask, block=(s.block, s.block), init_mode=INIT_BLOCK_MEAN, **common)
    if method == "SST":
        return predict(z, mask, block=(s.block, s.block), init_mode=INIT_BLOCK_MEAN, sst=(s.r_s, s.n_s), **common)
    if method == "BST-DC":
        return predict(z, mask, block=(s.block, s.block), init_mode=INIT_BLOCK_MEAN, order=ORDER_DC, **common)
    if method == "BST-DIR":
        return predict(z, mask, block=(s.block, s.block), init_mode=INIT_BLOCK_MEAN, directional=True, **common)
    raise ValueError(f"unknown method {method}")


def variants(methods, s0: Setting, blocks, ns):
    """(method, setting) pairs: MPR once, BST and BST-DC per block size, SST per block size and smoothing count."""
    out = []
    for mt in methods:
        if mt == "MPR":
            out.append((mt, s0))
        elif mt == "SST":
            out += [(mt, dataclasses.replace(s0, block=b, n_s=n)) for b in blocks for n in ns]
        else:
            out += [(mt, dataclasses.replace(s0, block=b)) for b in blocks]
    return out


def run(field: np.ndarray, ps, M: int, methods=METHODS, setting: Setting | None = None, device="cuda",
        blocks=None, ns=None, on_row=None):
    """Rows {p, method, block, n_s, MAAE, MRASE, t_ms, sweeps, k_star} for every p and variant (sweeps: mean of
    k* + n_samp; k_star: mean k*); the same masks for every variant; on_row(row), if given, is called with each
    row as soon as it is complete."""
    s0 = setting or Setting()
    blocks = list(blocks) if blocks else [s0.block]
    ns = list(ns) if ns else [s0.n_s]
    dev = torch.device(device)
    H, W = field.shape
    truth = torch.from_numpy(np.ascontiguousarray(field, dtype=np.float32)).to(dev)
    curve = reference_curve(0.5, dev)
    rows = []
    for p in ps:
        big = H * W >= (1 << 24)
        masks = masks_for(H, W, float(p), M, s0.seed,
                          progress=(lambda m: print(f"[validation] p={p}: mask {m + 1}/{M}", file=sys.stderr,
                                                    flush=True)) if big else None)
        for method, s in variants(methods, s0, blocks, ns):
            aae, rase, times, sweeps, kst = [], [], [], [], []
            for m, mk in enumerate(masks):
                mask = torch.from_numpy(mk).to(dev)
                ev = (1 - mask).contiguous()
                z = (truth * mask).contiguous()         # removed values are not read; zeroed for clarity
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pr = predict_method(method, z, mask, s, curve, scene_id=m)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                e = mpr_validate(pr.zhat, truth, ev).cpu().numpy()
                aae.append(float(e[0]))
                rase.append(float(e[1]))
                sweeps.append(pr.sim.sweeps + s.n_samp)
                kst.append(pr.sim.sweeps)
                if big and (m + 1) % 10 == 0:
                    print(f"[validation] p={p} {method}: {m + 1}/{M} predictions", file=sys.stderr, flush=True)
            rows.append(dict(p=float(p), method=method, block=None if method == "MPR" else s.block,
                             n_s=s.n_s if method == "SST" else None, MAAE=float(np.mean(aae)), MRASE=float(np.mean(rase)),
                             t_ms=1e3 * float(np.mean(times)), sweeps=float(np.mean(sweeps)),
                             k_star=float(np.mean(kst)), stop="chain" if s.stop_mode == STOP_AUTO_CHAIN else "mean",
                             n_real=s.n_real, M=M, L=[H, W]))
            if on_row is not None:
                on_row(rows[-1])        # each row as soon as it is complete
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--M", type=int, default=100)
    ap.add_argument("--p", type=str, default="0.1,0.2,0.3,0.4,0.5,0.6,0.7,0.8,0.9")
    ap.add_argument("--methods", type=str, default=",".join(METHODS))
    ap.add_argument("--n-real", type=int, default=10)
    ap.add_argument("--blocks", type=str, default="32", help="block sizes l_b of the SV-MPR methods")
    ap.add_argument("--ns", type=str, default="5", help="smoothing counts n_s of SST")
    ap.add_argument("--field", choices=("skewed", "ns", "aniso"), default="skewed")
    ap.add_argument("--field-seed", type=int, default=synth.seed_for(6, synth.ROLE_FIELD))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--stop", choices=("mean", "chain"), default="mean",
                    help="equilibrium test on the realization-averaged energy (mean) or on every chain's own (chain)")
    a = ap.parse_args()
    if a.field == "skewed":
        field = synth.skewed_field(a.L, a.field_seed)
    elif a.field == "aniso":
        field = synth.grf_aniso(a.L, a.L, 16.0, 2.0, np.random.default_rng(a.field_seed)).astype(np.float32)
    else:
        field = synth.ns_field(a.L, a.L, 4, (2.0, 32.0), np.random.default_rng(a.field_seed)).astype(np.float32)
    run(field, [float(x) for x in a.p.split(",")], a.M, a.methods.split(","),
        Setting(n_real=a.n_real, seed=a.seed, stop_mode=STOP_AUTO_CHAIN if a.stop == "chain" else STOP_AUTO),
        blocks=[int(b) for b in a.blocks.split(",")], ns=[int(n) for n in a.ns.split(",")],
        on_row=lambda r: print(json.dumps(r), flush=True))


if __name__ == "__main__":
    main()
