"""torch.autograd binding of the temperature gradient (mpr_block_energy + mpr_temperature_grad).

``MPRFunction.apply(T_map, t, mask, z, rng, block, cfg)`` returns the realization-averaged prediction zhat of a
conditional simulation at block temperatures T_map (one sampling sweep); its backward gives dL/dT_map by the
score-function estimate Cov_r(g_r, H_rb) / T_b^2 computed on the device in FP64.
"""
from __future__ import annotations

import dataclasses

import torch

from ._lib import SimConfig, mpr_block_energy, mpr_predict, mpr_simulate, mpr_temperature_grad


class MPRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T_map, t, mask, z, rng, block, cfg: SimConfig):
        lb_h, lb_w = int(block[0]), int(block[1])
        if cfg.n_real < 2:
            raise ValueError("the gradient needs at least two realizations")
        c = dataclasses.replace(cfg, n_samp=1)
        T32 = T_map.detach().to(torch.float32).contiguous()
        sim = mpr_simulate(t, mask, T32, lb_h, lb_w, c, want_energy=False)
        zhat = mpr_predict(sim.acc, z, mask, c.n_real, rng)
        Hrb = mpr_block_energy(sim.state, mask, lb_h, lb_w, c.q, c.J)
        ctx.save_for_backward(sim.state, Hrb, mask, rng, T32)
        ctx.t_shape = T_map.shape
        ctx.t_dtype = T_map.dtype
        ctx.sweeps = sim.sweeps
        return zhat

    @staticmethod
    def backward(ctx, grad_zhat):
        state, Hrb, mask, rng, T32 = ctx.saved_tensors
        dT = mpr_temperature_grad(state, Hrb, grad_zhat.to(torch.float32).contiguous(), mask, rng, T32)
        return dT.reshape(ctx.t_shape).to(ctx.t_dtype), None, None, None, None, None, None
