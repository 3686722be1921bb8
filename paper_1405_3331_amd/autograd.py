"""torch.autograd binding of the trajectory-loss gradient.

``trajectory_loss(q, D, k, scenario, n_steps, assign, weight)`` runs the scenario with the
source amounts q (every species' sources concatenated, species 0 first), diffusion
coefficients D and decay rates k taken from the given tensors, and returns the loss
sum_i weight[i] |p_i^N - target[assign[i]]|^2 as a differentiable FP64 tensor.  Forward
and reverse sweeps both run in the HIP library (sim_adjoint_run / sim_adjoint_backward);
this module only moves scalars between torch and the C ABI.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import binding as B


def _with_parameters(sc, q, D, k):
    out = copy.deepcopy(sc)
    at = 0
    for s, spc in enumerate(out.species):
        n = len(spc.source_q)
        spc.source_q = np.asarray(q[at:at + n], dtype=np.float32).astype(np.float64)
        at += n
        spc.D = float(D[s])
        spc.k = float(k[s])
    return out


class TrajectoryLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, D, k, sc, n_steps, assign, weight, checkpoint_every, block_steps):
        run = _with_parameters(sc, q.detach().cpu().double().numpy(),
                               D.detach().cpu().double().numpy(),
                               k.detach().cpu().double().numpy())
        sim = B.Simulation(run, block_steps=block_steps)
        loss = sim.adjoint(n_steps, assign, weight, checkpoint_every)
        ctx.sim = sim
        ctx.devices = (q.device, D.device, k.device)
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad):
        dq, dD, dk = ctx.sim.adjoint_backward()
        ctx.sim.close()
        g = float(grad)
        out = [torch.as_tensor(v * g, dtype=torch.float64, device=dev)
               for v, dev in zip((dq, dD, dk), ctx.devices)]
        return out[0], out[1], out[2], None, None, None, None, None, None


def trajectory_loss(q, D, k, sc, n_steps, assign, weight, checkpoint_every=100, block_steps=0):
    return TrajectoryLoss.apply(q, D, k, sc, n_steps, np.asarray(assign), np.asarray(weight),
                                checkpoint_every, block_steps)
