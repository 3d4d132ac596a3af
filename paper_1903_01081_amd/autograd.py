"""torch.autograd wrapper: recorded waveforms as a differentiable function of
the line parameters, with the backward pass run by the HIP adjoint kernel
(reverse-time transposed solves through the same factors, from checkpoints).
"""
from __future__ import annotations

import torch

from .sim import Simulator


class EMTFunction(torch.autograd.Function):
    """rec = EMTFunction.apply(theta, sim): theta [S, P] -> rec [S, T, R].

    The simulator must be built with checkpoint_every > 0. Its state after
    forward is consumed by backward, so run backward before the next forward
    on the same simulator.
    """

    @staticmethod
    def forward(ctx, theta: torch.Tensor, sim: Simulator):
        sim.set_params(theta.detach().contiguous())
        sim.factor()
        rec = sim.run()
        ctx.sim = sim
        return rec

    @staticmethod
    def backward(ctx, grad_rec: torch.Tensor):
        grad = ctx.sim.adjoint(grad_rec.contiguous())
        return grad, None


def simulate(theta: torch.Tensor, sim: Simulator) -> torch.Tensor:
    return EMTFunction.apply(theta, sim)
