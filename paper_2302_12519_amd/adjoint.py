"""Activation-time loss as a differentiable function of the per-voxel
conductivity scale (``torch.autograd.Function``).

When the scale needs a gradient, the forward call runs the explicit
monodomain simulation and the discrete adjoint together in the HIP library
(``ep_adjoint_scale``: checkpointed forward, per-segment recompute, one fused
adjoint kernel per step) and autograd's backward only multiplies the stored
gradient by the incoming cotangent; otherwise it runs the forward simulation
and the loss alone.  torch carries the tensors; no arithmetic of the method
runs here.
"""
from __future__ import annotations

import numpy as np
import torch

from .ep import Grid


class ActivationTimeLoss(torch.autograd.Function):
    """L(s) = sum over voxels activated in the run with a finite target of
    (T_act(s) - T*)^2, for D = s D0 on an explicit monodomain ``Grid``."""

    @staticmethod
    def forward(ctx, scale, grid, fibre, sig_l, sig_t, v0, w0, step0, tstar, nsteps,
                ckpt_every):
        s = scale.detach().to("cpu", torch.float64).numpy()
        grid.set_conductivity(fibre, s, sig_l, sig_t)
        grid.write("v", v0)
        grid.write("w", w0)
        grid.step_index = int(step0)
        want = bool(ctx.needs_input_grad[0])
        loss, grad, used = grid.adjoint_scale(tstar, nsteps, ckpt_every, grad=want)
        ctx.grad = (torch.from_numpy(np.ascontiguousarray(grad)).to(scale.device, scale.dtype)
                    if want else None)
        ctx.n_used = used
        return torch.tensor(loss, dtype=scale.dtype, device=scale.device)

    @staticmethod
    def backward(ctx, gout):
        return (gout * ctx.grad if ctx.grad is not None else None,) + (None,) * 10


def activation_time_loss(grid: Grid, scale, fibre, sig_l, sig_t, tstar, nsteps, v0=None,
                         w0=None, step0=0, ckpt_every=0):
    """Differentiable activation-time loss; ``scale`` is a box-shaped tensor.
    The run starts from (v0, w0) at step ``step0`` (default: rest, v = 0,
    w = 1) and leaves ``grid`` in its final state."""
    if v0 is None:
        v0 = np.zeros(grid.n)
    if w0 is None:
        w0 = np.ones(grid.n)
    return ActivationTimeLoss.apply(scale, grid, fibre, sig_l, sig_t, v0, w0, step0, tstar,
                                    nsteps, ckpt_every)
