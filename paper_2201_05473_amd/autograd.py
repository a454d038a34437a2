"""torch.autograd.Function around lbm_adjoint: the witness wakefield J(theta) with
theta = (ramp_len, n0, sigma_r, nb), differentiable through the hand-written HIP adjoint."""
from __future__ import annotations

import torch

from .binding import Lattice

THETA_NAMES = ("ramp_len", "n0", "sigma_r", "nb")


class LbmWake(torch.autograd.Function):
    """forward(theta, cfg, nsteps, ckpt_every, n_pert, z_behind, row) -> J (FP64 scalar).

    When theta needs a gradient, the forward pass runs lbm_adjoint (forward with checkpoints,
    reverse sweep), so backward only scales the stored gradient: dL/dtheta = dL/dJ * dJ/dtheta.
    Otherwise (no_grad, or theta without requires_grad) it runs the plain forward steps and
    evaluates the same objective with lbm_witness, at the cost of a forward run."""

    @staticmethod
    def forward(ctx, theta, cfg, nsteps, ckpt_every, n_pert, z_behind, row):
        th = theta.detach().to(torch.float64).cpu()
        c = dict(cfg)
        for name, v in zip(THETA_NAMES, th.tolist()):
            c[name] = v
        lat = Lattice(c, n_pert)
        if ctx.needs_input_grad[0]:
            J, grad = lat.adjoint(int(nsteps), ckpt_every, float(z_behind), int(row))
        else:
            lat.step(int(nsteps))
            J, grad = lat.witness(float(z_behind), int(row)), [float("nan")] * 4
        lat.close()
        ctx.save_for_backward(torch.as_tensor(grad, dtype=torch.float64))
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        gt = (grad_out.to(torch.float64).cpu() * g).to(ctx.theta_dtype).to(ctx.theta_device)
        return gt, None, None, None, None, None, None


def wake_objective(theta: torch.Tensor, cfg: dict, nsteps: int, ckpt_every: int | None = None,
                   n_pert=None, z_behind: float = 4.0, row: int = 0) -> torch.Tensor:
    """J(theta) as a differentiable torch scalar."""
    return LbmWake.apply(theta, cfg, nsteps, ckpt_every, n_pert, z_behind, row)
