"""torch.autograd.Function over the library's forward step and gradient.

theta = (eps2/eps1, eps3/eps1, sigma2/sigma1, sigma3/sigma1, E0): the
forward builds the instance's parameters from theta (phases 2 and 3 scaled
against phase 1; the applied field scaled about the electrodes' mean
potential, initial potential guess included), runs the steps in the chosen
precision (FP32 or FP64) while checkpointing every ckpt_every steps
(lbm_ehd_record), and returns the order parameters of the last step.  The
backward passes the incoming gradient as the seed of lbm_ehd_adjoint, whose
reverse sweep recomputes the segments from those checkpoints and returns
dJ/dtheta in the forward's precision.
"""
from __future__ import annotations

import torch

from . import binding
from .inputs import applied_field, theta_of, with_theta  # noqa: F401  (re-exported)


class LbmEhdFn(torch.autograd.Function):
    """phi = LbmEhdFn.apply(theta, cfg, init, n_steps, precision, ckpt_every):
    order parameters [3, ny, nx] after n_steps."""

    @staticmethod
    def forward(ctx, theta, cfg, init, n_steps, precision="fp32", ckpt_every=250):
        c, ini = with_theta(cfg, init, theta.detach().cpu().tolist())
        sim = binding.Sim(c, ini, precision=precision)
        sim.record(int(n_steps), int(ckpt_every))
        f = sim.fields(["phi1", "phi2", "phi3"])
        ctx.sim, ctx.n, ctx.every = sim, int(n_steps), int(ckpt_every)
        ctx.dtype, ctx.device = theta.dtype, theta.device
        return torch.stack([f["phi1"], f["phi2"], f["phi3"]])

    @staticmethod
    def backward(ctx, grad_phi):
        g = ctx.sim.adjoint(ctx.n, {"phi1": grad_phi[0], "phi2": grad_phi[1], "phi3": grad_phi[2]}, ctx.every)
        ctx.sim = None
        return torch.tensor(g, dtype=ctx.dtype, device=ctx.device), None, None, None, None, None


def drop_indicator(w):
    """The deformation indicator of lbm_ehd_diagnostics (tail below 0.005
    dropped, smoothstep to full weight at 0.02), differentiable."""
    s = torch.clamp((w - 0.005) / 0.015, 0.0, 1.0)
    return torch.where(w <= 0.005, torch.zeros_like(w), w * s * s * (3 - 2 * s))


def deformation(w):
    """(sqrt(I_par) - sqrt(I_perp)) / (sqrt(I_par) + sqrt(I_perp)) of an
    indicator field w [ny, nx], parallel = y."""
    ny, nx = w.shape
    y = torch.arange(ny, dtype=w.dtype, device=w.device)[:, None]
    x = torch.arange(nx, dtype=w.dtype, device=w.device)[None, :]
    W = w.sum()
    xb, yb = (w * x).sum() / W, (w * y).sum() / W
    a = torch.sqrt((w * (y - yb) ** 2).sum() / W)
    b = torch.sqrt((w * (x - xb) ** 2).sum() / W)
    return (a - b) / (a + b)
