"""Torch-facing helpers over the C ABI: output allocation and a
torch.autograd.Function whose backward uses the library's hand-written adjoint.

PyTorch provides device memory and streams only; every step of the evaluation
runs in librtu.so.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import GEOM_EPL, GEOM_UNIFORM, Plan, make_geometry


@dataclasses.dataclass
class Result:
    loss: torch.Tensor            # float64 [B]
    chi2_mask: torch.Tensor       # float64 [B]
    status: torch.Tensor          # int32 [B] (uint32 bits)
    grad_lens: Optional[torch.Tensor] = None
    grad_ps: Optional[torch.Tensor] = None
    grad_latent: Optional[torch.Tensor] = None
    model: Optional[torch.Tensor] = None


def plan_for_problem(problem, max_batch: Optional[int] = None, device: int = 0, flags: int = 0) -> Plan:
    """Plan + observation for a problem from the seeded input generator."""
    g = problem.geom
    if getattr(g, "uniform", False):
        flags |= GEOM_UNIFORM
    if getattr(g, "epl", False):
        flags |= GEOM_EPL
    geom = make_geometry(g.n_img, g.supersample, g.n_src, g.psf_size, g.pixel_scale,
                         g.n_sub_max, g.tnfw_tau, flags, g.n_gauss)
    plan = Plan(geom, max_batch or problem.batch, device)
    plan.set_observation(problem.image, problem.noise_sigma, problem.psf, problem.mask)
    if getattr(problem, "ray_weights", None) is not None:
        plan.set_ray_weights(problem.ray_weights)
    return plan


def device_inputs(problem, device="cuda"):
    """Upload a problem's per-sample inputs (lens, ps, latent, n_sub)."""
    return (torch.from_numpy(problem.lens).to(device), torch.from_numpy(problem.ps).to(device),
            torch.from_numpy(problem.latent).to(device),
            torch.from_numpy(problem.n_sub.astype(np.int32)).to(device))


def evaluate(plan: Plan, lens, ps, latent, n_sub=None, want_grad=True, want_model=False,
             stream=None) -> Result:
    """Allocate outputs and queue one evaluation (asynchronous)."""
    B = lens.shape[0]
    dev = lens.device
    res = Result(loss=torch.empty(B, dtype=torch.float64, device=dev),
                 chi2_mask=torch.empty(B, dtype=torch.float64, device=dev),
                 status=torch.empty(B, dtype=torch.int32, device=dev))
    if want_grad:
        res.grad_lens = torch.empty_like(lens)
        res.grad_ps = torch.empty_like(ps)
        res.grad_latent = torch.empty_like(latent)
    if want_model:
        n = plan.geom.n_img
        res.model = torch.empty((B, n, n), dtype=torch.float32, device=dev)
    plan.loss_grad(lens, ps, latent, n_sub, loss=res.loss, status=res.status, chi2_mask=res.chi2_mask,
                   grad_lens=res.grad_lens, grad_ps=res.grad_ps, grad_latent=res.grad_latent,
                   model=res.model, stream=stream)
    return res


class RTULoss(torch.autograd.Function):
    """loss[B] = chi^2/2 + |w|^2/2 per sample.  The forward call computes the
    gradients with the library's adjoint chain; backward scales them."""

    @staticmethod
    def forward(ctx, lens, ps, latent, plan: Plan, n_sub=None):
        r = evaluate(plan, lens.detach().contiguous(), ps.detach().contiguous(),
                     latent.detach().contiguous(), n_sub, want_grad=True)
        ctx.save_for_backward(r.grad_lens, r.grad_ps, r.grad_latent)
        ctx.status = r.status
        return r.loss

    @staticmethod
    def backward(ctx, gout):
        gl, gp, gw = ctx.saved_tensors
        g = gout.to(gl.dtype)
        return g[:, None] * gl, g[:, None] * gp, g[:, None, None] * gw, None, None
