"""torch.autograd wrapper of the differentiable chaos game.

``CFSSplat.apply(theta, run, image_desc, sigma_px, ckpt_every)`` maps the map
parameters theta [n][6] = (a00, a01, a10, a11, b0, b1) of a 2D affine system
to its Gaussian-splatted FP32 density [H][W] (cfs_splat); its backward runs
the hand-written adjoint kernel through the checkpointed trajectory
(cfs_splat_backward).  Selection probabilities are not differentiated.
"""
from __future__ import annotations

import torch

from . import api


class CFSSplat(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, run, image_desc, sigma_px=1.0, ckpt_every=8, prob=None):
        system = api.theta_to_system(theta, prob=prob)
        dev = theta.device
        img = api.Image(image_desc, device=dev).clear()
        N, T = int(run["n_points"]), int(run["n_iters"])
        ckpt = torch.empty((api.n_checkpoints(T, ckpt_every), N, 2), dtype=torch.float32,
                           device=dev)
        api.splat(system, run, img, sigma_px, ckpt=ckpt, ckpt_every=ckpt_every)
        ctx.system, ctx.run, ctx.sigma, ctx.every = system, run, sigma_px, ckpt_every
        ctx.img = img
        ctx.save_for_backward(ckpt)
        return img.data.clone()

    @staticmethod
    def backward(ctx, grad_out):
        (ckpt,) = ctx.saved_tensors
        g = api.splat_backward(ctx.system, ctx.run, ctx.img, ctx.sigma,
                               grad_out.to(torch.float32).contiguous(), ckpt, ctx.every)
        return g, None, None, None, None, None


def cfs_splat(theta, run, image_desc, sigma_px=1.0, ckpt_every=8, prob=None):
    return CFSSplat.apply(theta, run, image_desc, sigma_px, ckpt_every, prob)
