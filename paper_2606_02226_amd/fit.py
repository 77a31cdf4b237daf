"""Fitting the maps of a 2D affine system to a target density.

Section 4 of the paper proposes generating a primitive's point distribution
automatically with autodiff-like tools.  `fit` does that for the parameters
theta [n][6] = (a00, a01, a10, a11, b0, b1) of an affine system: every step
renders the Gaussian-splatted density with cfs_splat, forms the L2 loss
against the target and its gradient with cfs_l2_loss, runs the adjoint
(cfs_splat_backward) and applies an Adam update to the few parameters on
the host.  The random streams are the same
every step (common random numbers), so the loss is a deterministic function
of theta and reaches zero at the target's parameters.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api


def fit(theta0, target, run, image_desc, *, sigma_px=1.0, steps=200, lr=2e-3,
        ckpt_every=8, betas=(0.9, 0.999), eps=1e-12, prob=None, device="cuda"):
    """Minimise sum((D(theta) - target)^2) over theta from theta0.

    Returns (theta, history) with history the loss of every step.  The
    learning rate follows a cosine schedule from lr down to lr / 20."""
    theta = np.asarray(theta0, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    tgt = torch.as_tensor(target, dtype=torch.float32, device=device).contiguous()
    N, T = int(run["n_points"]), int(run["n_iters"])
    ckpt = torch.empty((api.n_checkpoints(T, ckpt_every), N, 2), dtype=torch.float32,
                       device=device)
    img = api.Image(image_desc, device=device)
    dLdD = torch.empty_like(tgt)
    loss_ws = None
    history = []
    for step in range(steps):
        system = api.theta_to_system(theta.astype(np.float32), prob=prob)
        img.clear()
        api.splat(system, run, img, sigma_px, ckpt=ckpt, ckpt_every=ckpt_every)
        loss, dLdD = api.l2_loss(img.data, tgt, grad=dLdD, workspace=loss_ws)
        g = api.splat_backward(system, run, img, sigma_px, dLdD, ckpt,
                               ckpt_every).double().cpu().numpy()
        history.append(float(loss.item()))
        m = betas[0] * m + (1 - betas[0]) * g
        v = betas[1] * v + (1 - betas[1]) * g * g
        mh = m / (1 - betas[0] ** (step + 1))
        vh = v / (1 - betas[1] ** (step + 1))
        rate = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / max(steps - 1, 1))))
        theta = theta - rate * mh / (np.sqrt(vh) + eps)
    return theta, history
