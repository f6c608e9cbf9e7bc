"""Multi-step optimisation through the stochastic ray tracer.

Sec. 7 of the paper points at differentiable rendering as the use of a
gradient through stochastic transparency. This loop fits Gaussian parameters
to target images: every step renders the views with the forward kernel,
takes the L2 loss, runs the hand-written backward (an unbiased estimate of
the exact composite's gradient) and applies Adam. The BVH is built once and
refit to the updated parameters before each step's forward (same topology,
new records and boxes), so a step costs a refit instead of a build.
"""
from __future__ import annotations

import torch

from . import DeviceScene, render, srt_build_bvh

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def fit(params, sh_degree, origins, dirs, target, *, steps, lr, spp=4, n_per_traversal=4,
        seed=0, image_width=0, width=4, leaf_size=4, estimator="plain", log=None):
    """Adam on mean((render - target)^2) over the parameters named in `lr`.

    params: dict of the five device tensors (FP32, contiguous) of a scene;
    those named in `lr` (a dict name -> learning rate) are updated in place.
    origins, dirs, target: [R,3] device tensors (several views may be stacked;
    image_width > 0 declares them a row-major image of that width).
    Step k draws samples k*spp .. k*spp+spp-1, so steps see fresh noise.
    Returns the list of per-step (stochastic) losses.
    """
    for name in lr:
        if name not in PARAM_NAMES:
            raise ValueError(f"unknown parameter {name!r}")
    leaves = {n: params[n] for n in PARAM_NAMES}
    for n in lr:
        leaves[n].requires_grad_(True)
    opt = torch.optim.Adam([{"params": [leaves[n]], "lr": float(v)} for n, v in lr.items()])
    scene = DeviceScene(*(leaves[n].detach() for n in PARAM_NAMES), sh_degree)
    bvh = srt_build_bvh(scene, width, leaf_size)
    losses = []
    R = int(origins.shape[0])
    for k in range(int(steps)):
        opt.zero_grad(set_to_none=True)
        rgb = render(*(leaves[n] for n in PARAM_NAMES), origins, dirs, sh_degree=sh_degree,
                     spp=spp, n_per_traversal=n_per_traversal, seed=seed,
                     sample_offset=k * spp, image_width=image_width, estimator=estimator,
                     bvh=bvh)
        loss = ((rgb - target) ** 2).sum() / (3 * R)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
        if log:
            log(k, losses[-1])
    for n in lr:
        leaves[n].requires_grad_(False)
    return losses
