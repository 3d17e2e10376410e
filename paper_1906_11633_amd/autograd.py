"""Differentiable shading: a torch.autograd.Function over the HIP renderer.

The forward pass renders RGB (and keeps the visibility keys); the backward pass calls
the library's hand-written shading adjoint over that fixed visibility.  Gradients flow
to the per-object albedo, roughness and specular, the per-light world position and
intensity, and the per-frame exposure (the randomization parameters of ORRB's
material, light and post-processing randomizers).  Geometry (poses, cameras) is held
fixed: visibility does not depend on the differentiated parameters.
"""
from __future__ import annotations

import torch

from .renderer import render_batch, shade_backward

PARAMS = ("albedo", "roughness", "specular", "light_vec", "light_intensity", "exposure")


class ShadeFn(torch.autograd.Function):
    """rgb = ShadeFn.apply(renderer, job, albedo, roughness, specular, light_vec,
    light_intensity, exposure); rgb is the planar [3P] float32 image buffer."""

    @staticmethod
    def forward(ctx, renderer, job, albedo, roughness, specular, light_vec, light_intensity, exposure):
        state = dict(job.state)
        for k, t in zip(PARAMS, (albedo, roughness, specular, light_vec, light_intensity, exposure)):
            state[k] = t.detach().contiguous()
        out = renderer.alloc_outputs(job, vis=True)
        render_batch(renderer.ctx, job.layout, state, out, job.workspace)
        ctx.renderer, ctx.job, ctx.state, ctx.vis = renderer, job, state, out["vis"]
        return out["rgb"]

    @staticmethod
    def backward(ctx, grad_rgb):
        g = shade_backward(ctx.renderer.ctx, ctx.job.layout, ctx.state, ctx.vis, grad_rgb.float(),
                           workspace=ctx.job.extra.get("grad_workspace"))
        return (None, None, g["albedo"], g["roughness"], g["specular"], g["light_vec"], g["light_intensity"],
                g["exposure"])


def shade(renderer, job, albedo, roughness, specular, light_vec, light_intensity, exposure):
    return ShadeFn.apply(renderer, job, albedo, roughness, specular, light_vec, light_intensity, exposure)
