"""Differentiable ERP rasterisation as a torch.autograd.Function.

``OmniRasterize.apply(means, scales, quats, opacities, sh, camera, settings)``
renders the [3, H, W] ERP image with ``omnigs_forward`` and, on backward,
calls ``omnigs_backward`` with the saved state (final transmittance and
contributor counts per pixel, sorted tile lists, blend records), which
re-walks each pixel's list instead of storing it.  Gradients are returned
for the five parameter tensors as the library defines them: w.r.t. the
activated scales and opacities, the raw quaternion, the means and the SH
coefficients.  Parameter activations (exp, sigmoid, ...) belong to the
caller's PyTorch graph.  The screen-space gradient dL/ds (used by
densification) is stored on ``ctx.screen_grad_sink`` when one is given.
"""
from __future__ import annotations

import torch

from . import omnigs


class OmniRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, camera, settings=None, screen_grad_sink=None):
        sh_degree = int(round((sh.shape[1]) ** 0.5)) - 1 if settings is None or "sh_degree" not in settings \
            else int(settings["sh_degree"])
        st = {k: v for k, v in (settings or {}).items() if k != "sh_degree"}
        g = dict(means=means.contiguous(), scales=scales.contiguous(), quats=quats.contiguous(),
                 opacities=opacities.contiguous(), sh=sh.contiguous(), sh_degree=sh_degree)
        fwd = omnigs.omnigs_forward(g, camera, st)
        ctx.g = g
        ctx.camera = camera
        ctx.settings = st
        ctx.fwd = fwd
        ctx.sink = screen_grad_sink
        ctx.mark_non_differentiable(fwd.final_T, fwd.n_contrib)
        return fwd.image, fwd.final_T, fwd.n_contrib

    @staticmethod
    def backward(ctx, grad_image, grad_T=None, grad_nc=None):
        grads = omnigs.omnigs_backward(ctx.g, ctx.camera, ctx.settings, ctx.fwd, grad_image.contiguous())
        if ctx.sink is not None:
            ctx.sink.append(grads["screen"])
        return grads["means"], grads["scales"], grads["quats"], grads["opacities"], grads["sh"], None, None, None


def rasterize(means, scales, quats, opacities, sh, camera, settings=None, sh_degree=None, screen_grad_sink=None):
    """Render; returns (image [3,H,W], final_T [H,W], n_contrib [H,W])."""
    st = dict(settings or {})
    if sh_degree is not None:
        st["sh_degree"] = sh_degree
    return OmniRasterize.apply(means, scales, quats, opacities, sh, camera, st, screen_grad_sink)
