"""torch.autograd.Function over the C ABI.

The forward keeps only what the backward needs to replay the blending in
reverse: per pixel the final transmittance and the index of the last
composited list entry, plus the view's projection records and tile lists.
No per-fragment state is stored; the backward recovers each fragment's
transmittance from the final one (T_before = T_after / (1 - alpha)).

Inputs are activated parameters (opacity in (0,1], sigma > 0); any
reparameterisation (sigmoid, exp) belongs to the caller.
"""
from __future__ import annotations

import torch

from .render import Rasterizer, ViewState


class TriangleRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, o, sigma, sh, cam, cfg, capacity_hint=None):
        scene_t = tuple(t.detach().contiguous().float() for t in (v, o, sigma, sh))
        N = scene_t[0].shape[0]
        cap = capacity_hint or max(4 * N, 1 << 16)
        st = ViewState(N, cam.width, cam.height, cap, device=v.device)
        ras = Rasterizer(cfg, device=v.device)
        out = ras.forward(st, scene_t, cam, sync=True)
        ctx.state = (ras, st, scene_t, out)
        ctx.mark_non_differentiable(out.T_final)
        return out.rgb, out.alpha, out.depth

    @staticmethod
    def backward(ctx, g_rgb, g_alpha, g_depth):
        ras, st, scene_t, out = ctx.state
        dC = (g_rgb if g_rgb is not None else torch.zeros_like(out.rgb)).contiguous().float()
        dA = None if g_alpha is None else g_alpha.contiguous().float()
        dD = None if g_depth is None else g_depth.contiguous().float()
        gv, go, gs, gsh = ras.backward(st, scene_t, out, dC, dA, dD)
        ctx.state = None
        return gv, go, gs, gsh, None, None, None


def rasterize(v, o, sigma, sh, cam, cfg, capacity_hint=None):
    """Differentiable render of one view: (rgb [3,H,W], alpha [H,W], depth [H,W])."""
    return TriangleRasterize.apply(v, o, sigma, sh, cam, cfg, capacity_hint)
