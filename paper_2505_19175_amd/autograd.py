"""torch.autograd.Function over the C ABI.

The forward keeps only what the backward needs to replay the blending in
reverse: per pixel the final transmittance and the index of the last
composited list entry, plus the view's projection records and tile lists.
No per-fragment state is stored; the backward recovers each fragment's
transmittance from the final one (T_before = T_after / (1 - alpha)).

Inputs are activated parameters (opacity in (0,1], sigma > 0); any
reparameterisation (sigmoid, exp) belongs to the caller.  The gradient is
end to end through every parameter of every triangle (Sec. 3.3): vertices,
opacity, window sharpness and SH coefficients.

Outputs the loss does not use arrive as None in the backward (gradients are
not materialised), so an rgb-only loss reads no alpha or depth upstream.
The backward itself is not differentiable (no double backward).
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from .render import Rasterizer, ViewState


def _check_inputs(v, o, sigma, sh, cfg):
    ts = (v, o, sigma, sh)
    for name, t in zip(("v", "o", "sigma", "sh"), ts):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"rasterize: {name} must be a tensor")
        if t.device.type != "cuda":
            raise ValueError(f"rasterize: {name} is on {t.device}; every input must be on the GPU")
        if t.device != v.device:
            raise ValueError(f"rasterize: {name} is on {t.device}, v on {v.device}")
        if not t.is_floating_point():
            raise TypeError(f"rasterize: {name} must be floating point, got {t.dtype}")
    N = v.shape[0] if v.dim() == 3 else -1
    if v.dim() != 3 or tuple(v.shape[1:]) != (3, 3):
        raise ValueError(f"rasterize: v must be [N,3,3], got {tuple(v.shape)}")
    if tuple(o.shape) != (N,) or tuple(sigma.shape) != (N,):
        raise ValueError(f"rasterize: o and sigma must be [N]={N}, got {tuple(o.shape)}, "
                         f"{tuple(sigma.shape)}")
    K = (int(cfg.sh_degree) + 1) ** 2
    if tuple(sh.shape) != (N, K, 3):
        raise ValueError(f"rasterize: sh must be [N,(deg+1)^2,3]=[{N},{K},3] for SH degree "
                         f"{cfg.sh_degree}, got {tuple(sh.shape)}")


class TriangleRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, o, sigma, sh, cam, cfg, capacity_hint=None):
        _check_inputs(v, o, sigma, sh, cfg)
        ctx.set_materialize_grads(False)
        scene_t = tuple(t.detach().contiguous().float() for t in (v, o, sigma, sh))
        N = scene_t[0].shape[0]
        cap = capacity_hint or max(4 * N, 1 << 16)
        st = ViewState(N, cam.width, cam.height, cap, device=v.device)
        ras = Rasterizer(cfg, device=v.device)
        out = ras.forward(st, scene_t, cam, sync=True)
        ctx.state = (ras, st, scene_t, out)
        ctx.dtypes = tuple(t.dtype for t in (v, o, sigma, sh))
        return out.rgb, out.alpha, out.depth

    @staticmethod
    @once_differentiable
    def backward(ctx, g_rgb, g_alpha, g_depth):
        ras, st, scene_t, out = ctx.state
        if g_rgb is None and g_alpha is None and g_depth is None:
            return None, None, None, None, None, None, None
        dC = (g_rgb if g_rgb is not None else torch.zeros_like(out.rgb)).contiguous().float()
        dA = None if g_alpha is None else g_alpha.contiguous().float()
        dD = None if g_depth is None else g_depth.contiguous().float()
        # the library leaves the per-triangle accumulators zeroed after each
        # backward, so a retained graph can run this again
        gv, go, gs, gsh = ras.backward(st, scene_t, out, dC, dA, dD)
        return tuple(g.to(dt) for g, dt in zip((gv, go, gs, gsh), ctx.dtypes)) + (None, None, None)


def rasterize(v, o, sigma, sh, cam, cfg, capacity_hint=None):
    """Differentiable render of one view: (rgb [3,H,W], alpha [H,W], depth [H,W])."""
    return TriangleRasterize.apply(v, o, sigma, sh, cam, cfg, capacity_hint)
