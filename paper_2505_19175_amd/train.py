"""One synthetic training step on the device (Sec. 3.3): render, the
photometric loss and its image gradient, the backward pass, then the opacity
and size losses and Adam on the raw parameters -- every step in the
library's kernels; torch only holds the buffers."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import binding as B
from .render import Outputs, Rasterizer, ViewState


# Learning rates (Supp. hyperparameter table, outdoor), Adam constants and
# loss weights; lambda weighs D-SSIM against L1.
DEFAULTS = dict(lr_v=0.0018, lr_opacity=0.014, lr_sigma=0.0008, lr_sh_dc=0.0025,
                lr_sh_rest=0.0025 / 20.0, beta1=0.9, beta2=0.999, eps=1e-15,
                beta_opacity=0.0055, beta_size=1e-8, lam=0.2)


class TrainState:
    """Raw parameters (v, a = logit o, b = log sigma, sh), the activated
    copies the renderer reads (o, sigma), gradients and Adam moments."""

    def __init__(self, scene, device="cuda", **opt):
        self.device = torch.device(device)
        self.N = int(scene.n)
        self.deg = int(round(np.sqrt(scene.sh.shape[1]))) - 1
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(self.device)
        o = np.asarray(scene.o, np.float64)
        s = np.asarray(scene.sigma, np.float64)
        self.v = f32(scene.v)
        self.sh = f32(scene.sh)
        self.a = f32(np.log(o) - np.log1p(-np.minimum(o, 1 - 1e-7)))
        self.b = f32(np.log(s))
        self.o = f32(o)
        self.sigma = f32(s)
        self.grads = tuple(torch.zeros_like(t) for t in (self.v, self.o, self.sigma, self.sh))
        self.moments = [torch.zeros_like(t) for t in (self.v, self.v, self.a, self.a, self.b,
                                                      self.b, self.sh, self.sh)]
        m = self.moments
        self.state = B.ts_adam_state(*(x.data_ptr() for x in m))
        cfg = dict(DEFAULTS)
        cfg.update(opt)
        self.lam = float(cfg.pop("lam"))
        self.opt = B.ts_optimizer(**{k: float(v) for k, v in cfg.items()}, step=0)
        self.t = 0
        self._loss_ws = None
        self.loss = torch.zeros(2, dtype=torch.float32, device=self.device)
        self.dC = None

    def scene_t(self):
        return (self.v, self.o, self.sigma, self.sh)

    def _ws(self, W, H):
        need = B.ts_image_loss_workspace_bytes(W, H)
        if self._loss_ws is None or self._loss_ws.numel() < need:
            self._loss_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.dC = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        return need

    def image_loss(self, rgb, target):
        H, W = rgb.shape[1], rgb.shape[2]
        need = self._ws(W, H)
        if self.dC.shape != (3, H, W):
            self.dC = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        B.ts_image_loss(rgb, target, W, H, self.lam, self.dC, self.loss, self._loss_ws, need,
                        torch.cuda.current_stream().cuda_stream)
        return self.dC

    def step(self, ras: Rasterizer, st: ViewState, cam, target, sync: bool = False,
             stats=None, fused: bool = True) -> Outputs:
        """forward -> image loss -> backward -> regularizers + Adam.  With
        stats (render.PruneStats) the forward also keeps the pruning
        statistics of the view.  fused: the backward projection applies Adam
        where each triangle's gradient is formed (no gradient arrays); else
        the gradients are written to self.grads and the optimizer reads them."""
        stream = torch.cuda.current_stream().cuda_stream
        out = ras.forward(st, self.scene_t(), cam, sync=sync, stats=stats)
        dC = self.image_loss(out.rgb, target)
        self.t += 1
        self.opt.step = self.t
        if fused:
            B.ts_raster_backward(st.proj, st.bins, st.ccam, ras.ccfg, dC, None, None, out.T_final,
                                 out.last, stream)
            B.ts_project_backward_adam(self.v, self.a, self.b, self.sh, self.o, self.sigma, self.N,
                                       st.proj, st.ccam, ras.ccfg, self.state, self.opt, stream)
            return out
        gv, go, gs, gsh = self.grads
        B.ts_render_backward(self.v, self.o, self.sigma, self.sh, self.N, st.proj, st.bins,
                             st.ccam, ras.ccfg, dC, None, None, out.T_final, out.last, gv, go, gs,
                             gsh, stream)
        B.ts_optimizer_step(self.v, self.a, self.b, self.sh, self.o, self.sigma, self.deg, self.N,
                            gv, go, gs, gsh, self.state, self.opt, stream)
        return out

    def loss_value(self) -> float:
        l1, ssim = (float(x) for x in self.loss.cpu())
        return (1 - self.lam) * l1 + self.lam * (1 - ssim)
