"""Device buffers and the four-call pipeline for one view.

`ViewState` owns every buffer the C ABI needs for N triangles and one
camera (torch tensors are only storage); `Rasterizer` runs
ts_project -> ts_bin_sort -> ts_render_forward and ts_render_backward on the
current torch stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import torch

from . import binding as B


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


@dataclasses.dataclass
class Outputs:
    rgb: torch.Tensor      # [3,H,W]
    alpha: torch.Tensor    # [H,W]
    depth: torch.Tensor    # [H,W]
    T_final: torch.Tensor  # [H,W]
    last: torch.Tensor     # [H,W] int32 (uint32 bits)


class ViewState:
    """Projection state, tile lists and workspace of one view."""

    def __init__(self, N: int, width: int, height: int, capacity: int, device="cuda",
                 keys: bool = False):
        self.N, self.W, self.H = int(N), int(width), int(height)
        self.device = torch.device(device)
        self.num_tiles = B.ts_num_tiles(self.W, self.H)
        n = max(self.N, 1)
        rb = B.ts_proj_record_bytes()
        dev = self.device
        self.rec = torch.empty(n * rb, dtype=torch.uint8, device=dev)
        self.rect = torch.empty((n, 4), dtype=torch.int16, device=dev)
        self.depth_key = torch.empty(n, dtype=torch.float32, device=dev)
        self.ntiles = torch.empty(n, dtype=torch.int32, device=dev)
        # zero once; every backward consumes its accumulations and clears them
        self.g2d = torch.zeros((n, B.TS_G2D_STRIDE), dtype=torch.float32, device=dev)
        self.cgrad = torch.empty((n, B.TS_CGRAD_STRIDE), dtype=torch.float32, device=dev)
        self.ranges = torch.empty((self.num_tiles, 2), dtype=torch.int32, device=dev)
        self.order = torch.empty(max(self.num_tiles, 1), dtype=torch.int32, device=dev)
        self.d_count = torch.zeros(4, dtype=torch.int32, device=dev)
        self.want_keys = keys
        self.segmented = False   # tiles of more than 4096 instances seen: segmented sort
        self._alloc_lists(capacity)
        self.proj = B.ts_proj(self.rec.data_ptr(), self.rect.data_ptr(), self.depth_key.data_ptr(),
                              self.ntiles.data_ptr(), self.g2d.data_ptr(),
                              self.cgrad.data_ptr())
        self.count = (ctypes.c_uint32 * 2)()
        self.M = None
        self.N_v = None

    def _alloc_lists(self, capacity: int):
        self.capacity = int(max(capacity, 1))
        dev = self.device
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.keys = torch.empty(self.capacity, dtype=torch.int64, device=dev) if self.want_keys else None
        self.blocks = torch.empty(self.capacity, dtype=torch.int16, device=dev)
        self.ws_bytes = B.ts_bin_sort_workspace_bytes(self.N, self.capacity, self.num_tiles)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.bins = B.ts_bins(None if self.keys is None else self.keys.data_ptr(),
                              self.vals.data_ptr(), self.ranges.data_ptr(),
                              self.d_count.data_ptr(), self.capacity, self.order.data_ptr(),
                              self.blocks.data_ptr(),
                              B.TS_BINS_SEGMENTED_SORT if self.segmented else 0)

    def outputs(self) -> Outputs:
        dev, H, W = self.device, self.H, self.W
        return Outputs(torch.empty((3, H, W), dtype=torch.float32, device=dev),
                       torch.empty((H, W), dtype=torch.float32, device=dev),
                       torch.empty((H, W), dtype=torch.float32, device=dev),
                       torch.empty((H, W), dtype=torch.float32, device=dev),
                       torch.empty((H, W), dtype=torch.int32, device=dev))


class PruneStats:
    """Pruning statistics over the views rendered with them (Sec. 3.2,
    "Pruning"): per triangle the largest blending weight T*o and the number
    of views that rendered it with more than one pixel."""

    def __init__(self, N: int, device="cuda"):
        n = max(N, 1)
        self.max_weight = torch.zeros(n, dtype=torch.float32, device=device)
        self.pixels = torch.zeros(n, dtype=torch.int32, device=device)   # per view, cleared
        self.views = torch.zeros(n, dtype=torch.int32, device=device)
        self.c = B.ts_prune_stats(self.max_weight.data_ptr(), self.pixels.data_ptr())

    def prune_mask(self, tau_prune: float, min_views: int = 2):
        """Triangles to prune: largest weight below tau_prune, or rendered with
        more than one pixel in fewer than min_views views."""
        return (self.max_weight < tau_prune) | (self.views < min_views)


class Rasterizer:
    """Runs the four library calls for one camera."""

    def __init__(self, cfg, device="cuda"):
        self.cfg = cfg
        self.ccfg = B.make_config(cfg)
        self.device = torch.device(device)

    def project(self, st: ViewState, scene_t, cam):
        v, o, sigma, sh = scene_t
        ccam = B.make_camera(cam)
        B.ts_project(v, o, sigma, sh, st.N, ccam, self.ccfg, st.proj, _stream())
        return ccam

    def bin_sort(self, st: ViewState, ccam, sync: bool = True):
        """With sync, read back (M, N_v) and grow the lists until they fit."""
        while True:
            try:
                B.ts_bin_sort(st.proj, st.N, ccam, st.ws, st.ws_bytes, st.bins,
                              st.count if sync else None, _stream())
            except B.TSError as e:
                if e.code != B.TS_ECAPACITY:
                    raise
                st._alloc_lists(int(st.count[0] * 1.25) + 1024)
                continue
            break
        if sync:
            st.M, st.N_v = int(st.count[0]), int(st.count[1])
            # a view with tiles of more than 4096 instances: later calls on the
            # same state sort those tiles with the segmented sort
            if not st.segmented and int(st.d_count[3].item()) > 0:
                st.segmented = True
                st.bins.flags = B.TS_BINS_SEGMENTED_SORT

    def forward(self, st: ViewState, scene_t, cam, out: Optional[Outputs] = None,
                sync: bool = True, stats: Optional["PruneStats"] = None) -> Outputs:
        ccam = self.project(st, scene_t, cam)
        self.bin_sort(st, ccam, sync=sync)
        if out is None:
            out = st.outputs()
        if stats is None:
            B.ts_render_forward(st.proj, st.bins, ccam, self.ccfg, out.rgb, out.alpha, out.depth,
                                out.T_final, out.last, _stream())
        else:
            B.ts_render_forward_stats(st.proj, st.bins, ccam, self.ccfg, out.rgb, out.alpha,
                                      out.depth, out.T_final, out.last, stats.c, _stream())
            B.ts_prune_count_views(stats.pixels, stats.views, st.N, _stream())
        st.ccam = ccam
        return out

    def backward(self, st: ViewState, scene_t, out: Outputs, dC, dA=None, dD=None, grads=None):
        v, o, sigma, sh = scene_t
        if grads is None:
            grads = (torch.empty_like(v), torch.empty_like(o), torch.empty_like(sigma),
                     torch.empty_like(sh))
        gv, go, gs, gsh = grads
        B.ts_render_backward(v, o, sigma, sh, st.N, st.proj, st.bins, st.ccam, self.ccfg, dC, dA,
                             dD, out.T_final, out.last, gv, go, gs, gsh, _stream())
        return grads


class StoredFragments:
    """The stored-fragment variant of one view (kept to measure the memory
    the recompute backward saves): a counting forward, then a forward that
    keeps every composited fragment (tile-list entry, alpha, transmittance
    in front of it: 12 bytes each), and a backward that reads them."""

    def __init__(self, ras: "Rasterizer", st: ViewState):
        self.ras, self.st = ras, st
        dev, H, W = st.device, st.H, st.W
        self.count = torch.empty((H, W), dtype=torch.int32, device=dev)
        self.offset = torch.empty((H, W), dtype=torch.int32, device=dev)
        self.total = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_bytes = B.ts_fragment_workspace_bytes(W, H)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.entry = self.alpha = self.T = None
        self.F = 0

    def forward(self, scene_t, cam, out: Optional[Outputs] = None) -> Outputs:
        """Project, bin, count, size the fragment arrays (one host read of
        F), then the storing forward."""
        st, ras = self.st, self.ras
        ccam = ras.project(st, scene_t, cam)
        ras.bin_sort(st, ccam, sync=True)
        st.ccam = ccam
        if out is None:
            out = st.outputs()
        B.ts_render_forward_count(st.proj, st.bins, ccam, ras.ccfg, out.rgb, out.alpha, out.depth,
                                  out.T_final, out.last, self.count, self.offset, self.total,
                                  self.ws, self.ws_bytes, _stream())
        F = int(self.total.item())
        if self.entry is None or self.entry.numel() < max(F, 1):
            n = max(F, 1)
            self.entry = torch.empty(n, dtype=torch.int32, device=st.device)
            self.alpha = torch.empty(n, dtype=torch.float32, device=st.device)
            self.T = torch.empty(n, dtype=torch.float32, device=st.device)
        self.F = F
        B.ts_render_forward_store(st.proj, st.bins, ccam, ras.ccfg, out.rgb, out.alpha, out.depth,
                                  out.T_final, out.last, self.offset, self.entry, self.alpha,
                                  self.T, _stream())
        return out

    def backward(self, scene_t, out: Outputs, dC, dA=None, dD=None, grads=None):
        st, ras = self.st, self.ras
        v, o, sigma, sh = scene_t
        if grads is None:
            grads = (torch.empty_like(v), torch.empty_like(o), torch.empty_like(sigma),
                     torch.empty_like(sh))
        gv, go, gs, gsh = grads
        B.ts_raster_backward_stored(st.proj, st.bins, st.ccam, ras.ccfg, dC, dA, dD, out.T_final,
                                    out.last, self.count, self.offset, self.entry, self.alpha,
                                    self.T, _stream())
        B.ts_project_backward(v, sh, st.N, st.proj, st.ccam, ras.ccfg, gv, go, gs, gsh, _stream())
        return grads


def scene_to_device(scene, device="cuda"):
    """Float32 contiguous device copies (v, o, sigma, sh) of a synth.Scene."""
    return tuple(torch.as_tensor(a).to(device=device, dtype=torch.float32).contiguous()
                 for a in (scene.v, scene.o, scene.sigma, scene.sh))
