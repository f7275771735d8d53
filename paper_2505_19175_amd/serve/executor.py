"""GPU executors of the render server.

BatchedExecutor  -- `slots` independent buffer sets, each with its own HIP
                    stream and a HIP graph of one ts_render_forward_batched
                    call captured once; a batch is submitted by copying its
                    view descriptor (pinned host -> device) and replaying
                    the graph, so batches on different slots overlap.
PlainExecutor    -- the baseline: one view per launch on one stream, the
                    staged pipeline ts_project -> ts_bin_sort (host read of
                    the instance count) -> ts_render_forward, no graph.

Delivery: after the render, on the same stream, each request's frame is
copied out of the slot's buffers into memory the request owns
(`Request.result`): (rgb [3,H,W], alpha [H,W], depth [H,W]) device tensors,
or with d2h set the colour image alone in pinned host memory
([3,H,W], torch's caching host allocator).  A batch is complete once those
copies are, so the next batch on the slot can overwrite the slot's buffers
at once and latency includes handing the frame over.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional

import torch

from .. import binding as B
from ..render import ViewState
from .scheduler import BatchResult, Request

VIEW_BYTES = ctypes.sizeof(B.ts_view)


class _Slot:
    pass


def _deliver(rgb, alpha, depth, d2h: bool):
    """Copies of one view's outputs that the request owns, enqueued on the
    current stream (the one that rendered them)."""
    if d2h:
        host = torch.empty(rgb.shape, dtype=torch.float32, pin_memory=True)
        host.copy_(rgb, non_blocking=True)
        return (host, None, None)
    return (rgb.clone(), alpha.clone(), depth.clone())


class BatchedExecutor:
    def __init__(self, scene_t, cfg, clock, max_views: int = 8, max_tiles: int = 8 * 8160,
                 max_pixels: int = 8 * 1920 * 1080, capacity: int = 4 << 20, slots: int = 2,
                 use_graph: bool = True, device="cuda", d2h: bool = False):
        self.scene_t = scene_t
        self.N = int(scene_t[0].shape[0])
        self.cfg = B.make_config(cfg)
        self.clock = clock
        self.max_views, self.max_tiles, self.max_pixels = max_views, max_tiles, max_pixels
        self.capacity, self.slots = capacity, slots
        self.use_graph = use_graph
        self.d2h = d2h
        dev = torch.device(device)
        n = self.N * max_views
        self.ws_bytes = B.ts_batch_workspace_bytes(self.N, max_views, capacity, max_tiles)
        desc_bytes = max_views * VIEW_BYTES + 16
        self._slots = []
        for _ in range(slots):
            s = _Slot()
            s.rec = torch.empty(n * B.ts_proj_record_bytes(), dtype=torch.uint8, device=dev)
            s.rect = torch.empty((n, 4), dtype=torch.int16, device=dev)
            s.depth_key = torch.empty(n, dtype=torch.float32, device=dev)
            s.ntiles = torch.empty(n, dtype=torch.int32, device=dev)
            s.vals = torch.empty(capacity, dtype=torch.int32, device=dev)
            s.ranges = torch.empty((max_tiles, 2), dtype=torch.int32, device=dev)
            s.order = torch.empty(max_tiles, dtype=torch.int32, device=dev)
            s.d_count = torch.zeros(4, dtype=torch.int32, device=dev)
            s.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
            s.rgb = torch.empty(3 * max_pixels, dtype=torch.float32, device=dev)
            s.alpha = torch.empty(max_pixels, dtype=torch.float32, device=dev)
            s.depth = torch.empty(max_pixels, dtype=torch.float32, device=dev)
            s.desc_dev = torch.zeros(desc_bytes, dtype=torch.uint8, device=dev)
            s.desc_host = torch.zeros(desc_bytes, dtype=torch.uint8).pin_memory()
            s.count_host = torch.zeros(4, dtype=torch.int32).pin_memory()
            s.views = (B.ts_view * max_views)()
            s.proj = B.ts_proj(s.rec.data_ptr(), s.rect.data_ptr(), s.depth_key.data_ptr(),
                               s.ntiles.data_ptr(), None)
            s.bins = B.ts_bins(None, s.vals.data_ptr(), s.ranges.data_ptr(), s.d_count.data_ptr(),
                               capacity, s.order.data_ptr())
            s.stream = torch.cuda.Stream(device=dev)
            s.event = torch.cuda.Event()
            s.batch = None
            s.layout = None
            s.graph = None
            self._slots.append(s)
        for s in self._slots:
            self._prepare(s)

    # -- the batched call on a slot's buffers --------------------------------
    def _launch(self, s, stream: int):
        v, o, sg, sh = self.scene_t
        views_ptr = s.desc_dev.data_ptr()
        ctl_ptr = views_ptr + self.max_views * VIEW_BYTES
        B.ts_render_forward_batched(v, o, sg, sh, self.N, views_ptr, ctl_ptr, self.max_views,
                                    self.max_tiles, self.cfg, s.proj, s.bins, s.ws, self.ws_bytes,
                                    s.rgb, s.alpha, s.depth, stream)

    def _prepare(self, s):
        """One eager run (an empty batch), then capture the graph."""
        torch.cuda.synchronize()
        with torch.cuda.stream(s.stream):
            self._launch(s, s.stream.cuda_stream)
        torch.cuda.synchronize()
        if self.use_graph:
            s.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(s.graph, stream=s.stream):
                self._launch(s, torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()

    # -- executor protocol ----------------------------------------------------
    def layout(self, batch: List[Request], s=None):
        views = s.views if s is not None else (B.ts_view * self.max_views)()
        for i, r in enumerate(batch):
            views[i].cam = B.make_camera(r.camera)
        tiles, pixels = B.ts_batch_layout(views, len(batch))
        if len(batch) > self.max_views or tiles > self.max_tiles or pixels > self.max_pixels:
            raise ValueError("batch exceeds the executor's buffers")
        return views, tiles, pixels

    def submit(self, slot: int, batch: List[Request]) -> None:
        s = self._slots[slot]
        views, tiles, pixels = self.layout(batch, s)
        s.batch, s.layout = batch, (tiles, pixels)
        raw = bytes(views)[: len(batch) * VIEW_BYTES]
        hb = s.desc_host.numpy()
        hb[: len(raw)] = memoryview(raw)
        ctl = hb[self.max_views * VIEW_BYTES: self.max_views * VIEW_BYTES + 8].view("uint32")
        ctl[0], ctl[1] = len(batch), tiles
        with torch.cuda.stream(s.stream):
            s.desc_dev.copy_(s.desc_host, non_blocking=True)
            if s.graph is not None:
                s.graph.replay()
            else:
                self._launch(s, s.stream.cuda_stream)
            for i, r in enumerate(batch):
                po, W, H = int(views[i].pixel_offset), r.camera.width, r.camera.height
                r.result = _deliver(s.rgb[3 * po: 3 * po + 3 * W * H].view(3, H, W),
                                    s.alpha[po: po + W * H].view(H, W),
                                    s.depth[po: po + W * H].view(H, W), self.d2h)
            s.event.record(s.stream)
            s.count_host.copy_(s.d_count, non_blocking=True)

    def poll(self, slot: int) -> Optional[BatchResult]:
        s = self._slots[slot]
        if s.batch is None or not s.event.query():
            return None
        done = self.clock()
        s.stream.synchronize()            # the 16-byte count copy queued after the event
        c = s.count_host.numpy()
        res = BatchResult(done=done, instances=int(c[0]), overflow=bool(c[2]))
        s.batch = None
        return res

    def outputs(self, slot: int, batch: List[Request]):
        """Per-request (rgb [3,H,W], alpha, depth) views into the slot's
        buffers (valid until the slot's next submission)."""
        s = self._slots[slot]
        views, _, _ = self.layout(batch)
        out = []
        for i, r in enumerate(batch):
            po, W, H = int(views[i].pixel_offset), r.camera.width, r.camera.height
            out.append((s.rgb[3 * po: 3 * po + 3 * W * H].view(3, H, W),
                        s.alpha[po: po + W * H].view(H, W), s.depth[po: po + W * H].view(H, W)))
        return out


class PlainExecutor:
    """One view per launch, FIFO, one stream, no graph."""

    def __init__(self, scene_t, cfg, clock, capacity: int = 4 << 20, device="cuda",
                 d2h: bool = False):
        from ..render import Rasterizer
        self.scene_t = scene_t
        self.N = int(scene_t[0].shape[0])
        self.ras = Rasterizer(cfg, device=device)
        self.clock = clock
        self.capacity = capacity
        self.max_views, self.max_tiles, self.slots = 1, 1 << 30, 1
        self.states = {}
        self.outs = {}
        self.event = torch.cuda.Event()
        self.batch = None
        self.d2h = d2h

    def _state(self, W, H):
        key = (W, H)
        if key not in self.states:
            self.states[key] = ViewState(self.N, W, H, self.capacity)
            self.outs[key] = self.states[key].outputs()
        return self.states[key], self.outs[key]

    def submit(self, slot: int, batch: List[Request]) -> None:
        (r,) = batch
        st, out = self._state(r.camera.width, r.camera.height)
        self.ras.forward(st, self.scene_t, r.camera, out=out, sync=True)
        r.result = _deliver(out.rgb, out.alpha, out.depth, self.d2h)
        self.event.record()
        self.batch = batch
        self.last = (st, out)

    def poll(self, slot: int) -> Optional[BatchResult]:
        if self.batch is None or not self.event.query():
            return None
        self.batch = None
        st, _ = self.last
        return BatchResult(done=self.clock(), instances=st.M or 0, overflow=False)
