"""Continuous-batching scheduler of the forward-only render server.

Pure host logic (no GPU): a FIFO of camera requests, admission of requests
into a batch by the sort-buffer memory they are expected to need, a fixed
number of batches in flight, re-queueing of the requests of a batch whose
instance list overflowed.  The executor and the clock are injected, so the
same code runs the GPU server and the CPU tests (fake executor, mock clock).

Admission: a request of W x H pixels is expected to need
    est(W, H) = instances_per_pixel * W * H
instances; a batch takes requests in arrival order while the sum of the
estimates stays within `fill` of the executor's capacity, the views fit in
its slots and the tiles in its tile budget.  instances_per_pixel starts at a
prior and follows the largest ratio seen in completed batches (times a
safety margin), so an overflow is rare and is repaired by a retry.

Delivery: the executor writes each request's frame into memory the request
owns (`Request.result`) before the batch counts as complete, so a slot can
be refilled at once; `sink(request)` is called for every completed (or
failed) request inside step(), before any slot is refilled, and is where a
consumer takes the frame.
"""
from __future__ import annotations

import collections
import dataclasses
import math
from typing import Callable, List, Optional, Protocol

TILE = 16


def tiles_of(width: int, height: int) -> int:
    return ((width + TILE - 1) // TILE) * ((height + TILE - 1) // TILE)


@dataclasses.dataclass
class Request:
    rid: int
    camera: object            # synth.Camera
    arrival: float            # seconds, scheduler clock
    submitted: Optional[float] = None
    done: Optional[float] = None
    attempts: int = 0
    failed: bool = False       # too large for the sort buffer even alone
    result: object = None      # the delivered frame, set by the executor at submission and
                               # valid once `done` is set (memory the request owns)

    @property
    def pixels(self) -> int:
        return self.camera.width * self.camera.height

    @property
    def tiles(self) -> int:
        return tiles_of(self.camera.width, self.camera.height)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


@dataclasses.dataclass
class BatchResult:
    done: float                 # completion time (scheduler clock)
    instances: int              # instance count of the batch (may exceed capacity)
    overflow: bool


class Executor(Protocol):
    max_views: int
    max_tiles: int
    capacity: int               # instances per batch
    slots: int                  # batches in flight at once

    def submit(self, slot: int, batch: List[Request]) -> None: ...

    def poll(self, slot: int) -> Optional[BatchResult]: ...


class Scheduler:
    def __init__(self, executor: Executor, clock: Callable[[], float],
                 instances_per_pixel: float = 0.5, margin: float = 1.25, fill: float = 0.9,
                 sink: Optional[Callable[[Request], None]] = None):
        self.ex = executor
        self.sink = sink
        self.clock = clock
        self.ipp = instances_per_pixel
        self.margin = margin
        self.fill = fill
        self.queue: collections.deque = collections.deque()
        self.in_flight: dict = {}           # slot -> list[Request]
        self.completed: List[Request] = []
        self.failed: List[Request] = []
        self.batches: List[dict] = []
        self.overflows = 0

    # -- admission ---------------------------------------------------------
    def estimate(self, req: Request) -> int:
        return int(math.ceil(self.ipp * self.margin * req.pixels))

    def form_batch(self) -> List[Request]:
        batch, inst, tiles = [], 0, 0
        budget = self.fill * self.ex.capacity
        while self.queue and len(batch) < self.ex.max_views:
            r = self.queue[0]
            e = self.estimate(r)
            if batch and (inst + e > budget or tiles + r.tiles > self.ex.max_tiles):
                break
            if not batch and r.tiles > self.ex.max_tiles:
                raise ValueError(f"request {r.rid} has more tiles than a batch holds")
            batch.append(self.queue.popleft())
            inst += e
            tiles += r.tiles
        return batch

    # -- one iteration of the serving loop ----------------------------------
    def arrive(self, req: Request) -> None:
        self.queue.append(req)

    def step(self) -> bool:
        """Collect finished batches, then fill free slots.  Returns True if
        anything happened."""
        progressed = False
        for slot in list(self.in_flight):
            res = self.ex.poll(slot)
            if res is None:
                continue
            batch = self.in_flight.pop(slot)
            progressed = True
            px = sum(r.pixels for r in batch)
            self.batches.append(dict(views=len(batch), pixels=px, instances=res.instances,
                                     overflow=res.overflow, done=res.done))
            if px:
                self.ipp = max(self.ipp, res.instances / px)
            if res.overflow:
                self.overflows += 1
                if len(batch) == 1 and batch[0].attempts >= 2:
                    # alone and still too large for the sort buffer: give up
                    batch[0].failed = True
                    batch[0].done = res.done
                    batch[0].result = None
                    self.failed.append(batch[0])
                    if self.sink is not None:
                        self.sink(batch[0])
                    continue
                for r in reversed(batch):          # back to the front, in order
                    self.queue.appendleft(r)
                continue
            for r in batch:
                r.done = res.done
                self.completed.append(r)
                if self.sink is not None:
                    self.sink(r)
        for slot in range(self.ex.slots):
            if slot in self.in_flight or not self.queue:
                continue
            batch = self.form_batch()
            now = self.clock()
            for r in batch:
                r.submitted = now
                r.attempts += 1
            self.ex.submit(slot, batch)
            self.in_flight[slot] = batch
            progressed = True
        return progressed

    def idle(self) -> bool:
        return not self.queue and not self.in_flight


def percentile(xs, q):
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = (len(s) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    if s[lo] == s[hi] or not math.isfinite(s[hi]):
        return s[hi] if k > lo else s[lo]
    return s[lo] + (s[hi] - s[lo]) * (k - lo)
