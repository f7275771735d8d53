"""Continuous-batching scheduler on the CPU: a fake executor with a
simulated service time and instance count, driven by a mock clock."""
import dataclasses

import numpy as np
import pytest

from paper_2505_19175_amd.serve.loadgen import drive, poisson_requests, summarize
from paper_2505_19175_amd.serve.scheduler import BatchResult, Request, Scheduler, tiles_of


class MockClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=20e-6):
        self.t += dt


class FakeExecutor:
    """Batch time = launch + per_pixel * pixels; instances = ipp * pixels."""

    def __init__(self, clock, slots=2, max_views=4, capacity=2_000_000, max_tiles=40000,
                 launch=300e-6, per_pixel=0.5e-9, ipp=0.3):
        self.clock, self.slots, self.max_views = clock, slots, max_views
        self.capacity, self.max_tiles = capacity, max_tiles
        self.launch, self.per_pixel, self.ipp = launch, per_pixel, ipp
        self.running = {}
        self.submitted = []
        self.busy_until = 0.0

    def submit(self, slot, batch):
        px = sum(r.pixels for r in batch)
        # one device: batches execute one after another
        start = max(self.clock(), self.busy_until)
        end = start + self.launch + self.per_pixel * px
        self.busy_until = end
        inst = int(self.ipp * px)
        self.running[slot] = (end, inst, inst > self.capacity)
        self.submitted.append((self.clock(), slot, [r.rid for r in batch], inst))

    def poll(self, slot):
        if slot not in self.running or self.clock() < self.running[slot][0]:
            return None
        end, inst, ovf = self.running.pop(slot)
        return BatchResult(done=self.clock(), instances=inst, overflow=ovf)


def _run(rate=2000, duration=1.0, **kw):
    clock = MockClock()
    ex = FakeExecutor(clock, **kw)
    sch = Scheduler(ex, clock, instances_per_pixel=kw.get("ipp", 0.3))
    reqs = poisson_requests(rate, duration, seed=3)
    drive(sch, reqs, clock, spin=clock.advance, t0=0.0)
    return clock, ex, sch, reqs


def test_every_request_completes_once_in_order():
    clock, ex, sch, reqs = _run()
    assert len(sch.completed) == len(reqs) > 1000
    assert sorted(r.rid for r in sch.completed) == list(range(len(reqs)))
    order = [rid for _, _, rids, _ in ex.submitted for rid in rids]
    assert order == sorted(order)                       # FIFO admission
    for r in reqs:
        assert r.done >= r.submitted >= r.arrival


def test_batches_respect_slots_views_tiles_and_memory():
    clock, ex, sch, reqs = _run(max_views=3, capacity=1_200_000)
    by_id = {r.rid: r for r in reqs}
    for _, slot, rids, inst in ex.submitted:
        assert 1 <= len(rids) <= 3 and 0 <= slot < 2
        est = sum(sch.estimate(by_id[i]) for i in rids)
        assert len(rids) == 1 or est <= 0.9 * 1_200_000 + 1
        assert sum(by_id[i].tiles for i in rids) <= ex.max_tiles
    assert max(len(r) for _, _, r, _ in ex.submitted) >= 2     # it does batch


def test_overflow_requeues_and_learns():
    """The prior under-estimates instances per pixel by 3x: batches
    overflow, their requests go back to the front, the estimate rises and
    everything completes."""
    from paper_2505_19175_amd import synth
    clock = MockClock()
    ex = FakeExecutor(clock, capacity=3_000_000, ipp=0.9)
    sch = Scheduler(ex, clock, instances_per_pixel=0.3, margin=1.0)
    cam = synth.look_at((5, -1, 0), width=1280, height=720)
    reqs = [Request(i, cam, 0.0) for i in range(8)]        # a burst of 720p requests
    reqs += poisson_requests(3000, 0.3, seed=4)
    for i, r in enumerate(reqs):
        r.rid = i
    drive(sch, reqs, clock, spin=clock.advance, t0=0.0)
    assert sch.overflows >= 1
    assert sch.ipp >= 0.9 - 1e-9
    assert len(sch.completed) == len(reqs) and not sch.failed
    assert all(r.attempts >= 1 for r in reqs)
    assert any(r.attempts >= 2 for r in reqs)


def test_request_larger_than_the_sort_buffer_fails_cleanly():
    clock = MockClock()
    ex = FakeExecutor(clock, capacity=100_000, ipp=0.9)
    sch = Scheduler(ex, clock, instances_per_pixel=0.9)
    reqs = poisson_requests(500, 0.05, seed=5)
    drive(sch, reqs, clock, spin=clock.advance, t0=0.0)
    assert len(sch.failed) == len(reqs) and not sch.completed
    assert all(r.failed and r.attempts == 2 for r in reqs)


def test_continuous_batching_overlaps_slots():
    """A request that arrives while one batch is running is submitted on the
    second slot before the first batch finishes."""
    clock = MockClock()
    ex = FakeExecutor(clock, launch=5e-3)
    sch = Scheduler(ex, clock)
    from paper_2505_19175_amd import synth
    cam = synth.look_at((5, -1, 0), width=640, height=360)
    a, b = Request(0, cam, 0.0), Request(1, cam, 1e-3)
    drive(sch, [a, b], clock, spin=clock.advance, t0=0.0)
    (t_a, slot_a, _, _), (t_b, slot_b, _, _) = ex.submitted
    assert slot_a != slot_b and t_b < a.done


def test_batching_beats_one_view_per_launch_at_saturation():
    """With a fixed per-launch cost, batching serves more frames per second
    than one view per launch under the same overload."""
    c1, e1, s1, r1 = _run(rate=4000, duration=0.5, max_views=8, launch=1e-3)
    c2, e2, s2, r2 = _run(rate=4000, duration=0.5, max_views=1, slots=1, launch=1e-3)
    f1 = summarize(r1, 0.0, 0.1, 0.5)["frames_per_s"]
    f2 = summarize(r2, 0.0, 0.1, 0.5)["frames_per_s"]
    assert f1 > 1.5 * f2


def test_tiles_of():
    assert tiles_of(1920, 1080) == 120 * 68
    assert tiles_of(640, 360) == 40 * 23
