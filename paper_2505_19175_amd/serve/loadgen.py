"""Open-loop load generator: Poisson arrivals of camera requests with mixed
resolutions, driven in real time against a Scheduler + executor, with
latency percentiles and throughput over a measurement window."""
from __future__ import annotations

import math
import time
from typing import Callable, List, Optional

import numpy as np

from .. import synth
from .scheduler import Request, Scheduler, percentile


def poisson_requests(rate: float, duration: float, seed: int, sizes=synth.SERVE_SIZES) -> List[Request]:
    """Arrivals of a Poisson process of `rate` per second on [0, duration);
    each request a hemisphere pose (radius 5) and a resolution drawn
    uniformly from `sizes`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        eye = synth.hemisphere_eyes(rng, 1)[0]
        w, h = sizes[int(rng.integers(len(sizes)))]
        out.append(Request(len(out), synth.look_at(eye, width=w, height=h), t))
    return out


def drive(sched: Scheduler, requests: List[Request], clock: Callable[[], float],
          spin: Callable[[], None] = lambda: None, t0: float = None,
          stop_at: Optional[float] = None) -> None:
    """Feed requests at their arrival times (relative to t0) until every one
    has completed, or, with stop_at (relative to t0), until that time once
    every request has arrived: a server past saturation then leaves its
    backlog queued (those requests never complete), while the batches in
    flight are still collected."""
    if t0 is None:
        t0 = clock()
    for r in requests:
        r.arrival += t0
    i = 0
    while i < len(requests) or not sched.idle():
        now = clock()
        while i < len(requests) and requests[i].arrival <= now:
            sched.arrive(requests[i])
            i += 1
        if stop_at is not None and i == len(requests) and now >= t0 + stop_at:
            sched.queue.clear()
            if not sched.in_flight:
                break
        if not sched.step():
            spin()


def summarize(requests: List[Request], t0: float, warmup: float, duration: float) -> dict:
    """Over the requests that arrived in [warmup, duration): frames/s
    delivered, and latency percentiles with a request that never completed
    counted as infinitely late (p99 is then None once more than 1% are
    missing: the server did not keep up)."""
    win = [r for r in requests if warmup <= r.arrival - t0 < duration]
    if not win:
        return dict(n=0)
    done = [r for r in win if r.done is not None and not r.failed]
    lat = [r.latency * 1e3 for r in done] + [math.inf] * (len(win) - len(done))
    t_start = t0 + warmup
    t_end = max((r.done for r in done), default=t_start)
    span = max(t_end - t_start, duration - warmup)
    fin = lambda x: round(x, 3) if math.isfinite(x) else None
    return dict(n=len(win), completed=len(done), frames_per_s=round(len(done) / span, 2),
                p50_ms=fin(percentile(lat, 50)), p99_ms=fin(percentile(lat, 99)),
                mean_ms=fin(float(np.mean(lat))) if len(done) == len(win) else None)


def drop_frame(r: Request) -> None:
    """The load generator's consumer: takes the delivered frame and lets it go."""
    r.result = None


def run_load(make_scheduler: Callable[[Callable[[Request], None]], Scheduler], rate: float,
             duration: float, warmup: float, seed: int, drain: Optional[float] = None) -> dict:
    """make_scheduler(sink) -> Scheduler.  With drain, requests still queued
    `drain` seconds after the last arrival are abandoned (see drive)."""
    reqs = poisson_requests(rate, duration, seed)
    sched = make_scheduler(drop_frame)
    clock = time.perf_counter
    t0 = clock()
    drive(sched, reqs, clock, spin=lambda: time.sleep(0), t0=t0,
          stop_at=None if drain is None else duration + drain)
    s = summarize(reqs, t0, warmup, duration)
    s.update(rate=rate, batches=len(sched.batches), overflows=sched.overflows,
             mean_views_per_batch=round(float(np.mean([b["views"] for b in sched.batches])), 2)
             if sched.batches else 0.0)
    return s
