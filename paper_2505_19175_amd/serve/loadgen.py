"""Open-loop load generator: Poisson arrivals of camera requests with mixed
resolutions, driven in real time against a Scheduler + executor, with
latency percentiles and throughput over a measurement window."""
from __future__ import annotations

import time
from typing import Callable, List

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
          spin: Callable[[], None] = lambda: None, t0: float = None) -> None:
    """Feed requests at their arrival times (relative to t0) until every one
    has completed."""
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
        if not sched.step():
            spin()


def summarize(requests: List[Request], t0: float, warmup: float, duration: float) -> dict:
    win = [r for r in requests if warmup <= r.arrival - t0 < duration]
    lat = [r.latency * 1e3 for r in win if r.latency is not None]
    if not win:
        return dict(n=0)
    t_start = t0 + warmup
    t_end = max(r.done for r in win)
    span = max(t_end - t_start, duration - warmup)
    return dict(n=len(win), frames_per_s=round(len(win) / span, 2),
                p50_ms=round(percentile(lat, 50), 3), p99_ms=round(percentile(lat, 99), 3),
                mean_ms=round(float(np.mean(lat)), 3))


def run_load(make_scheduler: Callable[[], Scheduler], rate: float, duration: float, warmup: float,
             seed: int) -> dict:
    reqs = poisson_requests(rate, duration, seed)
    sched = make_scheduler()
    clock = time.perf_counter
    t0 = clock()
    drive(sched, reqs, clock, spin=lambda: time.sleep(0), t0=t0)
    s = summarize(reqs, t0, warmup, duration)
    s.update(rate=rate, batches=len(sched.batches), overflows=sched.overflows,
             mean_views_per_batch=round(float(np.mean([b["views"] for b in sched.batches])), 2)
             if sched.batches else 0.0)
    return s
