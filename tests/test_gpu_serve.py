"""GPU tests of the serving path: the batched multi-view forward (HIP-graph
replays of ts_render_forward_batched) against single-view renders and the
oracle, the overflow flag, and a short continuous-batching load run."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2505_19175_amd import synth
from paper_2505_19175_amd.render import Rasterizer, ViewState, scene_to_device
from paper_2505_19175_amd.serve.executor import BatchedExecutor, PlainExecutor
from paper_2505_19175_amd.serve.loadgen import run_load
from paper_2505_19175_amd.serve.scheduler import Request, Scheduler

import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def soup():
    rng = np.random.Generator(np.random.PCG64(77))
    sc = synth.cluster_soup(77, 120_000, extent=3.0, std=0.4, edge_median=0.03, sh_degree=3,
                            rng=rng)
    cfg = synth.Config(sh_degree=3)
    return sc, cfg, scene_to_device(sc, "cuda:0")


def _cams(seed, sizes):
    rng = np.random.Generator(np.random.PCG64(seed))
    eyes = synth.hemisphere_eyes(rng, len(sizes))
    return [synth.look_at(e, width=w, height=h) for e, (w, h) in zip(eyes, sizes)]


def _alone(scene_t, cfg, cam):
    st = ViewState(scene_t[0].shape[0], cam.width, cam.height, 1 << 21)
    out = Rasterizer(cfg).forward(st, scene_t, cam, sync=True)
    torch.cuda.synchronize()
    return out.rgb.cpu().numpy(), out.alpha.cpu().numpy(), out.depth.cpu().numpy()


def _wait(ex, slot):
    while True:
        r = ex.poll(slot)
        if r is not None:
            return r


def test_batch_equals_alone_over_replays(soup):
    """Each view rendered inside mixed batches equals the same view rendered
    alone, bit for bit, over several graph replays with eager work between."""
    sc, cfg, st = soup
    cams = _cams(1, [(640, 360), (1280, 720), (320, 200), (1920, 1080), (641, 359)])
    ex = BatchedExecutor(st, cfg, time.perf_counter, max_views=4, max_tiles=4 * 8160,
                         max_pixels=4 * 1920 * 1080, capacity=1 << 21, slots=2)
    alone = [_alone(st, cfg, c) for c in cams]
    mixes = [[0, 1, 2], [3, 1], [4, 0, 2, 3], [1], [2, 4, 0]]
    for k, mix in enumerate(mixes):
        slot = k % 2
        batch = [Request(i, cams[i], 0.0) for i in mix]
        ex.submit(slot, batch)
        res = _wait(ex, slot)
        assert not res.overflow and res.instances > 0
        outs = ex.outputs(slot, batch)
        for i, (rgb, a, d) in zip(mix, outs):
            np.testing.assert_array_equal(rgb.cpu().numpy(), alone[i][0])
            np.testing.assert_array_equal(a.cpu().numpy(), alone[i][1])
            np.testing.assert_array_equal(d.cpu().numpy(), alone[i][2])
        _alone(st, cfg, cams[k % len(cams)])          # eager work between replays


def test_batch_matches_oracle_on_sampled_pixels(soup):
    sc, cfg, st = soup
    cams = _cams(2, [(640, 360), (960, 540)])
    ex = BatchedExecutor(st, cfg, time.perf_counter, max_views=2, max_tiles=2 * 2040,
                         max_pixels=2 * 960 * 540, capacity=1 << 21, slots=1)
    batch = [Request(i, c, 0.0) for i, c in enumerate(cams)]
    ex.submit(0, batch)
    _wait(ex, 0)
    for (rgb, a, d), cam in zip(ex.outputs(0, batch), cams):
        pix = synth.pixel_sample(9, cam.width, cam.height, 1500)
        ref = O.render(sc, cam, cfg, pix=pix)
        gpu = {"rgb": rgb.cpu().numpy().astype(np.float64), "alpha": a.cpu().numpy().astype(np.float64),
               "depth": d.cpu().numpy().astype(np.float64),
               "T_final": 1.0 - a.cpu().numpy().astype(np.float64)}
        G.assert_forward(gpu, ref, pix=pix)


def test_overflow_is_flagged(soup):
    sc, cfg, st = soup
    cams = _cams(3, [(1280, 720), (1280, 720)])
    ex = BatchedExecutor(st, cfg, time.perf_counter, max_views=2, max_tiles=2 * 3600,
                         max_pixels=2 * 1280 * 720, capacity=50_000, slots=1)
    ex.submit(0, [Request(i, c, 0.0) for i, c in enumerate(cams)])
    res = _wait(ex, 0)
    assert res.overflow and res.instances > 50_000


def test_short_load_run_completes(soup):
    sc, cfg, st = soup
    ex = BatchedExecutor(st, cfg, time.perf_counter, max_views=4, max_tiles=4 * 8160,
                         max_pixels=4 * 1920 * 1080, capacity=1 << 21, slots=2)
    s = run_load(lambda sink: Scheduler(ex, time.perf_counter, instances_per_pixel=0.3, sink=sink),
                 rate=300, duration=0.6, warmup=0.1, seed=4)
    assert s["n"] > 50 and s["overflows"] == 0 and np.isfinite(s["p99_ms"])
    px = PlainExecutor(st, cfg, time.perf_counter)
    s2 = run_load(lambda sink: Scheduler(px, time.perf_counter, sink=sink), rate=300,
                  duration=0.6, warmup=0.1, seed=4)
    assert s2["n"] == s["n"] and np.isfinite(s2["p99_ms"])
    print("batched", s, "plain", s2)


def test_host_copy_holds_the_images(soup):
    """With the host copy on, each request of a completed batch owns a pinned
    host copy of its colour image, equal bit for bit to the device image, for
    the batched and the plain executor."""
    sc, cfg, st = soup
    cams = _cams(5, [(640, 360), (320, 200), (1280, 720)])
    alone = [_alone(st, cfg, c) for c in cams]
    ex = BatchedExecutor(st, cfg, time.perf_counter, max_views=3, max_tiles=3 * 3600,
                         max_pixels=3 * 1280 * 720, capacity=1 << 21, slots=2, d2h=True)
    for k, mix in enumerate([[0, 1, 2], [2, 0], [1]]):
        slot = k % 2
        batch = [Request(i, cams[i], 0.0) for i in mix]
        ex.submit(slot, batch)
        _wait(ex, slot)
        for i, r in zip(mix, batch):
            host, a, d = r.result
            assert host.is_pinned() and a is None and d is None
            np.testing.assert_array_equal(host.numpy(), alone[i][0])
    px = PlainExecutor(st, cfg, time.perf_counter, d2h=True)
    r = Request(0, cams[1], 0.0)
    px.submit(0, [r])
    _wait(px, 0)
    np.testing.assert_array_equal(r.result[0].numpy(), alone[1][0])


@pytest.mark.parametrize("d2h", [False, True])
def test_continuous_batching_delivers_every_frame(soup, d2h):
    """Requests arriving while others are on the GPU: two slots in flight,
    slots refilled as soon as a batch completes.  Every request's delivered
    frame (taken by the consumer inside the scheduler step, after its slot
    may already hold the next batch) equals the same view rendered alone."""
    sc, cfg, st = soup
    sizes = [(640, 360), (1280, 720), (320, 200), (1920, 1080), (641, 359), (960, 540)] * 3
    cams = _cams(6, sizes)
    ex = BatchedExecutor(st, cfg, time.perf_counter, max_views=3, max_tiles=3 * 8160,
                         max_pixels=3 * 1920 * 1080, capacity=1 << 21, slots=2, d2h=d2h)
    got = {}

    def sink(r):
        rgb, a, d = r.result
        got[r.rid] = (rgb.cpu().numpy(), None if a is None else a.cpu().numpy(),
                      None if d is None else d.cpu().numpy())
        r.result = None

    sched = Scheduler(ex, time.perf_counter, instances_per_pixel=0.3, sink=sink)
    reqs = [Request(i, c, 0.0) for i, c in enumerate(cams)]
    # arrivals in three waves: the second and third come while batches run
    for r in reqs[:6]:
        sched.arrive(r)
    sched.step()
    for r in reqs[6:12]:
        sched.arrive(r)
    sched.step()
    for r in reqs[12:]:
        sched.arrive(r)
    while not sched.idle():
        sched.step()
    assert len(got) == len(reqs) and sched.overflows == 0
    assert max(b["views"] for b in sched.batches) > 1
    for i, c in enumerate(cams):
        ref = _alone(st, cfg, c)
        np.testing.assert_array_equal(got[i][0], ref[0])
        if not d2h:
            np.testing.assert_array_equal(got[i][1], ref[1])
            np.testing.assert_array_equal(got[i][2], ref[2])
