#!/usr/bin/env python
"""Benchmark of the triangle-splatting hot path on one MI355X.

One step = ts_project -> ts_bin_sort -> ts_render_forward ->
ts_raster_backward -> ts_project_backward on one view of the 3M-triangle
workload (SH degree 3, 70% dense clusters + 30% background shell,
1280x720 from the first hemisphere pose), inputs and the upstream image
gradient resident in HBM.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--view 0|1] [--no-cpu-baseline]
                  [--no-serve] [--no-other-view] [--no-prune-stats] [--no-windows]
                  [--no-densify] [--no-train]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpixel/s @3M tris 1280×720; serve frames/s + p50/p99 ms vs plain"
HBM_PEAK_GBS = 8000.0
P_REC = 48      # minimum raster record: 2D vertices, o, sigma, rgb, z (bytes)
G_REC = 48      # 2D gradient record (bytes)


# HBM traffic of one launch of a kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of `bench.py --steps 2 --warmup 1 --no-cpu-baseline
# --no-serve --no-other-view --no-windows --no-prune-stats` (KiB per dispatch
# of the benchmarked step's launches), each scaled by what the same counter reads
# for a 512 MiB device copy (`bench.py --copy-probe`: FETCH_SIZE reads half
# the copied bytes, WRITE_SIZE all of them).  Valid only for the kernel
# source the counters were taken on: `src` is the SHA-256 of its files.
TRAFFIC = {
    "project_bwd": {"files": ["paper_2505_19175_amd/csrc/backproject.hip",
                              "paper_2505_19175_amd/csrc/geometry.h",
                              "paper_2505_19175_amd/csrc/ts_device.h"],
                    "src": "2f75c1b29f27ca26ded13886dbdef84017ac581d79288b4e0be0c2219d11aea2",
                    "fetch_kib": 1.615e5, "write_kib": 7.807e5,
                    "fetch_scale": 2.0, "write_scale": 1.0},
    "project": {"files": ["paper_2505_19175_amd/csrc/project.hip",
                          "paper_2505_19175_amd/csrc/geometry.h",
                          "paper_2505_19175_amd/csrc/ts_device.h"],
                "src": "ff00d4a2a94574088ef47d699290f7606ccaf8e6ec59cef61445af4cc2573524",
                "fetch_kib": 2.148e5, "write_kib": 3.104e5,
                "fetch_scale": 2.0, "write_scale": 1.0},
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _sha(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(os.path.join(ROOT, path), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes(kernel):
    t = TRAFFIC.get(kernel)
    if t is None or t["src"] is None or _sha(t["files"]) != t["src"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def algorithmic_bytes(N, N_v, M, W, H, K, n_upstream=1):
    """Bytes each stage must move at minimum (radix passes beyond one,
    re-reads and atomic retries excluded)."""
    sh = 12 * K
    return {
        "project": 44 * N + sh * N_v + P_REC * N_v,
        "bin_sort": 36 * M,
        "raster_fwd": P_REC * N_v + 4 * M + 28 * W * H,
        "raster_bwd": 12 * n_upstream * W * H + 8 * W * H + 4 * M + P_REC * N_v + 2 * G_REC * N_v,
        "project_bwd": (44 + sh) * N_v + G_REC * N_v + (44 + sh) * N,
    }


def cpu_baseline(wl, cam, n_pix, seed=2024):
    """The oracle (FP64 brute force over all triangles, all host threads)
    forward + backward on a seeded sample of n_pix pixels of the view, or on
    the whole frame when n_pix is None; Mpixel/s and the time it would take
    for the whole frame (extrapolated linearly from a sample)."""
    import numpy as np

    from oracle import oracle as O
    from paper_2505_19175_amd import synth
    W, H = cam.width, cam.height
    dC, _, _ = synth.upstream(seed + 1, W, H)
    t0 = time.perf_counter()
    if n_pix is None or n_pix >= W * H:
        n = W * H
        ref = O.render(wl.scene, cam, wl.config)
        O.backward(wl.scene, cam, wl.config, dC)
        what = f"the whole {W}x{H} frame"
    else:
        n = n_pix
        pix = synth.pixel_sample(seed, W, H, n_pix)
        ref = O.render(wl.scene, cam, wl.config, pix=pix)
        O.backward(wl.scene, cam, wl.config, dC.reshape(3, -1)[:, pix], pix=pix)
        what = f"{n_pix} seeded pixels of the view"
    dt = time.perf_counter() - t0
    res = {"value": round(n / dt / 1e6, 7), "unit": "Mpixel/s", "cores": O.threads(),
           "kind": "oracle",
           "sample": f"{what}, forward + backward (FP64 brute force over all "
                     f"{wl.scene.n} triangles), {dt:.1f} s measured",
           "ms_per_frame": round(dt * 1e3 * W * H / n, 1),
           "frame_time": "measured" if n == W * H else "extrapolated linearly from the sample"}
    return res, float(np.mean(ref["nfrag"]))


def cpu_rows(wl, cam, cfg_windows, img, soup_slice=300_000, seed=2025):
    """The oracle beside each path beyond the step, on bounded samples of the
    same workload (about 20 s of host time in all): the statistics and the
    two windows on seeded pixel samples, the image loss on the whole frame,
    Adam on a slice of the soup, densification on the whole soup."""
    import numpy as np

    from oracle import densify as OD
    from oracle import oracle as O
    from oracle import train as OT
    from paper_2505_19175_amd import synth
    out = {}
    cores = O.threads()
    pix = synth.pixel_sample(seed, cam.width, cam.height, 256)
    t0 = time.perf_counter()
    O.prune_stats(wl.scene, cam, wl.config, pix=pix)
    dt = time.perf_counter() - t0
    out["prune_stats"] = {"value": round(256 / dt / 1e6, 6), "unit": "Mpixel/s", "cores": cores,
                          "kind": "oracle", "sample": f"256 seeded pixels, {dt:.1f} s"}
    dC, _, _ = synth.upstream(seed + 1, cam.width, cam.height)
    for name, cfg_w in cfg_windows.items():
        pw = pix[:128]
        t0 = time.perf_counter()
        O.render(wl.scene, cam, cfg_w, pix=pw)
        O.backward(wl.scene, cam, cfg_w, dC.reshape(3, -1)[:, pw], pix=pw)
        dt = time.perf_counter() - t0
        out[f"window_{name}"] = {"value": round(128 / dt / 1e6, 6), "unit": "Mpixel/s",
                                 "cores": cores, "kind": "oracle",
                                 "sample": f"128 seeded pixels, forward + backward, {dt:.1f} s"}
    rng = np.random.default_rng(seed)
    tgt = np.clip(img + rng.normal(0, 0.05, img.shape), 0, 1)
    t0 = time.perf_counter()
    OT.image_loss_grad(img, tgt)
    dt = time.perf_counter() - t0
    out["image_loss"] = {"value": round(dt * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                         "sample": f"the whole {cam.width}x{cam.height} frame"}
    n = min(soup_slice, wl.scene.n)
    sc = wl.scene
    raw = {"v": sc.v[:n].astype(np.float64), "a": np.log(sc.o[:n] / (1 - sc.o[:n] + 1e-7)),
           "b": np.log(sc.sigma[:n]), "sh": sc.sh[:n].astype(np.float64)}
    grads = {"v": rng.normal(0, 1e-3, raw["v"].shape), "o": rng.normal(0, 1e-3, n),
             "sigma": rng.normal(0, 1e-3, n), "sh": rng.normal(0, 1e-3, raw["sh"].shape)}
    state = {k: (np.zeros(np.shape(raw[k])), np.zeros(np.shape(raw[k]))) for k in raw}
    t0 = time.perf_counter()
    OT.optimizer_step(raw, grads, state, 1)
    dt = time.perf_counter() - t0
    out["optimizer"] = {"value": round(dt * 1e3 * sc.n / n, 1), "unit": "ms", "cores": 1,
                        "kind": "oracle",
                        "sample": f"{n} triangles in {dt:.2f} s, scaled to {sc.n}"}
    u = rng.random(sc.n).astype(np.float32)
    t0 = time.perf_counter()
    sel = OD.select(sc.o, sc.sigma, OD.INV_SIGMA, 0.1 * sc.n, u)
    OD.subdivide(sc.v, sc.o, sc.sigma, sc.sh, sel)
    dt = time.perf_counter() - t0
    out["densify"] = {"value": round(dt * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                      "sample": f"the whole {sc.n}-triangle soup, select + subdivide"}
    return out


def serve_bench(rates, duration, warmup, d2h_rates, d2h_duration, seed=5,
                budgets_ms=(2.0, 10.0), drain=1.0):
    """Forward-only serving of the resident 1M-triangle SH-3 soup: Poisson
    requests with resolutions from {640x360, 1280x720, 1920x1080} and
    hemisphere poses, batched server (HIP-graph replays, two batches in
    flight, admission by sort-buffer memory) vs one view per launch.  Each
    request's frame is copied into memory it owns before it counts as done
    (device tensors; with the host copy, pinned host memory).  Past
    saturation the backlog left `drain` seconds after the last arrival is
    abandoned and counted as never delivered."""
    import torch

    from paper_2505_19175_amd import synth
    from paper_2505_19175_amd.render import scene_to_device
    from paper_2505_19175_amd.serve.executor import BatchedExecutor, PlainExecutor
    from paper_2505_19175_amd.serve.loadgen import run_load
    from paper_2505_19175_amd.serve.scheduler import Scheduler

    wl = synth.workload_serve()
    scene_t = scene_to_device(wl.scene, "cuda:0")
    clock = time.perf_counter
    def executors(d2h):
        return (BatchedExecutor(scene_t, wl.config, clock, max_views=8, max_tiles=8 * 8160,
                                max_pixels=8 * 1920 * 1080, capacity=4 << 20, slots=2, d2h=d2h),
                PlainExecutor(scene_t, wl.config, clock, capacity=4 << 20, d2h=d2h))

    out = {"workload": "serve1M: resident 1M-triangle SH-3 cluster soup",
           "window_s": duration - warmup, "warmup_s": warmup,
           "window_s_d2h": d2h_duration - warmup, "rates": {},
           "latency_note": "arrival to the device event after the frame's copy into memory the "
                           "request owns (device tensors); the *_d2h entries copy the colour "
                           "image into pinned host memory instead; p99 null: more than 1% of "
                           "the window's requests were never delivered (server saturated)"}
    for d2h in (False, True):
        batched, plain = executors(d2h)
        sfx = "_d2h" if d2h else ""
        rr, dur = (d2h_rates, d2h_duration) if d2h else (rates, duration)
        for rate in rr:
            log(f"[bench] serving at {rate} req/s{' with the host copy' if d2h else ''}")
            b = run_load(lambda sink: Scheduler(batched, clock, instances_per_pixel=0.3,
                                                sink=sink), rate, dur, warmup, seed, drain)
            torch.cuda.synchronize()
            p = run_load(lambda sink: Scheduler(plain, clock, sink=sink), rate, dur, warmup, seed,
                         drain)
            torch.cuda.synchronize()
            out["rates"].setdefault(str(rate), {}).update({"batched" + sfx: b, "plain" + sfx: p})
        del batched, plain
        torch.cuda.empty_cache()

        def best_within(budget, sysname):
            ok = [out["rates"][str(r)][sysname + sfx] for r in rr
                  if out["rates"][str(r)][sysname + sfx]["p99_ms"] is not None
                  and out["rates"][str(r)][sysname + sfx]["p99_ms"] <= budget]
            return max((x["frames_per_s"] for x in ok), default=0.0)

        # frames/s each system delivers at the highest offered rate where its
        # p99 stays within a fixed interactive budget
        at = {}
        for budget in budgets_ms:
            fb, fp = best_within(budget, "batched"), best_within(budget, "plain")
            at[f"{budget:g}ms"] = {"frames_per_s": {"batched": fb, "plain": fp},
                                   "speedup": round(fb / fp, 3) if fp else None}
        out["at_p99_budget" + sfx] = at
        # the survey's equal-p99 comparison: the plain renderer's p99 at the
        # highest load it still serves is the budget
        plain_p99 = [out["rates"][str(r)]["plain" + sfx]["p99_ms"] for r in rr]
        finite = [x for x in plain_p99 if x is not None]
        if finite:
            budget = max(finite)
            fb, fp = best_within(budget, "batched"), best_within(budget, "plain")
            out["equal_p99" + sfx] = {"p99_budget_ms": budget,
                                      "frames_per_s": {"batched": fb, "plain": fp},
                                      "speedup": round(fb / fp, 3) if fp else None}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--view", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=2048,
                    help="oracle sample of the 3M-triangle view (about 30 s on 16 threads)")
    ap.add_argument("--cpu-pixels-mid", type=int, default=4096,
                    help="oracle sample of the 300k-triangle view")
    ap.add_argument("--no-memory", action="store_true",
                    help="skip the recompute vs stored-fragment memory comparison")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1k, 20k and 300k-triangle workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 512 MiB device to device (scale for HBM counters)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-other-view", action="store_true",
                    help="skip the second 3M-triangle view (1600x1040 for pose 0)")
    ap.add_argument("--no-cpu-rows", action="store_true",
                    help="skip timing the oracle beside the paths beyond the step")
    ap.add_argument("--no-train", action="store_true",
                    help="skip timing the synthetic training step")
    ap.add_argument("--no-densify", action="store_true",
                    help="skip timing the densification kernels")
    ap.add_argument("--no-windows", action="store_true",
                    help="skip timing the sigmoid and LogSumExp windows")
    ap.add_argument("--no-prune-stats", action="store_true",
                    help="skip timing the forward that keeps the pruning statistics")
    ap.add_argument("--serve-rates", default="200,500,1000,2000,3000,4000,6000,8000",
                    help="req/s; the quoted 200-2000 and rates up to past saturation")
    ap.add_argument("--serve-seconds", type=float, default=11.0,
                    help="load duration per rate, the first --serve-warmup s not measured")
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--serve-d2h-rates", default="500,2000,4000",
                    help="req/s of the runs that also copy each frame to pinned host memory")
    ap.add_argument("--serve-d2h-seconds", type=float, default=3.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the renderer runs on exactly one GPU: --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2505_19175_amd import binding as B
    from paper_2505_19175_amd import synth
    from paper_2505_19175_amd.render import Rasterizer, ViewState, scene_to_device

    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 4}))
        return
    t0 = time.perf_counter()
    wl = synth.workload_large()
    cam = wl.cameras[args.view]
    cfg = wl.config
    K = (cfg.sh_degree + 1) ** 2
    log(f"[bench] generated {wl.scene.n} triangles in {time.perf_counter() - t0:.1f}s")
    scene_t = scene_to_device(wl.scene, dev)
    W, H, N = cam.width, cam.height, wl.scene.n

    ccfg = B.make_config(cfg)
    v, o, sg, sh = scene_t
    gv_, go_, gs_, gsh_ = (torch.empty_like(t) for t in scene_t)
    stream = torch.cuda.current_stream()
    sh_ = stream.cuda_stream
    ras = Rasterizer(cfg, device=dev)

    def prepare(view_cam, rasv=ras, scn=None, seed_up=None):
        """Buffers of one view; the instance list is sized once with a host
        read-back, then every step runs without one."""
        scn = scene_t if scn is None else scn
        Nv_ = int(scn[0].shape[0])
        Wv, Hv = view_cam.width, view_cam.height
        stv = ViewState(Nv_, Wv, Hv, max(4 * Nv_, 1 << 16), device=dev)
        outv = rasv.forward(stv, scn, view_cam, sync=True)
        stv._alloc_lists(int(stv.M * 1.05) + 4096)
        up, _, _ = synth.upstream(wl.upstream_seed if seed_up is None else seed_up, Wv, Hv)
        return stv, outv, B.make_camera(view_cam), torch.tensor(up, device=dev)

    def make_step(stv, outv, ccam, dCv, ccfg=ccfg, scn=None, grads=None):
        v, o, sg, sh = scene_t if scn is None else scn
        gv, go, gs, gsh = (gv_, go_, gs_, gsh_) if grads is None else grads
        N = int(v.shape[0])

        def step(ev=None):
            if ev: ev[0].record(stream)
            B.ts_project(v, o, sg, sh, N, ccam, ccfg, stv.proj, sh_)
            if ev: ev[1].record(stream)
            B.ts_bin_sort(stv.proj, N, ccam, stv.ws, stv.ws_bytes, stv.bins, None, sh_)
            if ev: ev[2].record(stream)
            B.ts_render_forward(stv.proj, stv.bins, ccam, ccfg, outv.rgb, outv.alpha, outv.depth,
                                outv.T_final, outv.last, sh_)
            if ev: ev[3].record(stream)
            # ts_render_backward as its two halves, so each gets its own events
            B.ts_raster_backward(stv.proj, stv.bins, ccam, ccfg, dCv, None, None, outv.T_final,
                                 outv.last, sh_)
            if ev: ev[4].record(stream)
            B.ts_project_backward(v, sh, N, stv.proj, ccam, ccfg, gv, go, gs, gsh, sh_)
            if ev: ev[5].record(stream)
        return step

    def timed(step, steps, warmup, stv):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        assert int(stv.d_count[2].item()) == 0, "instance list overflow"
        # timed region: exactly `steps` steps, events only around them (events
        # between the stages cost ~20 us a step, so they get a pass of their own)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        for k in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        gpu_total_ms = float(e0.elapsed_time(e1))
        # per-stage breakdown: the same steps again with events between the stages
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        per = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(5)]
                        for k in range(steps)])               # ms
        return max(gpu_total_ms, wall * 1e3) / steps, per

    def memory_forms(capacity, reps=10):
        """Device memory of one forward + backward of the view in the two
        forms: the recompute backward (8 B per pixel kept: T_final, last) and
        the stored-fragment one (per pixel a count and an offset, per
        composited fragment 12 B: entry, alpha, T).  Each form runs on fresh
        buffers after the allocator's peak is reset; the scene and its
        gradient arrays stay resident in both.  Also the backward's time."""
        from paper_2505_19175_amd.render import StoredFragments
        outm = {}
        for form in ("recompute", "stored_fragments"):
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats(dev)
            base = int(torch.cuda.memory_allocated(dev))
            stm = ViewState(N, W, H, capacity, device=dev)
            dCm = torch.tensor(synth.upstream(wl.upstream_seed, W, H)[0], device=dev)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
            if form == "recompute":
                outf = ras.forward(stm, scene_t, cam, sync=True)
                for r in range(reps):
                    ev[2 * r].record(stream)
                    B.ts_raster_backward(stm.proj, stm.bins, stm.ccam, ccfg, dCm, None, None,
                                         outf.T_final, outf.last, sh_)
                    ev[2 * r + 1].record(stream)
                    B.ts_project_backward(v, sh, N, stm.proj, stm.ccam, ccfg, gv_, go_, gs_, gsh_,
                                          sh_)
                kept = 8 * W * H
            else:
                sfm = StoredFragments(ras, stm)
                outf = sfm.forward(scene_t, cam)
                for r in range(reps):
                    ev[2 * r].record(stream)
                    B.ts_raster_backward_stored(stm.proj, stm.bins, stm.ccam, ccfg, dCm, None, None,
                                                outf.T_final, outf.last, sfm.count, sfm.offset,
                                                sfm.entry, sfm.alpha, sfm.T, sh_)
                    ev[2 * r + 1].record(stream)
                    B.ts_project_backward(v, sh, N, stm.proj, stm.ccam, ccfg, gv_, go_, gs_, gsh_,
                                          sh_)
                kept = 8 * W * H + 12 * sfm.F
                outm["fragments"] = sfm.F
            torch.cuda.synchronize()
            peak = int(torch.cuda.max_memory_allocated(dev))
            outm[form] = {"device_peak_bytes": peak, "working_bytes": peak - base,
                          "kept_for_backward_bytes": kept,
                          "raster_backward_ms": round(float(np.mean(
                              [ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps)])), 4)}
            del stm, dCm, outf
            if form != "recompute":
                del sfm
        torch.cuda.empty_cache()
        outm["memory_note"] = ("device peak over one forward + backward of the view on fresh "
                               "buffers (torch.cuda.max_memory_allocated); working_bytes = peak "
                               "minus the resident scene and gradient arrays; the stored form "
                               "runs a counting forward, then a forward that keeps the fragments")
        return outm

    stages = ["project", "bin_sort", "raster_fwd", "raster_bwd", "project_bwd"]
    torch.cuda.reset_peak_memory_stats(dev)
    st, out, ccam, dC = prepare(cam)
    M, N_v = st.M, st.N_v
    log(f"[bench] N={N} N_v={N_v} M={M} {W}x{H}")
    ms_per_step, per = timed(make_step(st, out, ccam, dC), args.steps, args.warmup, st)
    peak_bytes = int(torch.cuda.max_memory_allocated(dev))
    stage_ms = {s: round(float(per[:, j].mean()), 4) for j, s in enumerate(stages)}

    byt = algorithmic_bytes(N, N_v, M, W, H, K)
    # every stage but the binning is one kernel launch
    single_kernel = ["project", "raster_fwd", "raster_bwd", "project_bwd"]
    dom = max(single_kernel, key=lambda s: stage_ms[s])
    ach = byt[dom] / (stage_ms[dom] * 1e-3) / 1e9
    tr = traffic_bytes(dom)
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
            "traffic": None if tr is None else round(tr),
            "timing": "mean over the timed steps of HIP events recorded on the launch stream "
                      "right before and after the kernel's library call (a second pass of the "
                      "same steps)"}
    total_bytes = sum(byt.values())
    step_gbs = total_bytes / (ms_per_step * 1e-3) / 1e9
    # the whole step against the same peak (all five stages, host-clocked)
    roof["step_frac"] = round(step_gbs / HBM_PEAK_GBS, 5)
    copy_gbs = copy_bandwidth(torch, dev)
    res = {
        "metric": METRIC,
        "value": round(W * H / (ms_per_step * 1e-3) / 1e6, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"tri3M_{W}x{H}: 3M triangles, SH degree 3, 70% in 64 dense "
                               f"clusters + 30% on a radius-20 shell, hemisphere pose {args.view}",
                   "N": N, "N_visible": N_v, "instances": M, "width": W, "height": H},
        "triangles_per_s": round(N / (ms_per_step * 1e-3), 1),
        "stage_ms": stage_ms,
        "stage_GBps_algorithmic": {s: round(byt[s] / (stage_ms[s] * 1e-3) / 1e9, 1) for s in stages},
        "step_hbm_frac": round(step_gbs / HBM_PEAK_GBS, 5),
        "copy_GBps": round(copy_gbs, 1),
        "step_copy_frac": round(step_gbs / copy_gbs, 5),
        "roofline": roof,
        "memory": {"device_peak_bytes": peak_bytes,
                   "backward_state_bytes": 8 * W * H,
                   "note": "device peak over the timed steps of this view (scene, gradients, "
                           "projection state, lists, images); the backward keeps 8 B per pixel "
                           "(T_final, last) and no per-fragment state"},
    }
    if not args.no_memory:
        res["memory"].update(memory_forms(st.capacity))
    if not args.no_configs:
        # the other workloads of the measurement plan: 1k triangles at 128x128,
        # 20k at 256x256 (sigma = 1), 300k at 1280x720, each with the oracle
        # timed beside it (whole frame for the two small ones, a pixel sample
        # of the 300k view)
        res["configs"] = {}
        for wname, mk, cpu_pix in (("tri1k_128x128", synth.workload_small, None),
                                   ("tri20k_256x256", lambda: synth.workload_grad(1.0), None),
                                   ("tri300k_1280x720", synth.workload_mid, args.cpu_pixels_mid)):
            wlc = mk()
            camc, cfgc = wlc.cameras[0], wlc.config
            scn = scene_to_device(wlc.scene, dev)
            grads = tuple(torch.empty_like(t) for t in scn)
            ccfg_c = B.make_config(cfgc)
            stc, outc, ccam_c, dCc = prepare(camc, Rasterizer(cfgc, device=dev), scn,
                                             wlc.upstream_seed)
            msc, perc = timed(make_step(stc, outc, ccam_c, dCc, ccfg_c, scn, grads),
                                 args.steps, args.warmup, stc)
            Kc = (cfgc.sh_degree + 1) ** 2
            Wc, Hc, Nc = camc.width, camc.height, wlc.scene.n
            bc = algorithmic_bytes(Nc, stc.N_v, stc.M, Wc, Hc, Kc)
            entry = {"ms_per_step": round(msc, 4),
                     "Mpixel_per_s": round(Wc * Hc / (msc * 1e-3) / 1e6, 3),
                     "triangles_per_s": round(Nc / (msc * 1e-3), 1),
                     "N": Nc, "N_visible": stc.N_v, "instances": stc.M, "width": Wc,
                     "height": Hc, "sh_degree": cfgc.sh_degree,
                     "stage_ms": {s_: round(float(perc[:, j].mean()), 4)
                                  for j, s_ in enumerate(stages)},
                     "step_hbm_frac": round(sum(bc.values()) / (msc * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                            5)}
            if not args.no_cpu_baseline:
                log(f"[bench] timing the oracle on {wname}")
                entry["cpu_oracle"], _ = cpu_baseline(wlc, camc, cpu_pix)
            res["configs"][wname] = entry
            del scn, grads, stc, outc, dCc
            torch.cuda.empty_cache()
    if not args.no_prune_stats:
        # the forward raster that also keeps the pruning statistics (Sec. 3.2),
        # plus the per-view count, against the plain forward of the same view
        from paper_2505_19175_amd.render import PruneStats
        ps = PruneStats(N, device=dev)
        reps = 20
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * reps)]
        for k in range(reps + 2):
            r = k - 2
            if r >= 0: ev[3 * r].record(stream)
            B.ts_render_forward_stats(st.proj, st.bins, ccam, ccfg, out.rgb, out.alpha, out.depth,
                                      out.T_final, out.last, ps.c, sh_)
            if r >= 0: ev[3 * r + 1].record(stream)
            B.ts_prune_count_views(ps.pixels, ps.views, N, sh_)
            if r >= 0: ev[3 * r + 2].record(stream)
        # one more statistics pass, outside the timing: the per-triangle pixel
        # counts sum to F, the number of composited fragments of the view
        ps.pixels.zero_()
        B.ts_render_forward_stats(st.proj, st.bins, ccam, ccfg, out.rgb, out.alpha, out.depth,
                                  out.T_final, out.last, ps.c, sh_)
        torch.cuda.synchronize()
        F = int(ps.pixels.sum(dtype=torch.int64).item())
        res["fragments"] = F
        fwd_s = float(np.mean([ev[3 * r].elapsed_time(ev[3 * r + 1]) for r in range(reps)]))
        cnt_s = float(np.mean([ev[3 * r + 1].elapsed_time(ev[3 * r + 2]) for r in range(reps)]))
        res["prune_stats"] = {
            "raster_fwd_stats_ms": round(fwd_s, 4), "count_views_ms": round(cnt_s, 4),
            "raster_fwd_ms": stage_ms["raster_fwd"],
            "overhead_frac": round((fwd_s + cnt_s) / stage_ms["raster_fwd"] - 1.0, 4),
            "triangles_rendered_gt1px": int((ps.views > 0).sum().item())}
        del ps
    if not args.no_windows:
        # the two window alternatives of Sec. 3.1 on the same view
        import dataclasses
        res["windows"] = {}
        for wname, wcode in (("sigmoid", synth.WINDOW_SIGMOID), ("lse", synth.WINDOW_LSE)):
            cfg_w = dataclasses.replace(cfg, window=wcode)
            stw, outw, ccw, dCw = prepare(cam, Rasterizer(cfg_w, device=dev))
            msw, perw = timed(make_step(stw, outw, ccw, dCw, B.make_config(cfg_w)), 20, 3, stw)
            res["windows"][wname] = {
                "steps": 20, "ms_per_step": round(msw, 4),
                "Mpixel_per_s": round(W * H / (msw * 1e-3) / 1e6, 3),
                "N_visible": stw.N_v, "instances": stw.M,
                "stage_ms": {s: round(float(perw[:, j].mean()), 4) for j, s in enumerate(stages)}}
            del stw, outw, dCw
    if not args.no_train:
        # one synthetic training step (Sec. 3.3) on the same view: fit a copy
        # of the soup with vertices moved by N(0, 0.002^2) to the original's
        # render; forward, L1 + D-SSIM loss, backward, regularizers + Adam
        import dataclasses
        from paper_2505_19175_amd.train import TrainState
        tgt = out.rgb.clone()
        rng_t = np.random.default_rng(88)
        sc_t = dataclasses.replace(wl.scene, v=(wl.scene.v + rng_t.normal(
            0, 0.002, wl.scene.v.shape)).astype(np.float32))
        ts = TrainState(sc_t, device=dev)
        stt = ViewState(N, W, H, 4 * N, device=dev)
        outt = stt.outputs()
        ras.forward(stt, ts.scene_t(), cam, out=outt, sync=True)
        stt._alloc_lists(int(stt.M * 1.3) + 4096)
        gv_t, go_t, gs_t, gsh_t = ts.grads

        def train_step(ev=None, fused=True):
            if ev: ev[0].record(stream)
            ras.forward(stt, ts.scene_t(), cam, out=outt, sync=False)
            if ev: ev[1].record(stream)
            dCt = ts.image_loss(outt.rgb, tgt)
            if ev: ev[2].record(stream)
            ts.t += 1
            ts.opt.step = ts.t
            if fused:
                # Adam where each triangle's gradient is formed: no gradient arrays
                B.ts_raster_backward(stt.proj, stt.bins, stt.ccam, ccfg, dCt, None, None,
                                     outt.T_final, outt.last, sh_)
                if ev: ev[3].record(stream)
                B.ts_project_backward_adam(ts.v, ts.a, ts.b, ts.sh, ts.o, ts.sigma, N, stt.proj,
                                           stt.ccam, ccfg, ts.state, ts.opt, sh_)
            else:
                B.ts_render_backward(ts.v, ts.o, ts.sigma, ts.sh, N, stt.proj, stt.bins,
                                     stt.ccam, ccfg, dCt, None, None, outt.T_final, outt.last,
                                     gv_t, go_t, gs_t, gsh_t, sh_)
                if ev: ev[3].record(stream)
                B.ts_optimizer_step(ts.v, ts.a, ts.b, ts.sh, ts.o, ts.sigma, ts.deg, N, gv_t,
                                    go_t, gs_t, gsh_t, ts.state, ts.opt, sh_)
            if ev: ev[4].record(stream)

        def time_train(fused, reps=20):
            for _ in range(3):
                train_step(fused=fused)
            torch.cuda.synchronize()
            evt = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
            w0 = time.perf_counter()
            for k in range(reps):
                train_step(evt[k], fused)
            torch.cuda.synchronize()
            wall_t = (time.perf_counter() - w0) / reps * 1e3
            assert int(stt.d_count[2].item()) == 0, "instance list overflow"
            part = np.array([[evt[k][j].elapsed_time(evt[k][j + 1]) for j in range(4)]
                             for k in range(reps)]).mean(0)
            return max(float(evt[0][0].elapsed_time(evt[-1][4])) / reps, wall_t), part

        reps = 20
        ms_sep, part_sep = time_train(False, reps)
        loss0 = ts.loss_value()
        ms_t, part = time_train(True, reps)
        K3 = 3 * K
        opt_bytes = N * (28.0 * (9 + K3) + 2 * 36.0)
        # fused: per parameter read p, m, s and write them (24 B); the
        # activated copies of o and sigma (16 B); rect and tile count (12 B);
        # per visible triangle its 2D gradients read and re-zeroed and the
        # colour Jacobian (176 B)
        fused_bytes = N * (24.0 * (9 + K3 + 2) + 16 + 12) + stt.N_v * 176.0
        loss_bytes = 44.0 * 3 * W * H
        res["train_step"] = {
            "workload": f"tri3M_{W}x{H}: fit a copy of the soup with vertices moved by "
                        f"N(0, 0.002^2) to the original's render",
            "steps": reps, "ms_per_step": round(ms_t, 4),
            "Mpixel_per_s": round(W * H / (ms_t * 1e-3) / 1e6, 3),
            "stage_ms": {"forward": round(float(part[0]), 4), "image_loss": round(float(part[1]), 4),
                         "raster_backward": round(float(part[2]), 4),
                         "backward_projection_adam": round(float(part[3]), 4)},
            "backward_projection_adam_GBps_algorithmic":
                round(fused_bytes / (part[3] * 1e-3) / 1e9, 1),
            "image_loss_GBps_algorithmic": round(loss_bytes / (part[1] * 1e-3) / 1e9, 1),
            "separate": {"ms_per_step": round(ms_sep, 4),
                         "stage_ms": {"forward": round(float(part_sep[0]), 4),
                                      "image_loss": round(float(part_sep[1]), 4),
                                      "backward": round(float(part_sep[2]), 4),
                                      "optimizer": round(float(part_sep[3]), 4)},
                         "optimizer_GBps_algorithmic":
                             round(opt_bytes / (part_sep[3] * 1e-3) / 1e9, 1)},
            "loss_first": round(loss0, 6), "loss_last": round(ts.loss_value(), 6),
            "bytes_note": "fused: the backward projection applies Adam where each triangle's "
                          "gradient is formed (24 B per parameter, 16 B for the activated "
                          "opacity and sigma, 12 B of tile data per triangle, 176 B per visible "
                          "triangle); separate: the gradients are written, then the optimizer "
                          "reads them (28 B per parameter, 36 B for each logit with its "
                          "activated copy); image loss: 44 B per value"}
        del ts, stt, outt, tgt
    if not args.no_densify:
        # densification (Sec. 3.2) on the same soup: Bernoulli selection of
        # 10% of the triangles by inverse sigma, then midpoint subdivision
        # in place (30% more triangles); the soup copy has room for them
        NSH = 3 * K
        cap = N + 3 * int(0.12 * N) + 1024
        dv = torch.zeros((cap, 9), dtype=torch.float32, device=dev)
        do_ = torch.zeros(cap, dtype=torch.float32, device=dev)
        ds = torch.zeros(cap, dtype=torch.float32, device=dev)
        dsh = torch.zeros((cap, NSH), dtype=torch.float32, device=dev)
        dv[:N].copy_(v.reshape(N, 9)); do_[:N].copy_(o); ds[:N].copy_(sg)
        dsh[:N].copy_(sh.reshape(N, NSH))
        gen = np.random.default_rng(77)
        u = torch.tensor(gen.random(N).astype(np.float32), device=dev)
        sel = torch.empty(N, dtype=torch.uint8, device=dev)
        dws_bytes = B.ts_densify_workspace_bytes(N)
        dws = torch.empty(dws_bytes, dtype=torch.uint8, device=dev)
        dcnt = torch.zeros(2, dtype=torch.int32, device=dev)
        reps = 20
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * reps)]
        for k in range(reps + 2):
            r = k - 2
            if r >= 0: ev[3 * r].record(stream)
            B.ts_densify_select(do_, ds, N, B.TS_DENSIFY_INV_SIGMA, 0.1 * N, u, sel, dws, dws_bytes,
                                sh_)
            if r >= 0: ev[3 * r + 1].record(stream)
            B.ts_densify_subdivide(dv, do_, ds, dsh, cfg.sh_degree, N, cap, sel, dws, dws_bytes,
                                   dcnt, None, sh_)
            if r >= 0: ev[3 * r + 2].record(stream)
        torch.cuda.synchronize()
        sel_ms = float(np.mean([ev[3 * r].elapsed_time(ev[3 * r + 1]) for r in range(reps)]))
        sub_ms = float(np.mean([ev[3 * r + 1].elapsed_time(ev[3 * r + 2]) for r in range(reps)]))
        n_sel = (int(dcnt[0].item()) - N) // 3
        assert int(dcnt[1].item()) == 0
        sel_bytes = 13.0 * N                     # weight twice (sum, test), u, flag
        sub_bytes = 1.0 * N + n_sel * (4 * (9 + 2 + NSH) + 4 * (4 * 9 + 3 * (2 + NSH)))
        res["densify"] = {
            "workload": f"{N} triangles, SH degree {cfg.sh_degree}, k = 0.1 N by inverse sigma",
            "selected": n_sel, "select_ms": round(sel_ms, 4), "subdivide_ms": round(sub_ms, 4),
            "select_GBps_algorithmic": round(sel_bytes / (sel_ms * 1e-3) / 1e9, 1),
            "subdivide_GBps_algorithmic": round(sub_bytes / (sub_ms * 1e-3) / 1e9, 1),
            "bytes_note": "select: 13 B per triangle; subdivide: 1 B per triangle + per selected "
                          "the parent row read (236 B at SH-3) and 4 vertex rows + 3 attribute "
                          "rows written (744 B)"}
        del dv, do_, ds, dsh, u, sel, dws
    if not args.no_other_view:
        ov = 1 - args.view if args.view in (0, 1) else 1
        cam2 = wl.cameras[ov]
        st2, out2, ccam2, dC2 = prepare(cam2)
        ms2, per2 = timed(make_step(st2, out2, ccam2, dC2), 20, 3, st2)
        res["other_view"] = {
            "workload": f"tri3M_{cam2.width}x{cam2.height}, hemisphere pose {ov}",
            "width": cam2.width, "height": cam2.height, "N_visible": st2.N_v,
            "instances": st2.M, "steps": 20, "ms_per_step": round(ms2, 4),
            "Mpixel_per_s": round(cam2.width * cam2.height / (ms2 * 1e-3) / 1e6, 3),
            "stage_ms": {s: round(float(per2[:, j].mean()), 4) for j, s in enumerate(stages)}}
        del st2, out2, dC2
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a pixel sample")
        res["cpu_baseline"], nfrag = cpu_baseline(wl, cam, args.cpu_pixels)
        F_est = nfrag * W * H
        res["memory"]["fragments_estimate"] = round(F_est)
        res["memory"]["stored_fragment_bytes_estimate"] = round(12 * F_est)
        res["memory"]["fragment_note"] = (
            "fragments: F, composited fragments of the view, summed from the statistics "
            "forward's per-triangle pixel counts; fragments_estimate: the oracle's mean count "
            "on the sample pixels times W*H; a backward that stored them would keep >= 12 B "
            "each (index, alpha, T)")
    if not args.no_cpu_baseline and not args.no_cpu_rows:
        import dataclasses
        log("[bench] timing the oracle beside the paths beyond the step")
        res["cpu_rows"] = cpu_rows(wl, cam, {
            "sigmoid": dataclasses.replace(cfg, window=synth.WINDOW_SIGMOID),
            "lse": dataclasses.replace(cfg, window=synth.WINDOW_LSE)},
            out.rgb.cpu().numpy().astype(np.float64))
    if not args.no_serve:
        rates = [int(r) for r in args.serve_rates.split(",")]
        d2h_rates = [int(r) for r in args.serve_d2h_rates.split(",") if r]
        res["serve"] = serve_bench(rates, args.serve_seconds, args.serve_warmup, d2h_rates,
                                   args.serve_d2h_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
