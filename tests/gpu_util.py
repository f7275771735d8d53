"""Helpers of the GPU parity tests: run the C-ABI path on synthetic inputs
and compare with the oracle to the stated bars."""
import numpy as np
import torch

from paper_2505_19175_amd import binding as B
from paper_2505_19175_amd.render import Rasterizer, ViewState, scene_to_device

# forward bar: |delta| <= 1e-5 per channel (depth: 1e-5 * max(1, z_max))
FWD_ATOL = 1e-5
# gradient bar: per element |delta| <= 1e-3 |ref| + 1e-6 max|ref of group|,
# and relative L2 error of every group <= 1e-3
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-6
GRAD_L2 = 1e-3


def gpu_forward(scene, cam, cfg, capacity=None, keys=True, sync=True):
    dev = torch.device("cuda:0")
    st_scene = scene_to_device(scene, dev)
    cap = capacity if capacity is not None else max(4 * scene.n, 1 << 16)
    st = ViewState(scene.n, cam.width, cam.height, cap, device=dev, keys=keys)
    ras = Rasterizer(cfg, device=dev)
    out = ras.forward(st, st_scene, cam, sync=sync)
    torch.cuda.synchronize()
    return ras, st, st_scene, out


def gpu_backward(ras, st, st_scene, out, dC, dA=None, dD=None):
    dev = out.rgb.device
    t = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dev)
    g = ras.backward(st, st_scene, out, t(dC), t(dA), t(dD))
    torch.cuda.synchronize()
    return {k: x.cpu().numpy().astype(np.float64) for k, x in zip(("v", "o", "sigma", "sh"), g)}


def to_np(out):
    return {"rgb": out.rgb.cpu().numpy().astype(np.float64),
            "alpha": out.alpha.cpu().numpy().astype(np.float64),
            "depth": out.depth.cpu().numpy().astype(np.float64),
            "T_final": out.T_final.cpu().numpy().astype(np.float64),
            "last": out.last.cpu().numpy()}


def _resolve_flagged(g, r, flag, zmax, pix_lin, resolve, max_dec=4):
    """Flagged pixels: the oracle renders every combination of the pixel's
    alpha / T decisions within their band taken the other way (both
    outcomes are correct), and the pixel counts as resolved when the GPU
    matches one of them within the forward bar.  A depth tie (flag bit 2)
    can only be resolved when the caller has checked that both sides hold
    bit-identical depth keys (resolve[3]): the blending order is then the
    same on both sides.  Returns the boolean mask (over the compared pixels)
    of the resolved ones."""
    from oracle import oracle as O
    scene, cam, cfg = resolve[:3]
    keys_equal = len(resolve) > 3 and bool(resolve[3])
    resolved = np.zeros(flag.shape, bool)
    cand = np.flatnonzero((flag != 0) & (keys_equal | ((flag & 4) == 0)))
    if cand.size == 0:
        return resolved
    lin = pix_lin[cand]
    nd = O.render_flip(scene, cam, cfg, lin, np.zeros(lin.size, np.uint32))["ndec"]
    rows, masks = [], []
    for c, n in zip(cand, nd):
        if n <= max_dec:
            m = np.arange(1 << int(n), dtype=np.uint32)
            rows.append(np.full(m.size, c))
            masks.append(m)
    if not rows:
        return resolved
    rows = np.concatenate(rows)
    masks = np.concatenate(masks)
    var = O.render_flip(scene, cam, cfg, pix_lin[rows], masks)
    ok = np.abs(g["rgb"][:, rows] - var["rgb"]).max(0) <= FWD_ATOL
    for k in ("alpha", "T_final"):
        ok &= np.abs(g[k][rows] - var[k]) <= FWD_ATOL
    ok &= np.abs(g["depth"][rows] - var["depth"]) <= FWD_ATOL * zmax
    resolved[rows[ok]] = True
    return resolved


def compare_forward(gpu, ref, pix=None, W=None, resolve=None):
    """gpu: full-frame arrays; ref: oracle arrays (full frame or sampled at
    pix).  Flagged pixels (a decision within a rounding band of its
    threshold) are left out and counted.  With resolve = (scene, camera,
    config[, depth keys checked equal]), a flagged pixel whose GPU value
    matches one of the outcomes of its near-threshold decisions counts as
    compared, not flagged.  Returns
    (n_compared, n_flagged, worst deltas)."""
    if pix is None:
        g = {k: gpu[k].reshape(gpu[k].shape[0], -1) if k == "rgb" else gpu[k].reshape(-1)
             for k in ("rgb", "alpha", "depth", "T_final")}
        r = {k: ref[k].reshape(ref[k].shape[0], -1) if k == "rgb" else ref[k].reshape(-1)
             for k in ("rgb", "alpha", "depth", "T_final")}
        flag = ref["flag"].reshape(-1)
    else:
        g = {"rgb": gpu["rgb"].reshape(3, -1)[:, pix]}
        for k in ("alpha", "depth", "T_final"):
            g[k] = gpu[k].reshape(-1)[pix]
        r = ref
        flag = ref["flag"]
    ok = flag == 0
    zmax = max(1.0, float(np.abs(r["depth"]).max()) if r["depth"].size else 1.0)
    if resolve is not None:
        pix_lin = np.arange(flag.size, dtype=np.int64) if pix is None else np.asarray(pix, np.int64)
        res = _resolve_flagged(g, r, flag, zmax, pix_lin, resolve)
        n_ok = int(ok.sum()) + int(res.sum())
        worst = {
            "rgb": float(np.abs(g["rgb"][:, ok] - r["rgb"][:, ok]).max(initial=0.0)),
            "alpha": float(np.abs(g["alpha"][ok] - r["alpha"][ok]).max(initial=0.0)),
            "T_final": float(np.abs(g["T_final"][ok] - r["T_final"][ok]).max(initial=0.0)),
            "depth": float(np.abs(g["depth"][ok] - r["depth"][ok]).max(initial=0.0)) / zmax,
        }
        return n_ok, int(flag.size) - n_ok, worst
    worst = {
        "rgb": float(np.abs(g["rgb"][:, ok] - r["rgb"][:, ok]).max(initial=0.0)),
        "alpha": float(np.abs(g["alpha"][ok] - r["alpha"][ok]).max(initial=0.0)),
        "T_final": float(np.abs(g["T_final"][ok] - r["T_final"][ok]).max(initial=0.0)),
        "depth": float(np.abs(g["depth"][ok] - r["depth"][ok]).max(initial=0.0)) / zmax,
    }
    return int(ok.sum()), int((~ok).sum()), worst


def assert_forward(gpu, ref, pix=None, max_flag_frac=0.01, resolve=None):
    n_ok, n_flag, worst = compare_forward(gpu, ref, pix, resolve=resolve)
    assert n_flag <= max_flag_frac * (n_ok + n_flag) + 2, (n_ok, n_flag)
    for k, d in worst.items():
        assert d <= FWD_ATOL, (k, d, worst)
    return n_ok, n_flag, worst


def compare_grads(g, r):
    """Per-element and per-group L2 comparison; returns worst stats."""
    stats = {}
    for k in ("v", "o", "sigma", "sh"):
        a = np.asarray(g[k], np.float64).reshape(-1)
        b = np.asarray(r[k], np.float64).reshape(-1)
        scale = float(np.abs(b).max(initial=0.0))
        tol = GRAD_RTOL * np.abs(b) + GRAD_FLOOR * scale
        bad = np.abs(a - b) > tol
        l2 = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        stats[k] = dict(n_bad=int(bad.sum()), n=int(a.size), l2=l2, scale=scale,
                        worst=float((np.abs(a - b) / np.maximum(tol, 1e-30)).max(initial=0.0)))
    return stats


def assert_grads(g, r):
    s = compare_grads(g, r)
    for k, d in s.items():
        assert d["n_bad"] == 0 and d["l2"] <= GRAD_L2, (k, s)
    return s
