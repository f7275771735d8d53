"""Small hand-built inputs for the tests (no rasterizer arithmetic here)."""
import json
import math
import os

import numpy as np

from paper_2505_19175_amd.synth import Camera, Config, Scene

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

DC_SCALE = 2.0 * math.sqrt(math.pi)   # 1 / Y_0^0 of the orthonormal SH basis


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def scene(v, o, sigma, sh, dtype=np.float32) -> Scene:
    v = np.asarray(v, dtype).reshape(-1, 3, 3)
    n = v.shape[0]
    o = np.broadcast_to(np.asarray(o, dtype), (n,)).copy()
    sigma = np.broadcast_to(np.asarray(sigma, dtype), (n,)).copy()
    sh = np.asarray(sh, dtype).reshape(n, -1, 3)
    return Scene(v, o, sigma, sh)


def dc_for_rgb(rgb):
    """SH degree-0 coefficients giving colour `rgb` (rgb = dc Y00 + 1/2)."""
    return (np.asarray(rgb, np.float64) - 0.5) * DC_SCALE


def camera(R, t, fx, fy, cx, cy, W, H) -> Camera:
    return Camera(np.asarray(R, np.float32).reshape(3, 3), np.asarray(t, np.float32).reshape(3),
                  fx, fy, cx, cy, W, H).astype32()


def worked_example(two=False, cfg=None):
    g = golden("worked_example.json")
    s3 = g["scene_3d"]
    cam = camera(s3["R"], s3["t"], s3["fx"], s3["fy"], s3["cx"], s3["cy"], s3["width"], s3["height"])
    v = [s3["vertices"]]
    sh = [[dc_for_rgb(s3["rgb"])]]
    if two:
        v.append(g["two_triangles"]["second_vertices"])
        sh.append([dc_for_rgb(g["two_triangles"]["second_rgb"])])
    sc = scene(v, s3["opacity"], s3["sigma"], sh, dtype=np.float64)
    if cfg is None:
        cfg = Config(sh_degree=0)
    return g, sc, cam, cfg


def random_soup(seed, n, W=48, H=40, size=0.6, deg=0, sigma=(0.5, 3.0), o=(0.2, 0.95),
                dtype=np.float64, zrange=(2.5, 4.0)):
    """Triangles of a few pixels in front of an identity camera."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = (W / 2.0) / math.tan(math.radians(30.0))
    z = rng.uniform(zrange[0], zrange[1], n)
    cx = rng.uniform(-0.55, 0.55, n) * z * (W / 2.0) / f
    cy = rng.uniform(-0.55, 0.55, n) * z * (H / 2.0) / f
    centre = np.stack([cx, cy, z], 1)
    v = centre[:, None, :] + rng.normal(0.0, size / 2.0, (n, 3, 3))
    K = (deg + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.uniform(-1.0, 1.0, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.3, (n, K - 1, 3))
    sc = Scene(v.astype(dtype), rng.uniform(o[0], o[1], n).astype(dtype),
               rng.uniform(sigma[0], sigma[1], n).astype(dtype), sh.astype(dtype))
    cam = Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, W / 2.0, H / 2.0,
                 W, H).astype32()
    return sc, cam
