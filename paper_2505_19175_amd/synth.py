"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds only data containers and random-input recipes.  It does
none of the rasterizer's arithmetic (no projection, no window, no
compositing, no spherical harmonics): both the GPU path and the oracle
receive these arrays and compute everything themselves.

The recipes stand in for the paper's Mip-NeRF360 / Tanks&Temples scenes
(Sec. 4, "Novel-view synthesis"; Garden is about 2M triangles, Sec. 4 game
engine table), which are not available: a soup of independent triangles with
59 floats each at SH degree 3 (Sec. 4 "Implementation details"), clustered
like an SfM-initialised scene, seen from posed pinhole cameras (Sec. 3.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


# ---------------------------------------------------------------------------
# Containers
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Camera:
    """Pinhole camera, world -> camera x_c = R v + t (OpenCV axes: x right,
    y down, z forward).  All values are float32 as the GPU receives them."""
    R: np.ndarray          # (3,3) float32, row-major
    t: np.ndarray          # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def astype32(self) -> "Camera":
        return Camera(np.asarray(self.R, np.float32).reshape(3, 3),
                      np.asarray(self.t, np.float32).reshape(3),
                      float(np.float32(self.fx)), float(np.float32(self.fy)),
                      float(np.float32(self.cx)), float(np.float32(self.cy)),
                      int(self.width), int(self.height))


# Window functions (Sec. 3.1): the paper's ReLU(phi/phi(s))^sigma (Eq. 1), and
# the two alternatives it discusses: sigmoid(-phi/sigma) (Eq. 2) and Eq. 1
# with the max of the SDF replaced by LogSumExp.
WINDOW_PAPER, WINDOW_SIGMOID, WINDOW_LSE = 0, 1, 2


@dataclasses.dataclass
class Config:
    """Rasterizer constants.  The paper names tau_cutoff but gives no value
    and is silent on the others; these are the readings both sides use."""
    alpha_min: float = 1.0 / 255.0   # tau_cutoff: fragments below are skipped
    alpha_max: float = 0.99          # opacity clamp (keeps 1-alpha >= 0.01)
    T_min: float = 1e-4              # early-termination transmittance
    z_near: float = 0.2              # near plane (whole-triangle cull)
    r_min: float = 1e-6              # degenerate 2D triangle cull (inradius, px)
    sh_degree: int = 3
    bg: tuple = (0.0, 0.0, 0.0)
    window: int = 0                  # WINDOW_PAPER, WINDOW_SIGMOID or WINDOW_LSE

    def as_f32(self) -> "Config":
        f = lambda x: float(np.float32(x))
        return Config(f(self.alpha_min), f(self.alpha_max), f(self.T_min),
                      f(self.z_near), f(self.r_min), int(self.sh_degree),
                      tuple(f(b) for b in self.bg), int(self.window))


@dataclasses.dataclass
class Scene:
    """Triangle soup (Sec. 3.1): vertices, opacity, smoothness, SH colour."""
    v: np.ndarray       # (N,3,3) float32
    o: np.ndarray       # (N,)   float32, activated opacity in (0,1]
    sigma: np.ndarray   # (N,)   float32, window smoothness > 0
    sh: np.ndarray      # (N,K,3) float32, K = (deg+1)^2

    @property
    def n(self) -> int:
        return int(self.v.shape[0])

    @property
    def sh_degree(self) -> int:
        return int(round(math.sqrt(self.sh.shape[1]))) - 1

    def subset(self, idx) -> "Scene":
        return Scene(self.v[idx], self.o[idx], self.sigma[idx], self.sh[idx])


def sh_count(deg: int) -> int:
    return (deg + 1) * (deg + 1)


def focal_for_fov60(width: int) -> float:
    """Horizontal field of view of 60 degrees: f = (W/2)/tan(30 deg)."""
    return (width / 2.0) / math.tan(math.radians(30.0))


def look_at(eye, target=(0.0, 0.0, 0.0), width=1280, height=720,
            f: Optional[float] = None) -> Camera:
    """Camera at `eye` looking at `target`, world 'up' = -y.
    Rows of R are the camera axes x^, y^, z^ in world coordinates."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.array([0.0, -1.0, 0.0]))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ eye
    if f is None:
        f = focal_for_fov60(width)
    return Camera(R.astype(np.float32), t.astype(np.float32), f, f,
                  width / 2.0, height / 2.0, width, height).astype32()


def identity_camera(width: int, height: int, f: Optional[float] = None) -> Camera:
    if f is None:
        f = focal_for_fov60(width)
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f,
                  width / 2.0, height / 2.0, width, height).astype32()


# ---------------------------------------------------------------------------
# Triangle generators
# ---------------------------------------------------------------------------

def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations from unit quaternions (Shoemake)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qw = a * np.sin(2 * np.pi * u2)
    qx = a * np.cos(2 * np.pi * u2)
    qy = b * np.sin(2 * np.pi * u3)
    qz = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def _equilateral_soup(rng, centres: np.ndarray, edge_median: float,
                      edge_sigma_log: float = 0.7) -> np.ndarray:
    """Approximately equilateral, randomly oriented triangles around
    `centres` (the paper's initialisation shape, Sec. 3.3), with log-normal
    edge lengths and a per-vertex jitter of 0.15 edge."""
    n = centres.shape[0]
    ell = rng.lognormal(math.log(edge_median), edge_sigma_log, n)
    ang = np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3])
    base = np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], axis=1) / math.sqrt(3.0)
    rot = _random_rotations(rng, n)
    v = np.einsum("nij,kj->nki", rot, base) * ell[:, None, None]
    v += rng.normal(0.0, 1.0, (n, 3, 3)) * (0.15 * ell)[:, None, None]
    v += centres[:, None, :]
    return v


def _sh_coeffs(rng, n: int, deg: int, hi_std: float = 0.05) -> np.ndarray:
    K = sh_count(deg)
    sh = np.empty((n, K, 3))
    sh[:, 0, :] = rng.random((n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, hi_std, (n, K - 1, 3))
    return sh


def _pack(v, o, sigma, sh) -> Scene:
    return Scene(np.ascontiguousarray(v, np.float32),
                 np.ascontiguousarray(o, np.float32),
                 np.ascontiguousarray(sigma, np.float32),
                 np.ascontiguousarray(sh, np.float32))


def box_soup(seed: int, n: int, jitter: float = 0.1, sh_degree: int = 0,
             sigma: float = 1.0, o_range=(0.1, 0.9)) -> Scene:
    """Centres uniform in x,y in [-1,1], z in [2,4]; each vertex is the
    centre plus N(0, jitter^2) per axis (the 1k-triangle 128x128 case)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.empty((n, 3))
    c[:, 0:2] = rng.uniform(-1.0, 1.0, (n, 2))
    c[:, 2] = rng.uniform(2.0, 4.0, n)
    v = c[:, None, :] + rng.normal(0.0, jitter, (n, 3, 3))
    o = rng.uniform(o_range[0], o_range[1], n)
    sh = _sh_coeffs(rng, n, sh_degree)
    s = np.full(n, sigma)
    return _pack(v, o, s, sh)


def cluster_soup(seed: int, n: int, n_clusters: int = 64, extent: float = 5.0,
                 std: float = 0.5, edge_median: float = 0.02, sh_degree: int = 3,
                 shell_frac: float = 0.0, shell_radius: float = 20.0,
                 rng: Optional[np.random.Generator] = None) -> Scene:
    """Mixture of isotropic Gaussian clusters (centres uniform in a cube of
    half-size `extent`), optionally with a fraction on a background shell."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    n_shell = int(round(n * shell_frac))
    n_dense = n - n_shell
    cc = rng.uniform(-extent, extent, (n_clusters, 3))
    lab = rng.integers(0, n_clusters, n_dense)
    centres = cc[lab] + rng.normal(0.0, std, (n_dense, 3))
    if n_shell:
        d = rng.normal(0.0, 1.0, (n_shell, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rad = shell_radius * (1.0 + rng.normal(0.0, 0.02, n_shell))
        centres = np.concatenate([centres, d * rad[:, None]], axis=0)
    v = _equilateral_soup(rng, centres, edge_median)
    o = rng.uniform(0.05, 1.0, n)
    sigma = rng.uniform(0.5, 2.0, n)
    sh = _sh_coeffs(rng, n, sh_degree)
    return _pack(v, o, sigma, sh)


def ring_camera(rng, radius=4.0, width=1280, height=720) -> Camera:
    phi = rng.uniform(0.0, 2 * np.pi)
    eye = (radius * math.cos(phi), 0.0, radius * math.sin(phi))
    return look_at(eye, width=width, height=height)


def hemisphere_cameras(rng, count: int, radius=5.0, sizes=((1280, 720),)):
    """Poses eye = r(cos e cos a, -sin e, cos e sin a), a~U(0,2pi),
    e~U(5deg,85deg), looking at the origin (above the scene: -y is up)."""
    cams = []
    for i in range(count):
        a = rng.uniform(0.0, 2 * np.pi)
        e = math.radians(rng.uniform(5.0, 85.0))
        eye = (radius * math.cos(e) * math.cos(a), -radius * math.sin(e),
               radius * math.cos(e) * math.sin(a))
        w, h = sizes[i % len(sizes)]
        cams.append(look_at(eye, width=w, height=h))
    return cams


def hemisphere_eyes(rng, count: int, radius=5.0):
    out = []
    for _ in range(count):
        a = rng.uniform(0.0, 2 * np.pi)
        e = math.radians(rng.uniform(5.0, 85.0))
        out.append((radius * math.cos(e) * math.cos(a), -radius * math.sin(e),
                    radius * math.cos(e) * math.sin(a)))
    return out


def upstream(seed: int, width: int, height: int, with_alpha=False, with_depth=False):
    """Upstream image gradients dL/drgb [3,H,W] (and optionally dL/dalpha,
    dL/ddepth [H,W]), standard normal, float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dC = rng.normal(0.0, 1.0, (3, height, width)).astype(np.float32)
    dA = rng.normal(0.0, 1.0, (height, width)).astype(np.float32) if with_alpha else None
    dD = rng.normal(0.0, 1.0, (height, width)).astype(np.float32) if with_depth else None
    return dC, dA, dD


def pixel_sample(seed: int, width: int, height: int, count: int) -> np.ndarray:
    """Seeded sample of distinct linear pixel indices y*W+x, sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, width * height)
    return np.sort(rng.choice(width * height, size=count, replace=False)).astype(np.int64)


# ---------------------------------------------------------------------------
# The workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cameras: list
    config: Config
    upstream_seed: int
    sigma_sweep: tuple = ()


def workload_small(n: int = 1000) -> Workload:
    """1,000 triangles at 128x128, SH degree 0, sigma = 1 (seed 1)."""
    sc = box_soup(1, n, jitter=0.1, sh_degree=0, sigma=1.0)
    cam = identity_camera(128, 128)
    return Workload("tri1k_128x128", sc, [cam], Config(sh_degree=0), 101)


def workload_mid(n: int = 300_000) -> Workload:
    """300k clustered triangles at 1280x720, SH degree 3 (seed 2)."""
    rng = np.random.Generator(np.random.PCG64(2))
    sc = cluster_soup(2, n, n_clusters=64, extent=5.0, std=0.5, edge_median=0.02,
                      sh_degree=3, rng=rng)
    cam = ring_camera(rng, 4.0, 1280, 720)
    return Workload("tri300k_1280x720", sc, [cam], Config(sh_degree=3), 102)


def workload_large(n: int = 3_000_000) -> Workload:
    """3M triangles, 70% in a dense central mixture and 30% on a shell of
    radius 20, SH degree 3; 8 hemisphere poses alternating 1280x720 and
    1600x1040 (seed 3)."""
    rng = np.random.Generator(np.random.PCG64(3))
    sc = cluster_soup(3, n, n_clusters=64, extent=2.0, std=0.3, edge_median=0.01,
                      sh_degree=3, shell_frac=0.3, shell_radius=20.0, rng=rng)
    cams = hemisphere_cameras(rng, 8, 5.0, sizes=((1280, 720), (1600, 1040)))
    return Workload("tri3M_1280x720", sc, cams, Config(sh_degree=3), 103)


def workload_grad(sigma: float, n: int = 20_000) -> Workload:
    """20k triangles at 256x256, SH degree 1, one sigma for all triangles
    (seed 4); the sigma sweep is {0.25, 1, 4}."""
    sc = box_soup(4, n, jitter=0.05, sh_degree=1, sigma=sigma)
    cam = identity_camera(256, 256)
    return Workload(f"tri20k_256x256_s{sigma:g}", sc, [cam], Config(sh_degree=1), 104,
                    sigma_sweep=(0.25, 1.0, 4.0))


def workload_serve(n: int = 1_000_000) -> Workload:
    """Resident 1M-triangle SH-3 soup from the cluster generator (seed 5)."""
    rng = np.random.Generator(np.random.PCG64(5))
    sc = cluster_soup(5, n, n_clusters=64, extent=5.0, std=0.5, edge_median=0.02,
                      sh_degree=3, rng=rng)
    return Workload("serve1M", sc, [], Config(sh_degree=3), 105)


SERVE_SIZES = ((640, 360), (1280, 720), (1920, 1080))
