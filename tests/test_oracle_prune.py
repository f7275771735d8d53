"""Pins of the oracle's pruning statistics (Sec. 3.2, "Pruning": the largest
blending weight T*o of each triangle over the rendered pixels, and the pixels
where it is composited).  Expected values come from closed forms written here
in numpy: the window of a triangle given in pixel coordinates is
u = (distance to the nearest edge) / inradius, alpha = min(alpha_max, o u^sigma)."""
import numpy as np

from oracle import oracle as O
from paper_2505_19175_amd.synth import Config

from helpers import camera, dc_for_rgb, scene

W = H = 32
F = 40.0                                        # focal length of the identity camera


def flat_triangles(q2d, z, o, sigma):
    """Triangles given by pixel-space vertices q2d[n][3][2] (pixel centre
    (i+1/2, j+1/2) convention), each flat at depth z[n]."""
    q2d = np.asarray(q2d, np.float64)
    z = np.asarray(z, np.float64)
    v = np.zeros(q2d.shape[:2] + (3,))
    v[..., 0] = (q2d[..., 0] - W / 2) * z[:, None] / F
    v[..., 1] = (q2d[..., 1] - H / 2) * z[:, None] / F
    v[..., 2] = z[:, None]
    n = len(z)
    return scene(v, o, sigma, [[dc_for_rgb([0.3, 0.5, 0.7])]] * n, dtype=np.float64)


def cam():
    return camera(np.eye(3), np.zeros(3), F, F, W / 2, H / 2, W, H)


def window_u(q):
    """u at every pixel centre for one triangle q[3][2] (pixel coordinates)."""
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    A2 = (q[1][0] - q[0][0]) * (q[2][1] - q[0][1]) - (q[1][1] - q[0][1]) * (q[2][0] - q[0][0])
    sgn = np.sign(A2)
    dists, per = [], 0.0
    for k in range(3):
        a, b = np.asarray(q[k]), np.asarray(q[(k + 1) % 3])
        e = b - a
        L = np.hypot(*e)
        per += L
        # inward signed distance: positive inside for either orientation
        dists.append(sgn * (e[0] * (py - a[1]) - e[1] * (px - a[0])) / L)
    r = abs(A2) / per
    return np.minimum(np.minimum(dists[0], dists[1]), dists[2]) / r


Q = [[4.0, 3.0], [27.0, 6.0], [9.0, 28.0]]      # a generic triangle inside the image


def test_single_triangle():
    cfg = Config(sh_degree=0)
    o, sig = 0.8, 1.7
    sc = flat_triangles([Q], [5.0], o, sig)
    st = O.prune_stats(sc, cam(), cfg)
    u = window_u(Q)
    a = np.minimum(cfg.alpha_max, o * np.where(u > 0, u, 0.0) ** sig)
    comp = (u > 0) & (a >= cfg.alpha_min)
    assert st["pixels"][0] == comp.sum() > 100
    assert abs(st["max_weight"][0] - o) < 1e-12          # T = 1 in front of the only triangle


def test_stack_with_termination():
    """Eight copies of one triangle at increasing depth: the transmittance in
    front of copy i is (1 - alpha)^i, and a pixel stops at the copy that would
    take it below T_min."""
    cfg = Config(sh_degree=0)
    o, sig, n = 0.95, 0.2, 8
    sc = flat_triangles([Q] * n, 4.0 + np.arange(n), o, sig)
    st = O.prune_stats(sc, cam(), cfg)
    u = window_u(Q)
    a = np.minimum(cfg.alpha_max, o * np.where(u > 0, u, 0.0) ** sig)
    T = np.ones_like(a)
    live = (u > 0) & (a >= cfg.alpha_min)
    for i in range(n):
        comp = live & (T * (1.0 - a) >= cfg.T_min)
        assert st["pixels"][i] == comp.sum(), i
        want = (T * o)[comp].max() if comp.any() else 0.0
        assert abs(st["max_weight"][i] - want) < 1e-12, i
        live = comp                                   # a stopped pixel composites nothing more
        T = np.where(comp, T * (1.0 - a), T)
    # deeper copies composite at fewer pixels: the centre stops after a few
    assert np.all(np.diff(st["pixels"]) <= 0) and st["pixels"][n - 1] < st["pixels"][0] // 2


def test_front_back_order_and_sample():
    """A smaller triangle behind a larger one: its weight is o times the
    front's transmittance; rendering a subset of pixels sums to the whole."""
    cfg = Config(sh_degree=0)
    big = [[1.0, 1.0], [31.0, 2.0], [3.0, 31.0]]
    small = [[8.0, 8.0], [18.0, 9.0], [9.0, 19.0]]
    ob, os_, sig = 0.6, 0.7, 1.0
    sc = flat_triangles([small, big], [6.0, 3.0], [os_, ob], sig)   # input order: back first
    st = O.prune_stats(sc, cam(), cfg)
    ub, us = window_u(big), window_u(small)
    ab = np.minimum(cfg.alpha_max, ob * np.clip(ub, 0, None) ** sig)
    as_ = np.minimum(cfg.alpha_max, os_ * np.clip(us, 0, None) ** sig)
    cb = (ub > 0) & (ab >= cfg.alpha_min)
    Tb = np.where(cb, 1.0 - ab, 1.0)
    cs = (us > 0) & (as_ >= cfg.alpha_min) & (Tb * (1.0 - as_) >= cfg.T_min)
    assert st["pixels"][1] == cb.sum() and st["pixels"][0] == cs.sum()
    assert abs(st["max_weight"][1] - ob) < 1e-12
    assert abs(st["max_weight"][0] - (Tb * os_)[cs].max()) < 1e-12
    # the statistics of a pixel subset: pixel counts add up, maxima combine by max
    idx = np.arange(W * H)
    a1 = O.prune_stats(sc, cam(), cfg, pix=idx[: W * H // 3])
    a2 = O.prune_stats(sc, cam(), cfg, pix=idx[W * H // 3:])
    np.testing.assert_array_equal(a1["pixels"] + a2["pixels"], st["pixels"])
    np.testing.assert_array_equal(np.maximum(a1["max_weight"], a2["max_weight"]), st["max_weight"])


def test_permutation_invariance():
    rng = np.random.default_rng(7)
    n = 40
    q = rng.uniform(2, 30, (n, 3, 2))
    sc = flat_triangles(q, rng.uniform(3, 9, n), rng.uniform(0.2, 0.9, n), rng.uniform(0.5, 2, n))
    cfg = Config(sh_degree=0)
    st = O.prune_stats(sc, cam(), cfg)
    perm = rng.permutation(n)
    sc2 = scene(sc.v[perm], sc.o[perm], sc.sigma[perm], sc.sh[perm], dtype=np.float64)
    st2 = O.prune_stats(sc2, cam(), cfg)
    np.testing.assert_array_equal(st2["pixels"], st["pixels"][perm])
    np.testing.assert_allclose(st2["max_weight"], st["max_weight"][perm], rtol=0, atol=1e-15)
    assert (st["pixels"] > 0).sum() > n // 2
