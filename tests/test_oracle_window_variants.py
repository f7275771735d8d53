"""Pins of the oracle's two window alternatives (Sec. 3.1, the discussion of
window functions): the sigmoid window of Eq. 2, I = sigmoid(-phi/sigma), and
Eq. 1 with the SDF's max replaced by LogSumExp.  The expected values come
from closed forms written here from the 2D vertices (edge lines found by a
centroid side test, SDFs by numpy), not from the oracle's own set-up."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_19175_amd.synth import (WINDOW_LSE, WINDOW_PAPER, WINDOW_SIGMOID, Camera,
                                        Config)

from helpers import random_soup, scene
import test_oracle_grad as TG

LN3 = math.log(3.0)


def _lines(q):
    """Unit normals n_k pointing away from the centroid and offsets d_k of
    the three edge lines: L_k(p) = n_k . p + d_k, negative inside."""
    q = np.asarray(q, np.float64)
    c = q.mean(0)
    out = []
    for k in range(3):
        a, b = q[k], q[(k + 1) % 3]
        e = b - a
        n = np.array([e[1], -e[0]]) / np.linalg.norm(e)
        if np.dot(n, c - a) > 0:
            n = -n
        out.append((n, -np.dot(n, a)))
    return out


def _L(q, p):
    return np.array([n @ np.asarray(p, np.float64) + d for n, d in _lines(q)])


def _inradius(q):
    q = np.asarray(q, np.float64)
    e1, e2 = q[1] - q[0], q[2] - q[0]
    area2 = abs(e1[0] * e2[1] - e1[1] * e2[0])
    per = sum(np.linalg.norm(q[(k + 1) % 3] - q[k]) for k in range(3))
    return area2 / per


def _incentre(q):
    q = np.asarray(q, np.float64)
    a, b, c = (np.linalg.norm(q[2] - q[1]), np.linalg.norm(q[0] - q[2]),
               np.linalg.norm(q[1] - q[0]))
    return (a * q[0] + b * q[1] + c * q[2]) / (a + b + c)


def _sigmoid_I(q, p, sig):
    return 1.0 / (1.0 + math.exp(_L(q, p).max() / sig))


def _lse_u(q, p):
    ps = np.logaddexp.reduce(_L(q, _incentre(q)))
    return np.logaddexp.reduce(_L(q, p)) / ps if ps < 0 else 0.0


def _tris(seed, n, scale=20.0, min_r=0.0):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        q = rng.uniform(-scale, scale, (3, 2))
        e1, e2 = q[1] - q[0], q[2] - q[0]
        if abs(e1[0] * e2[1] - e1[1] * e2[0]) > 0.05 * scale * scale and _inradius(q) > min_r:
            out.append(q)
    return out


# ---------------------------------------------------------------------------
# sigmoid window (Eq. 2)
# ---------------------------------------------------------------------------

def test_sigmoid_at_incentre_boundary_and_outside():
    """1/2 on the boundary, sigmoid(r/sigma) at the incentre, and the
    closed form at random points inside and outside."""
    rng = np.random.default_rng(1)
    for q in _tris(1, 30):
        r, s = _inradius(q), _incentre(q)
        for sig in (0.3, 1.0, 4.0):
            u, I = O.window(q, s, sig, WINDOW_SIGMOID)
            assert u == pytest.approx(-r, abs=1e-10)
            assert I == pytest.approx(1.0 / (1.0 + math.exp(-r / sig)), abs=1e-12)
            for k in range(3):
                pb = q[k] + rng.uniform(0.1, 0.9) * (q[(k + 1) % 3] - q[k])
                _, I = O.window(q, pb, sig, WINDOW_SIGMOID)
                assert I == pytest.approx(0.5, abs=1e-10)
            for p in rng.uniform(q.min(0) - 5, q.max(0) + 5, (20, 2)):
                u, I = O.window(q, p, sig, WINDOW_SIGMOID)
                assert u == pytest.approx(_L(q, p).max(), abs=1e-10)
                assert I == pytest.approx(_sigmoid_I(q, p, sig), abs=1e-12)


def test_sigmoid_breaks_the_two_properties():
    """Its largest value stays below 1 and its support reaches past the
    triangle; sigma -> infinity gives 1/2 everywhere."""
    for q in _tris(2, 10):
        s = _incentre(q)
        _, I = O.window(q, s, 1.0, WINDOW_SIGMOID)
        assert I < 1.0
        far = q.max(0) + 3.0
        _, I = O.window(q, far, 2.0, WINDOW_SIGMOID)
        assert I > 0.0
        for p in (s, far, q.min(0) - 10.0):
            _, I = O.window(q, p, 1e9, WINDOW_SIGMOID)
            assert I == pytest.approx(0.5, abs=1e-7)


# ---------------------------------------------------------------------------
# LogSumExp SDF in the window of Eq. 1
# ---------------------------------------------------------------------------

def test_lse_small_triangle_has_no_inside():
    """At the incentre every edge line is at distance r, so phi_lse(s) =
    log 3 - r: a triangle with r <= log 3 pixels has no point with
    phi_lse < 0 at s, and its window vanishes everywhere."""
    q = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 4.0]])   # 3-4-5: r = 1 < log 3
    assert _inradius(q) == pytest.approx(1.0)
    for p in ([1.0, 1.0], [0.5, 0.5], [1.5, 1.0], [5.0, 5.0]):
        u, I = O.window(q, p, 1.0, WINDOW_LSE)
        assert u == 0.0 and I == 0.0
    # scaled by 1.2 (r = 1.2 > log 3) the incentre is inside again: u(s) = 1
    u, I = O.window(1.2 * q, [1.2, 1.2], 1.0, WINDOW_LSE)
    assert u == pytest.approx(1.0, abs=1e-12) and I == pytest.approx(1.0, abs=1e-12)


def test_lse_pointwise_and_bounds():
    """u = phi_lse(p)/phi_lse(s) with phi_lse(s) = log 3 - r; since
    max <= LogSumExp <= max + log 3, the LSE region lies inside the
    triangle, and for large triangles u approaches Eq. 1's."""
    rng = np.random.default_rng(3)
    for q in _tris(3, 25, scale=30.0, min_r=2.0):
        r, s = _inradius(q), _incentre(q)
        assert np.logaddexp.reduce(_L(q, s)) == pytest.approx(LN3 - r, abs=1e-12)
        for p in rng.uniform(q.min(0) - 3, q.max(0) + 3, (25, 2)):
            u, I = O.window(q, p, 1.7, WINDOW_LSE)
            ue = _lse_u(q, p)
            assert u == pytest.approx(ue, abs=1e-11)
            assert I == pytest.approx(max(ue, 0.0) ** 1.7, abs=1e-11)
            u0, _ = O.window(q, p, 1.7, WINDOW_PAPER)
            if u > 0:
                assert u0 > 0                        # inside the triangle
            Lm = _L(q, p).max()
            assert Lm <= np.logaddexp.reduce(_L(q, p)) <= Lm + LN3 + 1e-12
        big = 500.0 * q
        for lam in rng.dirichlet([2, 2, 2], 10):
            p = lam @ big
            u, _ = O.window(big, p, 1.0, WINDOW_LSE)
            u0, _ = O.window(big, p, 1.0, WINDOW_PAPER)
            assert abs(u - u0) <= 2 * LN3 / (500.0 * _inradius(q)) + 1e-12


# ---------------------------------------------------------------------------
# tight boxes, the single-triangle render and gradients of both variants
# ---------------------------------------------------------------------------

def _pixel_camera(W, H):
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 1.0, 0.0, 0.0,
                  W, H).astype32()


def _closed_alpha(window, q, p, o, sig, amax):
    if window == WINDOW_SIGMOID:
        return min(amax, o * _sigmoid_I(q, p, sig))
    u = _lse_u(q, p)
    return min(amax, o * u ** sig) if u > 0 else 0.0


@pytest.mark.parametrize("window", [WINDOW_SIGMOID, WINDOW_LSE])
@pytest.mark.parametrize("seed", [0, 1])
def test_variant_tight_box_brute_force(window, seed):
    """Every pixel centre whose alpha reaches alpha_min lies in the tight
    rectangle, and the rectangle is the pixel-centre box of the triangle
    scaled about its incentre: by (r - d)/r with d = -sigma log(o/tau - 1)
    for the sigmoid (culled when d >= r), by 1 - u_min (r - log 3)/r for
    LogSumExp, u_min = (tau/o)^(1/sigma)."""
    rng = np.random.default_rng(10 + seed)
    W, H = 96, 80
    cam = _pixel_camera(W, H)
    cfg = Config(sh_degree=0, window=window)
    n = 50
    tris, os_, ss = [], [], []
    while len(tris) < n:
        q = rng.uniform([-10, -10], [W + 10, H + 10], (3, 2))
        if _inradius(q) < 1.5:
            continue
        tris.append(q)
        os_.append(rng.choice([0.009, 0.05, 0.4, 1.0]) if window == WINDOW_SIGMOID
                   else rng.uniform(0.02, 1.0))
        ss.append(rng.choice([0.3, 1.0, 2.5]))
    v = np.concatenate([np.array(tris), np.ones((n, 3, 1))], axis=2)
    sc = scene(v, os_, ss, np.zeros((n, 1, 3)), dtype=np.float64)
    st = O.setup(sc, cam, cfg)
    amin = float(np.float32(cfg.alpha_min))
    amax = float(np.float32(cfg.alpha_max))
    n_box = 0
    for i, q in enumerate(tris):
        o, sig, r, s = os_[i], ss[i], _inradius(q), _incentre(q)
        if window == WINDOW_SIGMOID:
            d = -sig * math.log(o / amin - 1.0)
            f = (r - d) / r
        else:
            f = 1.0 - (amin / o) ** (1.0 / sig) * (r - LN3) / r
        rect = list(st["rect"][i])
        if f <= 0:
            assert st["ntiles"][i] == 0
            continue
        shr = s + f * (q - s)
        ex = [max(0, math.ceil(shr[:, 0].min() - 0.5)), min(W - 1, math.floor(shr[:, 0].max() - 0.5)),
              max(0, math.ceil(shr[:, 1].min() - 0.5)), min(H - 1, math.floor(shr[:, 1].max() - 0.5))]
        if ex[0] > ex[1] or ex[2] > ex[3]:
            assert st["ntiles"][i] == 0
            continue
        assert rect == ex, (i, rect, ex)
        n_box += 1
        lo = np.floor(shr.min(0)).astype(int) - 2
        hi = np.ceil(shr.max(0)).astype(int) + 2
        for y in range(max(0, lo[1]), min(H, hi[1])):
            for x in range(max(0, lo[0]), min(W, hi[0])):
                a = _closed_alpha(window, q, (x + 0.5, y + 0.5), o, sig, amax)
                if a >= amin * (1 + 1e-9):
                    assert rect[0] <= x <= rect[1] and rect[2] <= y <= rect[3], (i, x, y, a)
    assert n_box >= 20


@pytest.mark.parametrize("window", [WINDOW_SIGMOID, WINDOW_LSE])
def test_variant_single_triangle_closed_form(window):
    """One triangle renders alpha = min(alpha_max, o I) where it reaches
    alpha_min, with I from the closed forms above."""
    W = H = 40
    cam = _pixel_camera(W, H)
    q = np.array([[6.0, 5.0], [33.0, 9.0], [14.0, 34.0]])
    for o, sig in ((0.8, 1.3), (1.0, 0.4)):
        sc = scene(np.concatenate([q, np.ones((3, 1))], 1)[None], o, sig, np.zeros((1, 1, 3)),
                   dtype=np.float64)
        cfg = Config(sh_degree=0, window=window)
        out = O.render(sc, cam, cfg)
        amin = float(np.float32(cfg.alpha_min))
        amax = float(np.float32(cfg.alpha_max))
        n_in = 0
        for y in range(H):
            for x in range(W):
                a = _closed_alpha(window, q, (x + 0.5, y + 0.5), o, sig, amax)
                a = a if a >= amin else 0.0
                n_in += a > 0
                assert out["alpha"][y, x] == pytest.approx(a, abs=1e-12), (x, y)
        assert n_in > 100


def test_sigmoid_without_cutoff_covers_the_image():
    """alpha_min = 0: the sigmoid has no bounded support, so the tight box
    is the whole image and every pixel is composited."""
    W, H = 24, 20
    cam = _pixel_camera(W, H)
    q = np.array([[6.0, 5.0], [12.0, 6.0], [8.0, 12.0]])
    sc = scene(np.concatenate([q, np.ones((3, 1))], 1)[None], 0.5, 1.0, np.zeros((1, 1, 3)),
               dtype=np.float64)
    cfg = Config(sh_degree=0, window=WINDOW_SIGMOID, alpha_min=0.0, T_min=0.0)
    st = O.setup(sc, cam, cfg)
    assert list(st["rect"][0]) == [0, W - 1, 0, H - 1]
    out = O.render(sc, cam, cfg)
    assert (out["alpha"] > 0).all()


@pytest.mark.parametrize("window", [WINDOW_SIGMOID, WINDOW_LSE])
@pytest.mark.parametrize("group", ["v", "o", "sigma"])
def test_variant_fd_gradients(window, group):
    """Analytic gradient of each variant against Richardson-extrapolated
    central differences on pixels whose discrete state is stable."""
    sc, cam = random_soup(31, 30, W=40, H=32, size=1.4, deg=1, sigma=(0.6, 2.0), o=(0.3, 0.95))
    cfg = Config(sh_degree=1, bg=(0.1, 0.2, 0.3), window=window)
    TG._run_fd(sc, cam, cfg, group, seed=7 + 3 * window + ["v", "o", "sigma"].index(group))
