"""Pins of the oracle's window function, projection and tight box against
what the paper fixes (Eq. 1 and its three properties, the sigma limits,
depth-consistent scaling, the supplementary tight-box formula) and against
independent derivations (barycentric form, homothety about the incentre)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_19175_amd.synth import Camera, Config

from helpers import golden, worked_example, scene


def _bary_u(q, p):
    """u(p) = min_k lambda_k(p) P / l_k: the barycentric coordinate of the
    vertex opposite edge k, scaled by perimeter over that edge's length.
    At the incentre lambda_k = l_k / P, so u = 1 there; on edge k it is 0."""
    q = np.asarray(q, np.float64)
    A = np.vstack([q.T, np.ones(3)])
    lam = np.linalg.solve(A, np.array([p[0], p[1], 1.0]))
    ell = [np.linalg.norm(q[(k + 1) % 3] - q[k]) for k in range(3)]
    P = sum(ell)
    return min(lam[(k + 2) % 3] * P / ell[k] for k in range(3))


def _incentre(q):
    q = np.asarray(q, np.float64)
    a = np.linalg.norm(q[2] - q[1])   # opposite vertex 0
    b = np.linalg.norm(q[0] - q[2])   # opposite vertex 1
    c = np.linalg.norm(q[1] - q[0])   # opposite vertex 2
    return (a * q[0] + b * q[1] + c * q[2]) / (a + b + c)


def _random_tris(seed, n, scale=20.0):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        q = rng.uniform(-scale, scale, (3, 2))
        e1, e2 = q[1] - q[0], q[2] - q[0]
        if abs(e1[0] * e2[1] - e1[1] * e2[0]) > 0.05 * scale * scale:
            out.append(q)
    return out


def test_worked_example_window():
    g = golden("worked_example.json")
    q = g["triangle_2d"]
    for pt in g["u_points"]:
        u, I = O.window(q, pt["p"], 2.0)
        assert u == pytest.approx(pt["u"], abs=1e-12), pt
        assert I == pytest.approx(max(pt["u"], 0.0) ** 2, abs=1e-12)
    for p in g["outside_points"]:
        u, I = O.window(q, p, 2.0)
        assert u < 0 and I == 0.0


def test_worked_example_render_3d():
    g, sc, cam, cfg = worked_example()
    out = O.render(sc, cam, cfg)
    for px in g["pixels_3d"]:
        x, y = px["pixel"]
        assert out["alpha"][y, x] == pytest.approx(px["alpha"], abs=1e-9)
        assert out["T_final"][y, x] == pytest.approx(px["T_final"], abs=1e-9)
        assert out["depth"][y, x] == pytest.approx(px["depth"], abs=1e-8)
        np.testing.assert_allclose(out["rgb"][:, y, x], px["rgb"], atol=1e-9)


def test_worked_example_setup_and_tight_box():
    g, sc, cam, cfg = worked_example()
    st = O.setup(sc, cam, cfg)
    assert st["vis"][0] == 1
    np.testing.assert_allclose(st["q"][0], g["triangle_2d"], atol=1e-12)
    assert st["r"][0] == pytest.approx(g["inradius"], abs=1e-12)
    np.testing.assert_allclose(st["s"][0], g["incentre"], atol=1e-12)
    assert st["phis"][0] == pytest.approx(-g["inradius"], abs=1e-12)
    assert list(st["rect"][0]) == g["tight_box"]["pixel_rect"]
    assert st["ntiles"][0] == 1
    # the shrunk vertices: u_min = (tau/o)^(1/sigma) reproduces the printed value
    u_min = (g["tight_box"]["tau_cutoff"] / 0.8) ** 0.5
    assert u_min == pytest.approx(g["tight_box"]["u_min"], rel=1e-12)
    s = np.array(g["incentre"])
    shr = s + (1 - u_min) * (np.array(g["triangle_2d"]) - s)
    np.testing.assert_allclose(shr, g["tight_box"]["shrunk_vertices"], atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_window_properties(seed):
    """Eq. 1: I = 1 at the incentre, 0 on the boundary and outside, in [0,1]."""
    rng = np.random.default_rng(100 + seed)
    for q in _random_tris(seed, 30):
        s = _incentre(q)
        u, I = O.window(q, s, 1.7)
        assert u == pytest.approx(1.0, abs=1e-12) and I == pytest.approx(1.0, abs=1e-12)
        for k in range(3):
            e = q[(k + 1) % 3] - q[k]
            t = rng.uniform(0.05, 0.95)
            pb = q[k] + t * e
            u, I = O.window(q, pb, 1.7)
            assert abs(u) < 1e-9 and I < 1e-9
            # step outward across edge k: the window vanishes
            nrm = np.array([e[1], -e[0]]) / np.linalg.norm(e)
            if np.dot(nrm, s - pb) > 0:
                nrm = -nrm
            u, I = O.window(q, pb + 0.5 * nrm, 1.7)
            assert u < 0 and I == 0.0
        # interior and exterior samples stay in [0,1]; maximum at s
        pts = rng.uniform(q.min(0) - 2, q.max(0) + 2, (200, 2))
        for p in pts:
            u, I = O.window(q, p, 0.8)
            assert 0.0 <= I <= 1.0 + 1e-15
            assert u <= 1.0 + 1e-12


@pytest.mark.parametrize("seed", [3, 4])
def test_sdf_equals_barycentric_form(seed):
    """phi(p)/phi(s) = min_k lambda_k(p) P / l_k (an independent derivation
    of the same quantity from barycentric coordinates)."""
    rng = np.random.default_rng(seed)
    for q in _random_tris(seed, 40):
        for p in rng.uniform(q.min(0) - 3, q.max(0) + 3, (25, 2)):
            u, _ = O.window(q, p, 1.0)
            ub = _bary_u(q, p)
            assert u == pytest.approx(ub, abs=1e-11 * max(1.0, abs(ub)))


def test_sigma_limits():
    """sigma -> 0: the indicator of the triangle; sigma -> inf: a delta at s."""
    rng = np.random.default_rng(7)
    for q in _random_tris(7, 20):
        s = _incentre(q)
        lam = rng.dirichlet([1, 1, 1], 50)
        for l in lam:
            p = l @ q
            u, _ = O.window(q, p, 1.0)
            if u < 1e-3:
                continue
            _, I0 = O.window(q, p, 1e-6)
            assert I0 > 1 - 1e-4            # indicator: 1 inside
            if u < 0.99:
                _, Iinf = O.window(q, p, 1e6)
                assert Iinf < 1e-10         # delta: 0 away from s
        _, Is = O.window(q, s, 1e6)
        assert Is == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("a", [0.01, 0.37, 3.0, 250.0])
def test_scale_invariance(a):
    """Supp. 'Depth-dependant scaling': scaling triangle and pixel by a
    leaves I unchanged, so one sigma serves all depths."""
    rng = np.random.default_rng(11)
    for q in _random_tris(11, 20):
        for p in rng.uniform(q.min(0) - 1, q.max(0) + 1, (10, 2)):
            u1, I1 = O.window(q, p, 1.3)
            u2, I2 = O.window(a * q, a * p, 1.3)
            assert u2 == pytest.approx(u1, abs=1e-10)
            assert I2 == pytest.approx(I1, abs=1e-10)


def _pixel_camera(W, H):
    # fx = fy = 1, principal point 0, triangles at z = 1: q = (x, y)
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 1.0, 0.0, 0.0,
                  W, H).astype32()


@pytest.mark.parametrize("seed", [0, 1])
def test_tight_box_brute_force(seed):
    """Supp. 'Tile assignment': every pixel whose fragment reaches
    alpha_min lies inside the tight rectangle, and the rectangle equals the
    pixel-centre box of the triangle scaled about its incentre by 1-u_min,
    u_min = (tau/o)^(1/sigma) (an independent construction)."""
    rng = np.random.default_rng(seed)
    W, H = 96, 80
    cam = _pixel_camera(W, H)
    cfg = Config(sh_degree=0)
    tris, os_, ss = [], [], []
    while len(tris) < 60:
        q = rng.uniform([-10, -10], [W + 10, H + 10], (3, 2))
        e1, e2 = q[1] - q[0], q[2] - q[0]
        if abs(e1[0] * e2[1] - e1[1] * e2[0]) < 20:
            continue
        tris.append(q)
        os_.append(rng.uniform(0.02, 1.0))
        ss.append(rng.choice([0.3, 1.0, 2.5, 6.0]))
    v = np.concatenate([np.array(tris), np.ones((60, 3, 1))], axis=2)
    sc = scene(v, os_, ss, np.zeros((60, 1, 3)), dtype=np.float64)
    st = O.setup(sc, cam, cfg)
    amin = float(np.float32(cfg.alpha_min))
    amax = float(np.float32(cfg.alpha_max))
    for i, q in enumerate(tris):
        px0, px1, py0, py1 = st["rect"][i]
        o, sig = os_[i], ss[i]
        # independent homothety construction
        s = _incentre(q)
        umin = (amin / o) ** (1.0 / sig)
        shr = s + (1 - umin) * (q - s)
        ex = [max(0, math.ceil(shr[:, 0].min() - 0.5)), min(W - 1, math.floor(shr[:, 0].max() - 0.5)),
              max(0, math.ceil(shr[:, 1].min() - 0.5)), min(H - 1, math.floor(shr[:, 1].max() - 0.5))]
        if ex[0] > ex[1] or ex[2] > ex[3]:
            assert st["ntiles"][i] == 0
        else:
            assert [px0, px1, py0, py1] == ex
        # brute force over every pixel centre of the image
        lo = np.floor(q.min(0)).astype(int)
        hi = np.ceil(q.max(0)).astype(int)
        for y in range(max(0, lo[1] - 1), min(H, hi[1] + 1)):
            for x in range(max(0, lo[0] - 1), min(W, hi[0] + 1)):
                u, I = O.window(q, (x + 0.5, y + 0.5), sig)
                a = min(amax, o * I)
                if a >= amin * (1 + 1e-9):
                    assert px0 <= x <= px1 and py0 <= y <= py1, (i, x, y, a)


def test_projection_pinhole():
    """Sec. 3.1 pinhole model with the perspective divide: scaling the scene
    about the camera centre leaves the image unchanged; the principal point
    and the two focal lengths place the vertices."""
    g, sc, cam, cfg = worked_example()
    # move the triangle to twice the depth and twice the size: same image
    sc2 = scene(np.asarray(sc.v) * 2.0, sc.o, sc.sigma, sc.sh, dtype=np.float64)
    st1, st2 = O.setup(sc, cam, cfg), O.setup(sc2, cam, cfg)
    np.testing.assert_allclose(st2["q"], st1["q"], atol=1e-12)
    assert st2["zc"][0] == pytest.approx(2 * st1["zc"][0])
    # principal point and focal length
    cam2 = Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 7.0, 5.0, 3.0, 2.0, 8, 8)
    sc3 = scene([[[0, 0, 4], [4, 0, 4], [0, 4, 4]]], 0.5, 1.0, [[[0, 0, 0]]], dtype=np.float64)
    st3 = O.setup(sc3, cam2, cfg)
    np.testing.assert_allclose(st3["q"][0], [[3, 2], [10, 2], [3, 7]], atol=1e-12)
