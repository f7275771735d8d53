"""Pins of the training-step oracle (photometric loss with SSIM, the
opacity and size losses, Adam): closed forms, a brute-force SSIM written
from its definition with explicit loops, finite differences of every
gradient, and Adam's first-step identity."""
import math

import numpy as np
import pytest

from oracle import train as TR


def _brute_ssim(x, y, i, j):
    """SSIM at pixel (i, j) of one channel from the definition: Gaussian
    weighted means over the 11x11 neighbourhood, pixels outside count 0."""
    w = np.array([math.exp(-(k - 5) ** 2 / (2 * 1.5 ** 2)) for k in range(11)])
    w /= w.sum()
    H, W = x.shape
    m = {"x": 0.0, "y": 0.0, "xx": 0.0, "yy": 0.0, "xy": 0.0}
    for a in range(11):
        for b in range(11):
            r, c = i + a - 5, j + b - 5
            if 0 <= r < H and 0 <= c < W:
                ww = w[a] * w[b]
                X, Y = x[r, c], y[r, c]
                m["x"] += ww * X; m["y"] += ww * Y
                m["xx"] += ww * X * X; m["yy"] += ww * Y * Y; m["xy"] += ww * X * Y
    vx = m["xx"] - m["x"] ** 2
    vy = m["yy"] - m["y"] ** 2
    cxy = m["xy"] - m["x"] * m["y"]
    return ((2 * m["x"] * m["y"] + TR.C1) * (2 * cxy + TR.C2)) / \
        ((m["x"] ** 2 + m["y"] ** 2 + TR.C1) * (vx + vy + TR.C2))


def test_window():
    w = TR.gaussian_window()
    assert w.shape == (11, 11) and w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1]) and w.argmax() == 60


def test_ssim_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.random((3, 14, 17))
    y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, 1)
    S = TR.ssim_map(x, y)
    for c in range(3):
        for (i, j) in [(0, 0), (3, 7), (13, 16), (7, 8), (13, 0)]:
            assert S[c, i, j] == pytest.approx(_brute_ssim(x[c], y[c], i, j), abs=1e-12)


def test_ssim_identity_symmetry_constants():
    rng = np.random.default_rng(2)
    x = rng.random((3, 20, 20))
    y = rng.random((3, 20, 20))
    np.testing.assert_allclose(TR.ssim_map(x, x), 1.0, atol=1e-12)
    np.testing.assert_allclose(TR.ssim_map(x, y), TR.ssim_map(y, x), atol=1e-14)
    a, b = 0.3, 0.7
    S = TR.ssim_map(np.full((1, 20, 20), a), np.full((1, 20, 20), b))
    # away from the border the window sees no zeros: both variances vanish
    c1 = 0.01 ** 2   # the constants of the SSIM the paper's loss takes from 3D Gaussian Splatting
    assert S[0, 10, 10] == pytest.approx((2 * a * b + c1) / (a * a + b * b + c1), abs=1e-12)
    # a pixel whose window holds one step edge: variances and covariance in closed form
    x = np.zeros((1, 11, 11)); y = np.zeros((1, 11, 11))
    x[0, :, 6:] = 1.0
    w = TR.gaussian_window()
    mx = w[:, 6:].sum(); vx = mx - mx * mx
    c2 = 0.03 ** 2
    want = (c1 * c2) / ((mx * mx + c1) * (vx + c2))     # y = 0: mu_y = var_y = cov = 0
    assert TR.ssim_map(x, y)[0, 5, 5] == pytest.approx(want, rel=1e-12)
    assert TR.image_loss(x, x) == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
def test_image_loss_gradient_by_differences(lam):
    rng = np.random.default_rng(3)
    C = rng.random((3, 9, 8))
    T = rng.random((3, 9, 8))
    g = TR.image_loss_grad(C, T, lam)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 4, 3), (2, 8, 7), (0, 2, 6), (2, 5, 0)]:
        Cp, Cm = C.copy(), C.copy()
        Cp[idx] += h
        Cm[idx] -= h
        fd = (TR.image_loss(Cp, T, lam) - TR.image_loss(Cm, T, lam)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10), idx
    if lam == 0.0:
        np.testing.assert_allclose(g, np.sign(C - T) / C.size, atol=1e-15)


def test_size_loss_closed_form_and_gradient():
    v = np.array([[[0, 0, 0], [3.0, 0, 0], [0, 4.0, 0]],
                  [[1, 1, 1], [1, 3, 1], [1, 1, 2]]])
    # |(v1 - v0) x (v2 - v0)| = 12 and 2: mean of 2/12 and 2/2
    assert TR.size_loss(v) == pytest.approx((2 / 12 + 2 / 2) / 2)
    rng = np.random.default_rng(4)
    v = rng.normal(0, 1, (6, 3, 3))
    g = TR.size_loss_grad(v)
    h = 1e-7
    for idx in [(0, 0, 0), (1, 1, 2), (2, 2, 1), (5, 0, 2), (3, 1, 0)]:
        vp, vm = v.copy(), v.copy()
        vp[idx] += h
        vm[idx] -= h
        fd = (TR.size_loss(vp) - TR.size_loss(vm)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6), idx


def test_adam_first_step_and_zero_gradient():
    p = np.array([1.0, -2.0, 3.0, 0.5])
    g = np.array([0.3, -1e-3, 5.0, 0.0])
    z = np.zeros(4)
    p1, m, s = TR.adam(p, g, z, z, 0.01, 1)
    # bias correction makes the first step lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + TR.ADAM_EPS), rtol=1e-12)
    assert p1[3] == p[3]
    p2, m, s = TR.adam(p1, g, m, s, 0.01, 2)
    np.testing.assert_allclose(p2, p1 - 0.01 * g / (np.abs(g) + TR.ADAM_EPS), rtol=1e-9)


def test_optimizer_step_chains_activations():
    """With renderer gradients of zero only the regularizers act: opacity
    logits move down (L_o grows with o) by the first-step size lr_o, and
    vertices move so the triangles grow (L_s shrinks with area)."""
    rng = np.random.default_rng(5)
    N, K = 5, 4
    raw = {"v": rng.normal(0, 1, (N, 3, 3)), "a": rng.normal(0, 1, N),
           "b": rng.normal(0, 0.3, N), "sh": rng.normal(0, 1, (N, K, 3))}
    z = {"v": np.zeros((N, 3, 3)), "o": np.zeros(N), "sigma": np.zeros(N),
         "sh": np.zeros((N, K, 3))}
    st = {k: (np.zeros_like(np.asarray(raw[k], float)),) * 2 for k in ("v", "a", "b", "sh")}
    out, st2 = TR.optimizer_step(raw, z, st, 1)
    np.testing.assert_allclose(out["a"], raw["a"] - TR.LR["o"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["b"], raw["b"])
    np.testing.assert_allclose(out["sh"], raw["sh"])
    assert TR.size_loss(out["v"]) < TR.size_loss(raw["v"])
    # the chain through o = sigmoid(a): a renderer gradient g_o gives g_a = g_o o (1 - o)
    g = dict(z, o=np.full(N, 2.0))
    _, st3 = TR.optimizer_step(raw, g, st, 1, beta_o=0.0)
    o = TR.sigmoid(raw["a"])
    np.testing.assert_allclose(st3["a"][0], 0.1 * 2.0 * o * (1 - o), rtol=1e-12)
    g = dict(z, sigma=np.full(N, 3.0))
    _, st4 = TR.optimizer_step(raw, g, st, 1)
    np.testing.assert_allclose(st4["b"][0], 0.1 * 3.0 * np.exp(raw["b"]), rtol=1e-12)
    # degree-0 SH at feature_lr, the rest at feature_lr / 20
    g = dict(z, sh=np.ones((N, K, 3)))
    out5, _ = TR.optimizer_step(raw, g, st, 1)
    np.testing.assert_allclose(raw["sh"][:, 0] - out5["sh"][:, 0], TR.LR["sh_dc"], rtol=1e-9)
    np.testing.assert_allclose(raw["sh"][:, 1:] - out5["sh"][:, 1:], TR.LR["sh_rest"], rtol=1e-9)


# ---------------------------------------------------------------------------
# planted mistakes: each must make one of the pins above fail
# ---------------------------------------------------------------------------

MUTANTS = [
    ("window width", "def gaussian_window(size: int = 11, std: float = 1.5)",
     "def gaussian_window(size: int = 11, std: float = 2.0)"),
    ("constants swapped", "C1 = 0.01 ** 2\nC2 = 0.03 ** 2", "C1 = 0.03 ** 2\nC2 = 0.01 ** 2"),
    ("covariance term dropped", "d_mx = dS_dmx - 2 * mx * dS_dvx - my * dS_dcxy",
     "d_mx = dS_dmx - 2 * mx * dS_dvx"),
    ("second moment not blurred", "2 * x * _blur(d_exx)", "2 * x * d_exx"),
    ("l1 weight", "g = (1 - lam) * np.sign(C - T) / n", "g = np.sign(C - T) / n"),
    ("size gradient operand order", "g1 = np.cross(e2, gc)", "g1 = np.cross(gc, e2)"),
    ("no bias correction", "mh = m / (1 - b1 ** t)", "mh = m"),
    ("sigmoid chain", "ga = go * o * (1 - o)", "ga = go * o"),
    ("exp chain", "gb = np.asarray(grads[\"sigma\"], np.float64) * sig",
     "gb = np.asarray(grads[\"sigma\"], np.float64)"),
    ("rest SH at the dc rate", "rate = np.full(sh.shape, lr[\"sh_rest\"])",
     "rate = np.full(sh.shape, lr[\"sh_dc\"])"),
]

_PINS = ["test_window", "test_ssim_matches_brute_force", "test_ssim_identity_symmetry_constants",
         "test_size_loss_closed_form_and_gradient", "test_adam_first_step_and_zero_gradient",
         "test_optimizer_step_chains_activations"]


@pytest.mark.parametrize("label,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(label, old, new):
    import types
    global TR
    src = open(TR.__file__).read()
    assert src.count(old) == 1, label
    M = types.ModuleType("train_mutant")
    exec(compile(src.replace(old, new), "train_mutant", "exec"), M.__dict__)
    saved, TR = TR, M
    caught = False
    try:
        pins = [globals()[n] for n in _PINS]
        pins += [lambda lam=lam: test_image_loss_gradient_by_differences(lam) for lam in (0.0, 0.2)]
        for pin in pins:
            try:
                pin()
            except Exception:
                caught = True
                break
    finally:
        TR = saved
    assert caught, f"no pin catches: {label}"
