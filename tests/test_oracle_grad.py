"""Pins of the oracle's analytic FP64 gradient (end-to-end gradients to
vertices, opacity, sigma and SH; Sec. 3.3) against central finite
differences of the oracle's own forward.

The forward is discontinuous at three decisions (alpha vs the cut-off,
early termination, depth order) and has kinks where the arg-max edge
changes.  Each probe therefore compares only pixels whose discrete state
(composited set, arg-max edges, clamps, stopping fragment) is the same at
theta-h, theta and theta+h: the loss restricted to those pixels is smooth
in theta, and the analytic gradient of that restricted loss must match."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_19175_amd.synth import Config, Scene

from helpers import random_soup

H_STEP = 1e-4


def _copy(sc):
    return Scene(np.array(sc.v, np.float64), np.array(sc.o, np.float64),
                 np.array(sc.sigma, np.float64), np.array(sc.sh, np.float64))


def _loss(out, mask, dC, dA, dD):
    L = (dC[:, mask] * out["rgb"][:, mask]).sum()
    L += (dA[mask] * out["alpha"][mask]).sum()
    L += (dD[mask] * out["depth"][mask]).sum()
    return L


def _probe_list(sc, st, rng, group, count):
    vis = np.nonzero(st["ntiles"] > 0)[0]
    probes = []
    for _ in range(count):
        i = int(rng.choice(vis))
        if group == "v":
            probes.append(("v", (i, int(rng.integers(3)), int(rng.integers(3)))))
        elif group == "o":
            probes.append(("o", (i,)))
        elif group == "sigma":
            probes.append(("sigma", (i,)))
        else:
            probes.append(("sh", (i, int(rng.integers(sc.sh.shape[1])), int(rng.integers(3)))))
    return probes


def _fd(sc, cam, cfg, name, idx, base, dC, dA, dD, mask=None):
    """Central differences at h and h/2 combined by Richardson extrapolation
    (error O(h^4)); the comparison set is the pixels whose state is the same
    at all four perturbed points."""
    outs = {}
    for h in (H_STEP, H_STEP / 2):
        for sgn in (+1, -1):
            s2 = _copy(sc)
            getattr(s2, name)[idx] += sgn * h
            outs[(h, sgn)] = O.render(s2, cam, cfg)
    stable = np.ones_like(base["hash"], bool) if mask is None else mask.copy()
    for o in outs.values():
        stable &= o["hash"] == base["hash"]
    d = {h: (_loss(outs[(h, 1)], stable, dC, dA, dD) - _loss(outs[(h, -1)], stable, dC, dA, dD)) / (2 * h)
         for h in (H_STEP, H_STEP / 2)}
    return (4 * d[H_STEP / 2] - d[H_STEP]) / 3, stable


def _run_fd(sc, cam, cfg, group, seed, count=24, rtol=2e-5):
    rng = np.random.default_rng(seed)
    H, W = cam.height, cam.width
    dC = rng.normal(size=(3, H, W))
    dA = rng.normal(size=(H, W))
    dD = rng.normal(size=(H, W))
    base = O.render(sc, cam, cfg)
    st = O.setup(sc, cam, cfg)
    checked = 0
    for name, idx in _probe_list(sc, st, rng, group, count):
        fd, stable = _fd(sc, cam, cfg, name, idx, base, dC, dA, dD)
        if stable.sum() == 0:
            continue
        pix = np.nonzero(stable.reshape(-1))[0]
        g = O.backward(sc, cam, cfg, dC.reshape(3, -1)[:, pix], dA.reshape(-1)[pix],
                       dD.reshape(-1)[pix], pix=pix)
        an = g[name][idx]
        scale = max(abs(an), abs(fd), 1e-3)
        assert abs(an - fd) <= rtol * scale + 1e-7, (name, idx, an, fd)
        checked += 1
    assert checked >= count // 2


@pytest.mark.parametrize("group", ["v", "o", "sigma", "sh"])
@pytest.mark.parametrize("sig", [(0.6, 0.9), (1.0, 1.5), (3.0, 5.0)])
def test_fd_state_stable_pixels(group, sig):
    sc, cam = random_soup(21, 40, W=40, H=32, size=1.0, deg=1, sigma=sig, o=(0.3, 0.999))
    cfg = Config(sh_degree=1, bg=(0.1, 0.2, 0.3))
    _run_fd(sc, cam, cfg, group, seed=100 * ["v", "o", "sigma", "sh"].index(group) + int(10 * sig[0]))


def test_fd_degree3_colour():
    sc, cam = random_soup(22, 25, W=32, H=32, size=1.2, deg=3, sigma=(0.8, 2.0))
    cfg = Config(sh_degree=3)
    _run_fd(sc, cam, cfg, "sh", seed=5)
    _run_fd(sc, cam, cfg, "v", seed=6)


def test_fd_clamped_and_terminated():
    """Opaque, overlapping triangles exercise the alpha_max clamp and early
    termination; the gradient through them is the one of the reading (zero
    through the clamp, nothing for the stopping fragment)."""
    sc, cam = random_soup(23, 60, W=32, H=32, size=1.6, deg=0, sigma=(0.03, 0.08), o=(0.995, 1.0))
    cfg = Config(sh_degree=0, T_min=2e-3)
    base = O.render(sc, cam, cfg)
    assert (base["T_final"] < 0.0021).any() and (base["nfrag"] >= 2).any()
    _run_fd(sc, cam, cfg, "v", seed=7)
    _run_fd(sc, cam, cfg, "o", seed=8)


def test_fd_global_smooth_setting():
    """With no cut-off, no termination and no clamp the whole loss is
    smooth in theta (away from arg-max switches and depth swaps)."""
    sc, cam = random_soup(24, 30, W=32, H=28, size=1.0, deg=1, sigma=(1.0, 3.0), o=(0.1, 0.9))
    cfg = Config(alpha_min=0.0, T_min=0.0, sh_degree=1)
    rng = np.random.default_rng(9)
    H, W = cam.height, cam.width
    dC = rng.normal(size=(3, H, W))
    dA = rng.normal(size=(H, W))
    dD = rng.normal(size=(H, W))
    g = O.backward(sc, cam, cfg, dC, dA, dD)
    base = O.render(sc, cam, cfg)
    st = O.setup(sc, cam, cfg)
    n_ok = 0
    for name, idx in _probe_list(sc, st, rng, "v", 20) + _probe_list(sc, st, rng, "sigma", 10):
        fd, stable = _fd(sc, cam, cfg, name, idx, base, dC, dA, dD)
        if not stable.all():
            continue
        an = g[name][idx]
        assert abs(an - fd) <= 2e-5 * max(abs(an), abs(fd), 1e-3) + 1e-7, (name, idx, an, fd)
        n_ok += 1
    assert n_ok >= 15


def test_sampled_backward_equals_masked_full_frame():
    """Backward over a pixel sample equals the full-frame backward with the
    upstream gradient zeroed off the sample."""
    sc, cam = random_soup(25, 50, W=32, H=24, deg=1)
    cfg = Config(sh_degree=1)
    rng = np.random.default_rng(10)
    dC = rng.normal(size=(3, 24, 32))
    pix = np.sort(rng.choice(24 * 32, 200, replace=False))
    mask = np.zeros(24 * 32, bool)
    mask[pix] = True
    dCm = dC.reshape(3, -1) * mask
    g_full = O.backward(sc, cam, cfg, dCm.reshape(3, 24, 32))
    g_s = O.backward(sc, cam, cfg, dC.reshape(3, -1)[:, pix], pix=pix)
    for k in ("v", "o", "sigma", "sh"):
        np.testing.assert_allclose(g_s[k], g_full[k], rtol=1e-12, atol=1e-14)


def test_culled_triangles_get_zero_gradient():
    sc, cam = random_soup(26, 30, W=32, H=24, deg=1)
    sc.v[0, 1, 2] = 0.05          # vertex in front of the near plane
    cfg = Config(sh_degree=1)
    rng = np.random.default_rng(11)
    g = O.backward(sc, cam, cfg, rng.normal(size=(3, 24, 32)))
    assert np.all(g["v"][0] == 0) and g["o"][0] == 0 and np.all(g["sh"][0] == 0)


def test_fd_posed_camera_and_clamped_colour():
    """A rotated, translated camera (R != I) and colours clamped at zero in
    some channels."""
    from paper_2505_19175_amd.synth import look_at
    rng = np.random.default_rng(12)
    n = 30
    cen = rng.uniform(-1.0, 1.0, (n, 3)) * [1.0, 0.7, 1.0]
    v = cen[:, None, :] + rng.normal(0.0, 0.35, (n, 3, 3))
    sh = np.zeros((n, 4, 3))
    sh[:, 0, :] = rng.uniform(-2.6, 1.0, (n, 3))
    sh[:, 1:, :] = rng.normal(0.0, 0.4, (n, 3, 3))
    sc = Scene(v, rng.uniform(0.3, 0.95, n), rng.uniform(0.7, 2.5, n), sh)
    cam = look_at((2.0, -1.5, -4.5), target=(0.1, 0.0, 0.2), width=40, height=32)
    cfg = Config(sh_degree=1, bg=(0.3, 0.1, 0.2))
    st = O.setup(sc, cam, cfg)
    assert (st["rgb"][st["vis"] == 1] == 0).any()     # some channels clamped
    for grp, seed in (("v", 13), ("sh", 14), ("o", 15)):
        _run_fd(sc, cam, cfg, grp, seed=seed, count=20)


def test_opacity_gradient_homogeneity():
    """alpha = o * I is linear in o below the clamp, so o dL/do equals
    alpha dL/dalpha summed over the triangle's composited fragments
    (clamped fragments contribute nothing).  With one pixel per backward each
    triangle has at most one fragment; dL/dalpha comes from a front-to-back
    composite written here, in which L is linear in each alpha, so the
    derivative is L(alpha_i = 1) - L(alpha_i = 0) exactly."""
    sc, cam = random_soup(27, 40, W=24, H=20, size=1.2, o=(0.3, 1.0))
    sc.o[:8], sc.sigma[:8] = 1.0, 0.01     # opaque and flat: clamped inside
    cfg = Config(sh_degree=0, T_min=0.0, bg=(0.2, 0.1, 0.3))
    amin, amax = float(np.float32(cfg.alpha_min)), float(np.float32(cfg.alpha_max))
    bg = np.array(cfg.bg, np.float32).astype(np.float64)
    st = O.setup(sc, cam, cfg)
    full = O.render(sc, cam, cfg)
    rng = np.random.default_rng(16)
    order = np.lexsort((np.arange(sc.n), st["key"]))
    cand = np.argwhere(full["nfrag"] >= 3)
    assert len(cand) > 20
    # the pixels holding the opaque triangles' incentres, and a random sample
    inc = [(int(st["s"][i, 1]), int(st["s"][i, 0])) for i in range(8) if st["vis"][i]]
    inc = [(y, x) for y, x in inc if 0 <= x < cam.width and 0 <= y < cam.height]
    checked = clamped = 0
    for y, x in inc + [tuple(c) for c in cand[rng.choice(len(cand), 20, replace=False)]]:
        p = (x + 0.5, y + 0.5)
        alpha = np.zeros(sc.n)
        for i in np.nonzero(st["vis"])[0]:
            alpha[i] = float(sc.o[i]) * O.window(st["q"][i], p, float(sc.sigma[i]))[1]
        assert not np.any(np.abs(alpha - amin) < 1e-9) and not np.any(np.abs(alpha - amax) < 1e-9)
        frags = [i for i in order if st["vis"][i] and alpha[i] >= amin]
        dC, dA, dD = rng.normal(size=3), rng.normal(), rng.normal()

        def loss(a):
            T, rgb, depth = 1.0, np.zeros(3), 0.0
            for i in frags:
                w = T * a[i]
                rgb += w * st["rgb"][i]
                depth += w * st["zc"][i]
                T *= 1.0 - a[i]
            return (dC * (rgb + T * bg)).sum() + dA * (1.0 - T) + dD * depth, rgb + T * bg, T, depth

        alpha_c = np.minimum(alpha, amax)
        L0, rgb, T, depth = loss(alpha_c)
        pix = np.array([y * cam.width + x])
        np.testing.assert_allclose(rgb, full["rgb"][:, y, x], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(1.0 - T, full["alpha"][y, x], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(depth, full["depth"][y, x], rtol=1e-12, atol=1e-14)
        g = O.backward(sc, cam, cfg, dC.reshape(3, 1), np.array([dA]), np.array([dD]), pix=pix)
        for i in range(sc.n):
            if i in frags and alpha[i] < amax:
                a1, a0 = alpha_c.copy(), alpha_c.copy()
                a1[i], a0[i] = 1.0, 0.0
                want = alpha[i] * (loss(a1)[0] - loss(a0)[0])
                np.testing.assert_allclose(float(sc.o[i]) * g["o"][i], want,
                                           rtol=1e-9, atol=1e-13)
                checked += 1
            else:
                clamped += i in frags
                assert g["o"][i] == 0.0
    assert checked >= 40 and clamped >= 1


@pytest.mark.parametrize("sigma", [0.25, 1.0, 4.0])
def test_fd_grad_workload_bbox(sigma):
    """The 20k-triangle gradient workload (SH degree 1, one sigma for all
    triangles, sigma in {0.25, 1, 4}): for each probed parameter only the
    pixels of that triangle's tight box (plus 2 px) are rendered at theta,
    theta +- h and theta +- h/2, and the analytic gradient of the loss over
    the box's state-stable pixels must match the extrapolated differences."""
    from paper_2505_19175_amd import synth
    wl = synth.workload_grad(sigma)
    sc, cam, cfg = _copy(wl.scene), wl.cameras[0], wl.config
    H, W = cam.height, cam.width
    st = O.setup(sc, cam, cfg)
    rng = np.random.default_rng(int(100 * sigma) + 7)
    dC = rng.normal(size=(3, H * W))
    dA = rng.normal(size=H * W)
    dD = rng.normal(size=H * W)

    def loss(out, m, px):
        return ((dC[:, px][:, m] * out["rgb"][:, m]).sum() + (dA[px][m] * out["alpha"][m]).sum()
                + (dD[px][m] * out["depth"][m]).sum())

    checked = 0
    for group in ("v", "o", "sigma", "sh"):
        for name, idx in _probe_list(sc, st, rng, group, 16):
            x0, x1, y0, y1 = (int(a) for a in st["rect"][idx[0]])
            xs = np.arange(max(x0 - 2, 0), min(x1 + 2, W - 1) + 1)
            ys = np.arange(max(y0 - 2, 0), min(y1 + 2, H - 1) + 1)
            px = (ys[:, None] * W + xs[None, :]).reshape(-1)
            base = O.render(sc, cam, cfg, pix=px)
            outs = {}
            for h in (H_STEP, H_STEP / 2):
                for sgn in (+1, -1):
                    s2 = _copy(sc)
                    getattr(s2, name)[idx] += sgn * h
                    outs[(h, sgn)] = O.render(s2, cam, cfg, pix=px)
            m = np.ones(px.size, bool)
            for o in outs.values():
                m &= o["hash"] == base["hash"]
            if not m.any():
                continue
            d = {h: (loss(outs[(h, 1)], m, px) - loss(outs[(h, -1)], m, px)) / (2 * h)
                 for h in (H_STEP, H_STEP / 2)}
            fd = (4 * d[H_STEP / 2] - d[H_STEP]) / 3
            ps = px[m]
            g = O.backward(sc, cam, cfg, dC[:, ps], dA[ps], dD[ps], pix=ps)
            an = g[name][idx]
            assert abs(an - fd) <= 2e-5 * max(abs(an), abs(fd), 1e-3) + 1e-7, (name, idx, an, fd)
            checked += 1
    assert checked >= 48
