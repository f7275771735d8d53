"""Pins of the densification oracle (Sec. 3.2 "Densification"; Supp.):
Bernoulli sampling with probabilities from opacity or inverse sigma, and
midpoint subdivision.  Checked against what the definitions fix: the
expected count, proportionality, capping, sampling frequencies over many
seeded draws, the children's areas, their exact cover of the parent, and
the output layout."""
import numpy as np
import pytest

from oracle import densify as D


def _soup(seed, n):
    rng = np.random.default_rng(seed)
    v = rng.normal(0, 1, (n, 3, 3)).astype(np.float32)
    o = rng.uniform(0.01, 1.0, n).astype(np.float32)
    s = rng.uniform(0.3, 4.0, n).astype(np.float32)
    sh = rng.normal(0, 1, (n, 4, 3)).astype(np.float32)
    return v, o, s, sh


@pytest.mark.parametrize("mode", [D.OPACITY, D.INV_SIGMA])
def test_expected_count_and_proportionality(mode):
    v, o, s, sh = _soup(1, 5000)
    k = 500.0
    p = D.probabilities(o, s, mode, k)
    w = o.astype(np.float64) if mode == D.OPACITY else 1.0 / s.astype(np.float64)
    assert p.max() < 1.0
    assert p.sum() == pytest.approx(k, rel=1e-12)
    i, j = 10, 20
    assert p[i] / p[j] == pytest.approx(w[i] / w[j], rel=1e-12)


def test_inverse_sigma_prefers_solid_triangles():
    o = np.full(3, 0.5, np.float32)
    s = np.array([0.5, 1.0, 2.0], np.float32)
    p = D.probabilities(o, s, D.INV_SIGMA, 1.0)
    np.testing.assert_allclose(p, np.array([4, 2, 1]) / 7.0, rtol=1e-15)
    p = D.probabilities(o, s, D.OPACITY, 1.0)
    np.testing.assert_allclose(p, np.full(3, 1 / 3), rtol=1e-15)


def test_capping_at_one():
    o = np.array([0.9, 0.01, 0.01, 0.01], np.float32)
    p = D.probabilities(o, np.ones(4, np.float32), D.OPACITY, 2.0)
    assert p[0] == 1.0 and p.sum() < 2.0
    assert p[1] == pytest.approx(2.0 * 0.01 / 0.93, rel=1e-6)


def test_zero_weights_select_nothing():
    o = np.zeros(5, np.float32)
    assert not D.select(o, np.ones(5, np.float32), D.OPACITY, 3.0, np.zeros(5)).any()


def test_sampling_frequencies():
    """Over 4000 seeded draws every triangle is selected with frequency
    p_i (binomial bound) and the mean count is sum p_i."""
    v, o, s, sh = _soup(2, 40)
    p = D.probabilities(o, s, D.INV_SIGMA, 8.0)
    rng = np.random.default_rng(3)
    T = 4000
    hits = np.zeros(40)
    counts = []
    for _ in range(T):
        sel = D.select(o, s, D.INV_SIGMA, 8.0, rng.random(40))
        hits += sel
        counts.append(sel.sum())
    freq = hits / T
    sd = np.sqrt(p * (1 - p) / T)
    assert np.all(np.abs(freq - p) <= 5 * sd + 1e-12)
    assert abs(np.mean(counts) - p.sum()) <= 5 * np.sqrt((p * (1 - p)).sum() / T)


def _area(t):
    t = np.asarray(t, np.float64)
    return 0.5 * np.linalg.norm(np.cross(t[..., 1, :] - t[..., 0, :], t[..., 2, :] - t[..., 0, :]), axis=-1)


def _inside(t, x):
    """Barycentric coordinates of x in the plane of triangle t (3D)."""
    t = np.asarray(t, np.float64)
    A = np.stack([t[1] - t[0], t[2] - t[0]], 1)
    ab, *_ = np.linalg.lstsq(A, x - t[0], rcond=None)
    return np.array([1 - ab.sum(), ab[0], ab[1]])


def test_children_quarter_area_and_exact_cover():
    v, o, s, sh = _soup(4, 50)
    rng = np.random.default_rng(5)
    for t in v.astype(np.float64):
        ch = D.midpoint_children(t)
        np.testing.assert_allclose(_area(ch), _area(t) / 4, rtol=1e-12)
        for lam in rng.dirichlet([1, 1, 1], 40):
            x = lam @ t
            inside = [np.all(_inside(c, x) > 1e-9) for c in ch]
            on_edge = [np.all(_inside(c, x) > -1e-9) for c in ch]
            assert sum(inside) <= 1 and sum(on_edge) >= 1
        # every child vertex is a parent vertex or an edge midpoint
        mids = {tuple(np.round((t[a] + t[b]) / 2, 6)) for a, b in ((0, 1), (1, 2), (2, 0))}
        corners = {tuple(np.round(x, 6)) for x in t}
        for c in ch:
            for x in c:
                assert tuple(np.round(x, 6)) in mids | corners


def test_float32_midpoint_is_one_rounding():
    v, o, s, sh = _soup(6, 200)
    ch = D.midpoint_children(v)
    exact = ((v[:, 0].astype(np.float64) + v[:, 1].astype(np.float64)) / 2).astype(np.float32)
    assert np.array_equal(ch[:, 0, 0], exact)


def test_subdivide_layout():
    v, o, s, sh = _soup(7, 30)
    sel = np.zeros(30, bool)
    sel[[3, 4, 17, 29]] = True
    ov, oo, os_, osh = D.subdivide(v, o, s, sh, sel)
    assert ov.shape[0] == 30 + 12
    keep = ~sel
    assert np.array_equal(ov[:30][keep], v[keep]) and np.array_equal(oo[:30], o)
    for r, i in enumerate([3, 4, 17, 29]):
        ch = D.midpoint_children(v[i])
        assert np.array_equal(ov[i], ch[0])
        for c in range(3):
            j = 30 + 3 * r + c
            assert np.array_equal(ov[j], ch[1 + c])
            assert oo[j] == o[i] and os_[j] == s[i] and np.array_equal(osh[j], sh[i])
    # total area is preserved
    assert _area(ov).sum() == pytest.approx(_area(v).sum(), rel=1e-6)


# ---------------------------------------------------------------------------
# planted mistakes: each must make one of the pins above fail
# ---------------------------------------------------------------------------

MUTANTS = [
    ("no cap at one", "return np.minimum(1.0, k * w / tot)", "return k * w / tot"),
    ("sigma instead of its inverse", "return 1.0 / np.asarray(sigma, np.float64)",
     "return np.asarray(sigma, np.float64)"),
    ("not normalised", "return np.minimum(1.0, k * w / tot)", "return np.minimum(1.0, k * w)"),
    ("select on >=", "return np.asarray(u, np.float64) < probabilities(",
     "return np.asarray(u, np.float64) >= probabilities("),
    ("wrong corner child", "np.stack([v0, m01, m20], -2),", "np.stack([v0, m01, m12], -2),"),
    ("centre child skipped", "out_v[idx] = ch[:, 0]", "out_v[idx] = v[idx]"),
    ("children without the parent's sigma",
     "out_o[j], out_s[j], out_sh[j] = np.asarray(o)[idx], np.asarray(sigma)[idx], np.asarray(sh)[idx]",
     "out_o[j], out_sh[j] = np.asarray(o)[idx], np.asarray(sh)[idx]"),
    ("append order", "j = N + 3 * np.arange(n) + c", "j = N + np.arange(n) + n * c"),
]


def _pins(M):
    import types
    g = globals()
    return [lambda: _with(M, g["test_expected_count_and_proportionality"], D.OPACITY),
            lambda: _with(M, g["test_expected_count_and_proportionality"], D.INV_SIGMA),
            lambda: _with(M, g["test_inverse_sigma_prefers_solid_triangles"]),
            lambda: _with(M, g["test_capping_at_one"]),
            lambda: _with(M, g["test_zero_weights_select_nothing"]),
            lambda: _with(M, g["test_sampling_frequencies"]),
            lambda: _with(M, g["test_children_quarter_area_and_exact_cover"]),
            lambda: _with(M, g["test_float32_midpoint_is_one_rounding"]),
            lambda: _with(M, g["test_subdivide_layout"])]


def _with(M, fn, *args):
    global D
    saved = D
    D = M
    try:
        fn(*args)
    finally:
        D = saved


@pytest.mark.parametrize("label,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(label, old, new):
    import types
    src = open(D.__file__).read()
    assert src.count(old) == 1, label
    M = types.ModuleType("densify_mutant")
    exec(compile(src.replace(old, new), "densify_mutant", "exec"), M.__dict__)
    caught = False
    for pin in _pins(M):
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"no pin catches: {label}"
