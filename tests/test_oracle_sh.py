"""Pins of the oracle's real spherical harmonics (colour of Sec. 3.1 with
degree 3, Sec. 4 'Implementation details'): orthonormality by quadrature,
agreement with scipy's complex harmonics, the degree-0 constant, and the
basis gradient against finite differences on the sphere."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O


def _dirs(n, seed=0):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d


def test_orthonormal_by_quadrature():
    deg = 3
    K = 16
    zs, wz = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phis = 2 * np.pi * np.arange(nphi) / nphi
    G = np.zeros((K, K))
    for z, w in zip(zs, wz):
        st = math.sqrt(1 - z * z)
        for ph in phis:
            Y = O.sh_basis(deg, [st * math.cos(ph), st * math.sin(ph), z])
            G += (w * 2 * np.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(K), atol=1e-12)


def test_matches_scipy_complex_harmonics():
    """Real basis, index l*l+l+m, without the Condon-Shortley phase:
    m>0: sqrt2 (-1)^m Re Y_l^m, m<0: sqrt2 (-1)^m Im Y_l^|m|, m=0: Y_l^0."""
    for d in _dirs(50, 1):
        theta = math.acos(d[2])
        phi = math.atan2(d[1], d[0])
        Y = O.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                am = abs(m)
                c = sp.sph_harm_y(l, am, theta, phi)
                if m == 0:
                    ref = c.real
                elif m > 0:
                    ref = math.sqrt(2) * (-1) ** am * c.real
                else:
                    ref = math.sqrt(2) * (-1) ** am * c.imag
                assert Y[l * l + l + m] == pytest.approx(ref, abs=1e-12), (l, m)


def test_degree0_constant():
    for d in _dirs(5, 2):
        Y = O.sh_basis(0, d)
        assert Y[0] == pytest.approx(1 / (2 * math.sqrt(math.pi)), abs=1e-15)


def test_gradient_on_sphere():
    h = 1e-6
    rng = np.random.default_rng(1003)
    for d in _dirs(30, 3):
        Y, dY = O.sh_basis(3, d, grad=True)
        t = rng.normal(size=3)
        t -= d * np.dot(t, d)
        t /= np.linalg.norm(t)
        dp = (d + h * t) / np.linalg.norm(d + h * t)
        dm = (d - h * t) / np.linalg.norm(d - h * t)
        fd = (O.sh_basis(3, dp) - O.sh_basis(3, dm)) / (2 * h)
        np.testing.assert_allclose(dY @ t, fd, atol=1e-8)
