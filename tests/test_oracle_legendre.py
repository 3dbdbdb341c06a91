"""Pins for the oracle's normalised associated Legendre functions
(App. B.3, eq. spherical_harmonics and the orthonormality relation after it).

Anchors: closed forms for l <= 2 (worked by hand), scipy's spherical
harmonics at moderate degree (scipy returns NaN near l = 719), mpmath's
associated Legendre function at 40 digits up to l = 719 (the degree range of
the 721 x 1440 grid), and the Gauss-Legendre Gram matrix, which is the
identity exactly when the functions are orthonormal.
"""
import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle

PI = np.pi


def _closed_forms(t):
    c, s = np.cos(t), np.sin(t)
    return {
        (0, 0): np.full_like(t, 1.0 / np.sqrt(4 * PI)),
        (1, 0): np.sqrt(3 / (4 * PI)) * c,
        (1, 1): -np.sqrt(3 / (8 * PI)) * s,
        (2, 0): np.sqrt(5 / (16 * PI)) * (3 * c * c - 1),
        (2, 1): -np.sqrt(15 / (8 * PI)) * s * c,
        (2, 2): np.sqrt(15 / (32 * PI)) * s * s,
    }


def test_closed_forms_l_le_2():
    t = np.linspace(0.0, PI, 37)
    tab = oracle.legendre_table(3, 3, t)
    for (l, m), ref in _closed_forms(t).items():
        np.testing.assert_allclose(tab[m, l], ref, atol=2e-16, rtol=1e-14)
    # zeros below the diagonal
    assert np.all(tab[1, 0] == 0) and np.all(tab[2, :2] == 0)


def test_against_scipy_moderate_degree():
    t = np.array([0.05, 0.4, 1.1, PI / 2, 2.0, 3.1])
    L = 64
    tab = oracle.legendre_table(L, L, t)
    for l in range(0, L, 7):
        for m in range(0, l + 1, 5):
            ref = np.real(sph_harm_y(l, m, t, 0.0))
            np.testing.assert_allclose(tab[m, l], ref, atol=1e-13, rtol=1e-11)


@pytest.mark.parametrize("l,m,t", [(719, 0, PI * 200 / 720), (719, 1, 0.9),
                                   (719, 301, PI * 200 / 720), (719, 600, PI * 200 / 720),
                                   (500, 251, 1.3), (360, 359, 1.2)])
def test_against_mpmath_high_degree(l, m, t):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    x = mpmath.cos(mpmath.mpf(t))
    c = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m) / mpmath.factorial(l + m))
    # mpmath's legenp (type 2) carries the Condon-Shortley phase itself
    ref = float(c * mpmath.legenp(l, m, x, type=2))
    val = oracle.legendre_table(l + 1, m + 1, np.array([t]))[m, l, 0]
    assert abs(val - ref) <= 1e-11 * max(1.0, abs(ref)) + 1e-14


@pytest.mark.parametrize("nlat", [8, 32, 96])
def test_gauss_gram_is_identity(nlat):
    th, x, w = oracle.grid(nlat, 1)
    L = nlat
    tab = oracle.legendre_table(L, L, th)
    for m in range(L):
        P = tab[m, m:]
        G = 2 * PI * (P * w[None, :]) @ P.T
        np.testing.assert_allclose(G, np.eye(L - m), atol=1e-13)


def test_parity_symmetry():
    # P^_l^m(-x) = (-1)^(l+m) P^_l^m(x): used by nobody in the oracle, pinned
    # here because the GPU path relies on it for the equatorial fold
    t = np.linspace(0.01, PI / 2, 11)
    a = oracle.legendre_table(40, 40, t)
    b = oracle.legendre_table(40, 40, PI - t)
    l = np.arange(40)[None, :, None]
    m = np.arange(40)[:, None, None]
    np.testing.assert_allclose(b, a * (-1.0) ** (l + m), atol=1e-14)
