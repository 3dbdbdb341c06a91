"""Pins for the oracle's grids and quadrature weights (App. B.1).

Independent anchors: textbook rules in tests/golden/quadrature_textbook.json,
numpy's Gauss-Legendre routine (a library special case), exact integration of
monomials (the defining property of each rule), symmetry and weight sums.
"""
import json
import os
from math import pi, sqrt  # noqa: F401  (used by eval of golden strings)

import numpy as np
import pytest

import oracle
from oracle import grids

GOLD = os.path.join(os.path.dirname(__file__), "golden", "quadrature_textbook.json")


def _num(v):
    return float(eval(v)) if isinstance(v, str) else float(v)


def _exact_monomial(p):
    # int_{-1}^{1} x^p dx
    return 0.0 if p % 2 else 2.0 / (p + 1)


def test_cc_textbook_values():
    gold = json.load(open(GOLD))["clenshaw_curtis"]
    for n, rule in gold.items():
        _, x = grids.equiangular_nodes(int(n))
        w = grids.clenshaw_curtis_weights(int(n))
        np.testing.assert_allclose(x, [_num(v) for v in rule["x"]], atol=1e-15)
        np.testing.assert_allclose(w, [_num(v) for v in rule["w"]], rtol=1e-14)


@pytest.mark.parametrize("nlat", [3, 5, 17, 33, 64, 181, 721])
def test_cc_exact_to_degree_N(nlat):
    _, x = grids.equiangular_nodes(nlat)
    w = grids.clenshaw_curtis_weights(nlat)
    N = nlat - 1
    for p in range(0, min(N, 60) + 1):
        assert abs(np.dot(w, x ** p) - _exact_monomial(p)) < 1e-13, p
    np.testing.assert_allclose(w, w[::-1], atol=1e-16)
    assert abs(w.sum() - 2.0) < 1e-13
    if N % 2 == 0:
        assert abs(w[0] * (N * N - 1.0) - 1.0) < 1e-13
    else:
        assert abs(w[0] * N * N - 1.0) < 1e-13


def test_cc_not_exact_beyond_degree():
    # a rule on N+1 points with exactness N+1 (odd N+1 is free by symmetry)
    # must fail at degree N+2: guards against a rule that is secretly Gaussian
    nlat = 9
    _, x = grids.equiangular_nodes(nlat)
    w = grids.clenshaw_curtis_weights(nlat)
    assert abs(np.dot(w, x ** (nlat + 1)) - _exact_monomial(nlat + 1)) > 1e-6


def test_gl_textbook_values():
    gold = json.load(open(GOLD))["gauss_legendre"]
    for n, rule in gold.items():
        _, x, w = grids.gauss_legendre(int(n))
        np.testing.assert_allclose(x, [_num(v) for v in rule["x"]], atol=1e-15)
        np.testing.assert_allclose(w, [_num(v) for v in rule["w"]], rtol=1e-14)


@pytest.mark.parametrize("nlat", [1, 2, 7, 32, 64, 360])
def test_gl_matches_numpy_leggauss(nlat):
    xr, wr = np.polynomial.legendre.leggauss(nlat)
    _, x, w = grids.gauss_legendre(nlat)
    # numpy returns ascending nodes; the oracle orders north -> south
    np.testing.assert_allclose(x, xr[::-1], atol=2e-15)
    # numpy's weights lose ~1e-10 relative next to the poles at n = 360
    np.testing.assert_allclose(w, wr[::-1], rtol=2e-10, atol=1e-15)


def test_gl_polar_weights_against_mpmath():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    n = 360
    _, x, w = grids.gauss_legendre(n)
    for i in (0, 1, 7, 179):
        r = mpmath.mpf(x[i])
        for _ in range(6):
            r = r - mpmath.legendre(n, r) / mpmath.diff(lambda t: mpmath.legendre(n, t), r)
        dp = mpmath.diff(lambda t: mpmath.legendre(n, t), r)
        ref = 2 / ((1 - r ** 2) * dp ** 2)
        assert abs(float(r) - x[i]) < 2e-16
        assert abs(float((w[i] - ref) / ref)) < 2e-11


@pytest.mark.parametrize("nlat", [4, 16, 45])
def test_gl_exact_to_degree_2n_minus_1(nlat):
    _, x, w = grids.gauss_legendre(nlat)
    for p in range(0, 2 * nlat):
        assert abs(np.dot(w, x ** p) - _exact_monomial(p)) < 1e-13, p
    if nlat <= 8:  # the degree-2n error term shrinks like 4^-n
        assert abs(np.dot(w, x ** (2 * nlat)) - _exact_monomial(2 * nlat)) > 1e-6


def test_trapezoid_weights_formula_properties():
    # eq. latlon_quad_weights: sin t dt, summing only approximately to 2
    for nlat in (9, 65, 721):
        th, _ = grids.equiangular_nodes(nlat)
        w = grids.trapezoid_weights(nlat)
        assert w[0] == 0.0 and abs(w[-1]) < 1e-15
        # the composite trapezoid rule for sin on [0, pi] equals
        # (pi/N) cot(pi/(2N)); N = nlat - 1
        N = nlat - 1
        assert abs(w.sum() - (pi / N) / np.tan(pi / (2 * N))) < 1e-12
        assert abs(w.sum() - 2.0) < 1e-1


def test_equiangular_nodes_include_both_poles():
    th, x = grids.equiangular_nodes(721)
    assert th[0] == 0.0 and abs(th[-1] - pi) < 1e-15
    assert abs(th[360] - pi / 2) < 1e-15
    assert x[0] == 1.0 and x[-1] == -1.0


def test_grid_dispatch():
    for kind in (0, 1, 2):
        th, x, w = oracle.grid(9, kind)
        assert th.shape == x.shape == w.shape == (9,)
    with pytest.raises(ValueError):
        oracle.grid(9, 7)
