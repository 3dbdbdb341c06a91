"""Pins for the oracle's isotropic spectral filter (App. B.4, eq.
s2_spectral_conv, one filter k[c, l] per channel): oracle/mix.py.

Anchors: the channel mix with diagonal per-degree weights (pinned on its
own); the diagonal of the channel mix's weight gradient; the adjoint dot
product; and the convolution theorem on a closed form, the heat kernel
k^_l = exp(-l (l + 1) t), which scales a single harmonic of degree l0 by
exp(-l0 (l0 + 1) t) on the grid.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.legendre import iter_orders


def _k(seed, C, L):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((C, L)) + 1j * rng.standard_normal((C, L))


def test_filter_is_a_diagonal_channel_mix():
    B, C, L, M = 2, 5, 12, 9
    x = synth.coefficients(1, B, C, L, M)
    k = _k(2, C, L)
    W = np.zeros((L, C, C), complex)
    for l in range(L):
        W[l] = np.diag(k[:, l])
    np.testing.assert_allclose(oracle.isotropic_filter(x, k), oracle.channel_mix(x, W), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(oracle.isotropic_filter_T(x, k), oracle.channel_mix_T(x, W), rtol=1e-14, atol=1e-15)


def test_filter_gradient_is_the_diagonal_of_the_mix_gradient():
    B, C, L, M = 3, 4, 10, 7
    g = synth.coefficients(3, B, C, L, M)
    x = synth.coefficients(4, B, C, L, M)
    dW = oracle.channel_mix_dW(g, x)
    dk = oracle.isotropic_filter_dk(g, x)
    np.testing.assert_allclose(dk, np.stack([np.diag(dW[l]) for l in range(L)], axis=1), rtol=1e-13, atol=1e-15)


def test_filter_adjoint_dot_product():
    B, C, L, M = 2, 3, 11, 11
    x = synth.coefficients(5, B, C, L, M)
    g = synth.coefficients(6, B, C, L, M)
    k = _k(7, C, L)
    lhs = np.sum(np.real(np.conj(oracle.isotropic_filter(x, k)) * g))
    rhs = np.sum(np.real(np.conj(x) * oracle.isotropic_filter_T(g, k)))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("l0,m0", [(2, 0), (5, 3), (9, 9)])
def test_heat_kernel_convolution_theorem(l0, m0):
    nlat, nlon, L, t = 16, 32, 12, 0.01
    th, x, _ = oracle.grid(nlat, 1)
    rows = dict(iter_orders(L, L, x, np.sin(th)))[m0]
    p = 2 * np.pi * np.arange(nlon) / nlon
    u = rows[l0 - m0][:, None] * np.cos(m0 * p)[None, :]
    l = np.arange(L)
    k = np.exp(-l * (l + 1.0) * t)[None, :]
    v = oracle.isht(oracle.isotropic_filter(oracle.sht(u[None, None], L, L, 1), k), nlat, nlon, 1)[0, 0]
    np.testing.assert_allclose(v, np.exp(-l0 * (l0 + 1.0) * t) * u, atol=1e-13)
