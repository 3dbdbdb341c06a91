"""Pins for the oracle's spherical diffusion noise (App. B.7, eq.
spherical_diffusion; Table 1): oracle/noise.py.

Anchors:
* Philox4x64-10 against numpy's own Philox bit generator (a library
  implementation of the same published generator; numpy advances the counter
  before each block);
* the vectorised block function against the scalar one;
* the Box-Muller pairs against the standard normal law (Kolmogorov-Smirnov,
  moments, independence of the pair);
* the F_0 normalisation: the stationary point-wise variance, computed
  numerically from the Legendre table at several rings (not through the
  addition theorem), equals sigma^2 for every length scale of Table 1;
* Monte Carlo: coefficient variances at the stationary start and the lag-one
  autocorrelation phi = e^{-lambda} of the AR(1) process.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import noise as Nz
from oracle.legendre import iter_orders


def test_philox_matches_numpy():
    rng = np.random.default_rng(0)
    for _ in range(5):
        key = [int(v) for v in rng.integers(0, 2 ** 63, 2, dtype=np.uint64)]
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, 4, dtype=np.uint64)]
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        raw = [int(v) for v in bg.random_raw(8)]
        nxt = list(ctr)
        nxt[0] += 1                       # numpy: counter + 1 for the first block
        assert Nz.philox4x64_10(nxt, key) == raw[:4]
        nxt[0] += 1
        assert Nz.philox4x64_10(nxt, key) == raw[4:]


def test_philox_array_matches_scalar():
    rng = np.random.default_rng(1)
    c = [rng.integers(0, 2 ** 64 - 1, 64, dtype=np.uint64, endpoint=True) for _ in range(4)]
    k0, k1 = 0xFFFFFFFFFFFFFFFF, 12345
    got = Nz.philox4x64_10_array(*c, k0, k1)
    for i in range(64):
        ref = Nz.philox4x64_10([int(c[j][i]) for j in range(4)], [k0, k1])
        assert [int(got[j][i]) for j in range(4)] == ref


def test_box_muller_pairs_are_standard_normal():
    idx = np.arange(200_000, dtype=np.uint64)
    er, ei = Nz.normal_pairs(idx, 3, 77)
    for z in (er, ei):
        assert stats.kstest(z, "norm").pvalue > 1e-3
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert abs(np.corrcoef(er, ei)[0, 1]) < 5 / np.sqrt(er.size)
    er2, _ = Nz.normal_pairs(idx, 4, 77)          # another step: fresh draws
    assert abs(np.corrcoef(er, er2)[0, 1]) < 5 / np.sqrt(er.size)


@pytest.mark.parametrize("kT", Nz.TABLE1_KT)
def test_stationary_pointwise_variance_is_sigma_squared(kT):
    """Var z(t) = sum_l E|a_l^0|^2 P^_l^0(t)^2 + sum_{m>=1} 2 E|a_l^m|^2 P^_l^m(t)^2
    with E|a_l^m|^2 = 2 sigma_l^2 / (1 - phi^2), evaluated from the table at
    721-ring nodes, must be sigma^2 at lmax = mmax = 720."""
    lmax, sigma, lam = 720, 1.7, 1.0
    phi, s = Nz.diffusion_params(lmax, kT, lam, sigma)
    th = np.array([0.3, 1.0, np.pi / 2, 2.5])
    x = np.cos(th)
    var = np.zeros_like(th)
    e2 = 2.0 * s ** 2 / (1.0 - phi ** 2)
    for m, rows in iter_orders(lmax, lmax, x, np.sin(th)):
        w = 1.0 if m == 0 else 2.0
        var += w * np.sum(e2[m:, None] * rows ** 2, axis=0)
    np.testing.assert_allclose(var, sigma ** 2, rtol=1e-12)


def test_stationary_start_and_ar1_statistics():
    B, L = 64, 24
    kT = np.array([1.97e-3, 0.126])
    lam = np.array([1.0, 0.5])
    sg = np.array([1.0, 2.0])
    st = Nz.diffusion_step(np.zeros((B, 2, L, L), complex), 0, 5, kT, lam, sg)
    l = np.arange(L)[:, None]
    m = np.arange(L)[None, :]
    live = (l >= 1) & (m <= l)
    for c in range(2):
        phi, s = Nz.diffusion_params(L, kT[c], lam[c], sg[c])
        ratio = np.abs(st[:, c]) ** 2 / (2 * s[:, None] ** 2 / (1 - phi ** 2) + ~live)
        vals = ratio[:, live]
        # m = 0: |a|^2 / E = chi^2_1; m >= 1: chi^2_2 / 2; both have mean 1
        assert abs(vals.mean() - 1) < 5 * vals.std() / np.sqrt(vals.size)
        assert np.all(st[:, c][:, ~live] == 0)
        assert np.all(st[:, c, :, 0].imag == 0)
    # lag-one autocorrelation of the coefficients over 60 steps
    prev = st
    num = np.zeros(2)
    den = np.zeros(2)
    for n in range(1, 61):
        cur = Nz.diffusion_step(prev, n, 5, kT, lam, sg)
        num += np.sum(np.real(np.conj(prev) * cur)[..., live], axis=(0, -1))
        den += np.sum((np.abs(prev) ** 2)[..., live], axis=(0, -1))
        prev = cur
    phi_hat = num / den
    np.testing.assert_allclose(phi_hat, np.exp(-lam), atol=0.01)


def test_field_variance_monte_carlo():
    """The synthesised field of the stationary start has point-wise variance
    sigma^2 (Gauss 32 x 64, lmax = mmax = 32, 256 members, short length
    scale so that points decorrelate)."""
    B, L, nlat, nlon = 256, 32, 32, 64
    st = Nz.diffusion_step(np.zeros((B, 1, L, L), complex), 0, 9, [0.126], [1.0], [1.5])
    z = oracle.isht(st, nlat, nlon, 1)
    v = np.mean(z ** 2, axis=0)                # per grid point over members
    assert abs(v.mean() - 1.5 ** 2) < 0.05 * 1.5 ** 2
