"""Pins for the oracle's ensemble scores and spectra (App. D.4, App. E.1,
App. F.7): oracle/scores.py.

Anchors, none of which re-types the formula under test:
* three independently written forms of the ensemble CRPS (the exact
  integral of eq. crps, the rank form eq. ensemble_crps_cdf and the
  spread-skill form eq. spread_skill_crps) agree on random ensembles with
  ties;
* worked examples (tests/golden/crps_examples.json), the single-member
  reduction to the absolute error and the two-member fair-CRPS property the
  paper states;
* the closed-form CRPS of a Gaussian forecast (Gneiting & Raftery): the fair
  CRPS of N-member ensembles drawn from it is unbiased, the biased form
  exceeds it by 1/(N sqrt(pi));
* the spectral loss against a brute-force sum over explicit negative orders
  built from the real-field symmetry;
* Parseval for the angular PSD on Gauss-Legendre grids and closed forms for
  single harmonics; closed forms and per-ring Parseval for the zonal PSD;
* planted mistakes that each fail one of the pins.
"""
import json
import os

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import synth
from oracle import scores as S
from oracle.legendre import iter_orders

GOLD = os.path.join(os.path.dirname(__file__), "golden", "crps_examples.json")


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_three_crps_forms_agree(n):
    rng = np.random.default_rng(n)
    ens = rng.standard_normal((n, 500))
    obs = rng.standard_normal(500)
    # ties: members equal to each other and to the observation
    if n >= 3:
        ens[1, :50] = ens[0, :50]
        ens[2, 50:100] = obs[50:100]
    a = S.crps_integral(ens, obs)
    b = S.crps_sorted(ens, obs)
    c = S.crps_spread_skill(ens, obs)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(c, a, rtol=1e-12, atol=1e-14)


def test_crps_worked_examples():
    for case in json.load(open(GOLD))["cases"]:
        ens = np.array(case["ens"])[:, None]
        obs = np.array([case["obs"]])
        for f in (S.crps_integral, S.crps_sorted, S.crps_spread_skill):
            assert f(ens, obs)[0] == pytest.approx(case["crps"], abs=1e-15)
        if case["fcrps"] is not None:
            assert S.crps_spread_skill(ens, obs, fair=True)[0] == pytest.approx(case["fcrps"], abs=1e-15)


def test_single_member_is_absolute_error_and_fair_two_member_property():
    rng = np.random.default_rng(3)
    u, y = rng.standard_normal((1, 100)), rng.standard_normal(100)
    np.testing.assert_allclose(S.crps_integral(u, y), np.abs(u[0] - y), rtol=1e-14)
    u2 = np.stack([y, rng.standard_normal(100) * 1e3])
    np.testing.assert_allclose(S.crps_spread_skill(u2, y, fair=True), 0.0, atol=1e-12)


@pytest.mark.parametrize("y", [-1.3, 0.0, 0.7, 2.5])
def test_gaussian_closed_form_bias(y):
    """CRPS(N(0,1), y) = y (2 Phi(y) - 1) + 2 phi(y) - 1/sqrt(pi).  Over many
    independent 4-member ensembles the fair form averages to it and the
    biased form to it plus 1/(4 sqrt(pi)) (E|U - U'| = 2/sqrt(pi))."""
    n, trials = 4, 400_000
    rng = np.random.default_rng(11)
    ens = rng.standard_normal((n, trials))
    obs = np.full(trials, y)
    exact = y * (2 * norm.cdf(y) - 1) + 2 * norm.pdf(y) - 1 / np.sqrt(np.pi)
    fair = S.crps_spread_skill(ens, obs, fair=True)
    biased = S.crps_spread_skill(ens, obs)
    se = 5 * fair.std() / np.sqrt(trials)
    assert abs(fair.mean() - exact) < se
    assert abs(biased.mean() - (exact + 1 / (n * np.sqrt(np.pi)))) < 5 * biased.std() / np.sqrt(trials)


def _full_orders(a):
    """Coefficients for -l <= m <= l from the stored m >= 0 of a real field:
    u^_l^{-m} = (-1)^m conj(u^_l^m).  Returns a dict m -> [..., lmax]."""
    mmax = a.shape[-1]
    out = {}
    for m in range(mmax):
        out[m] = a[..., m]
        if m > 0:
            out[-m] = (-1) ** m * np.conj(a[..., m])
    return out


@pytest.mark.parametrize("fair", [False, True])
def test_spectral_crps_against_explicit_negative_orders(fair):
    nlat, L, M, N = 16, 12, 9, 5
    ens = np.stack([synth.coefficients(20 + e, 1, 2, L, M) for e in range(N)])      # [N, 1, 2, L, M]
    obs = synth.coefficients(30, 1, 2, L, M)
    got = S.spectral_crps(ens, obs, nlat, fair=fair)
    fe, fo = _full_orders(ens), _full_orders(obs)
    ref = np.zeros(obs.shape[:-2])
    for l in range(1, min(L - 1, nlat // 2) + 1):
        for m in range(-min(l, M - 1), min(l, M - 1) + 1):
            ref += S.crps_integral(fe[m][..., l].real, fo[m][..., l].real) if not fair else \
                S.crps_spread_skill(fe[m][..., l].real, fo[m][..., l].real, fair=True)
            ref += S.crps_integral(fe[m][..., l].imag, fo[m][..., l].imag) if not fair else \
                S.crps_spread_skill(fe[m][..., l].imag, fo[m][..., l].imag, fair=True)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_spectral_crps_degenerate_cases():
    L, M = 10, 10
    obs = synth.coefficients(1, 1, 3, L, M)
    same = np.stack([obs, obs, obs])
    np.testing.assert_allclose(S.spectral_crps(same, obs, 20), 0.0, atol=1e-15)
    one = synth.coefficients(2, 1, 3, L, M)[None]
    d = one[0] - obs
    l = np.arange(L)[:, None]
    m = np.arange(M)[None, :]
    w = np.where((l >= 1) & (l <= 9) & (m <= l), np.where(m == 0, 1.0, 2.0), 0.0)
    ref = np.sum(w * (np.abs(d.real) + np.abs(d.imag)), axis=(-2, -1))
    np.testing.assert_allclose(S.spectral_crps(one, obs, 20), ref, rtol=1e-13)
    # degree range: l <= nlat // 2 (nlat = 8 -> l <= 4), l = 0 never counted
    w4 = np.where((l >= 1) & (l <= 4) & (m <= l), np.where(m == 0, 1.0, 2.0), 0.0)
    np.testing.assert_allclose(S.spectral_crps(one, obs, 8), np.sum(w4 * (np.abs(d.real) + np.abs(d.imag)),
                                                                   axis=(-2, -1)), rtol=1e-13)


@pytest.mark.parametrize("kind", [0, 1])
def test_spatial_crps_of_constant_fields(kind):
    """Constant members and observation: the sphere average of a constant
    CRPS is that CRPS (the weights integrate 1 over the sphere to 4 pi)."""
    nlat, nlon = 17, 32
    vals = np.array([0.3, -1.0, 2.0])
    ens = vals[:, None, None] * np.ones((3, nlat, nlon))
    obs = 0.5 * np.ones((nlat, nlon))
    ref = S.crps_integral(vals[:, None], np.array([0.5]))[0]
    assert S.spatial_crps(ens, obs, kind) == pytest.approx(ref, rel=1e-13)


def test_psd_parseval_gauss():
    """sum_l PSD(l) = integral of u^2 over the sphere for band-limited fields
    on a Gauss-Legendre grid (exact quadrature)."""
    nlat, nlon, L = 24, 48, 24
    a = synth.coefficients(5, 2, 3, L, L)
    u = oracle.isht(a, nlat, nlon, 1)
    _, _, w = oracle.grid(nlat, 1)
    integral = np.sum(u ** 2 * ((2 * np.pi / nlon) * w)[:, None], axis=(-2, -1))
    np.testing.assert_allclose(S.psd(a).sum(-1), integral, rtol=1e-12)


@pytest.mark.parametrize("l0,m0", [(0, 0), (3, 0), (3, 2), (7, 7)])
def test_psd_single_harmonic(l0, m0):
    """u = P^_l0^m0(cos t) cos(m0 p): PSD(l0) = 1 for m0 = 0 and 1/2 for
    m0 >= 1 (the integral of u^2), zero at every other degree."""
    nlat, nlon, L = 16, 32, 12
    th, x, _ = oracle.grid(nlat, 1)
    rows = dict(iter_orders(L, L, x, np.sin(th)))[m0]
    p = 2 * np.pi * np.arange(nlon) / nlon
    u = rows[l0 - m0][:, None] * np.cos(m0 * p)[None, :]
    spec = S.psd(oracle.sht(u, L, L, 1))
    ref = np.zeros(L)
    ref[l0] = 1.0 if m0 == 0 else 0.5
    np.testing.assert_allclose(spec, ref, atol=1e-13)


def test_zonal_psd_closed_forms_and_ring_parseval():
    nlat, nlon, M = 9, 24, 12
    th, _, _ = oracle.grid(nlat, 0)
    p = 2 * np.pi * np.arange(nlon) / nlon
    # cos(3 p) on every ring: the longitude integral is pi at m = 3
    z = S.zonal_psd(np.cos(3 * p)[None, :] * np.ones((nlat, 1)), 0, M)
    ref = np.zeros((nlat, M))
    ref[:, 3] = 2 * np.pi * np.sin(th) * np.pi ** 2
    np.testing.assert_allclose(z, ref, atol=1e-12)
    # a constant: (2 pi)^2 at m = 0
    z = S.zonal_psd(np.ones((nlat, nlon)), 0, M)
    np.testing.assert_allclose(z[:, 0], 2 * np.pi * np.sin(th) * (2 * np.pi) ** 2, rtol=1e-13)
    # per ring: integral of u^2 dp = (1/2pi) (|I_0|^2 + 2 sum_{m>=1} |I_m|^2)
    # for a field without a Nyquist component (mmax = nlon / 2)
    rng = np.random.default_rng(1)
    X = np.fft.rfft(rng.standard_normal((nlat, nlon)), axis=-1)
    X[:, nlon // 2] = 0
    u = np.fft.irfft(X, n=nlon, axis=-1)
    z = S.zonal_psd(u, 0, nlon // 2)
    inner = np.where(np.sin(th) > 0, 1.0, 0.0)
    lhs = np.sum(u ** 2, axis=-1) * (2 * np.pi / nlon)
    rhs = (z[:, 0] + 2 * z[:, 1:].sum(-1)) / (2 * np.pi * np.maximum(np.sin(th), 1e-300)) / (2 * np.pi)
    np.testing.assert_allclose(rhs * inner, lhs * inner, rtol=1e-12)


def test_planted_mistakes_are_caught():
    cases = json.load(open(GOLD))["cases"]
    ens = np.array(cases[3]["ens"])[:, None]
    obs = np.array([cases[3]["obs"]])

    def fair_with_biased_denominator(e, o):
        n = e.shape[0]
        return np.mean(np.abs(e - o[None]), 0) - sum(np.sum(np.abs(e[i][None] - e), 0) for i in range(n)) / (2 * n * n)

    assert fair_with_biased_denominator(ens, obs)[0] != pytest.approx(cases[3]["fcrps"])

    def sorted_with_swapped_weights(e, o):
        n = e.shape[0]
        s = np.sort(e, 0)
        k = np.arange(1, n + 1)[:, None]
        below = s <= o[None]
        return np.sum(np.where(below, (2 * n + 1 - 2 * k) / n ** 2 * (o[None] - s), (2 * k - 1) / n ** 2 * (s - o[None])), 0)

    assert sorted_with_swapped_weights(ens, obs)[0] != pytest.approx(cases[3]["crps"])
    # a PSD without the multiplicity 2 of m >= 1 breaks Parseval
    nlat, nlon, L = 16, 32, 16
    a = synth.coefficients(5, 1, 1, L, L)
    u = oracle.isht(a, nlat, nlon, 1)
    _, _, w = oracle.grid(nlat, 1)
    integral = np.sum(u ** 2 * ((2 * np.pi / nlon) * w)[:, None])
    assert not np.isclose(np.sum(np.abs(a) ** 2), integral, rtol=1e-6)


@pytest.mark.parametrize("fair", [False, True])
def test_crps_gradients_against_central_differences(fair):
    """The scores are piecewise linear in the members: central differences
    with a step far below the gap to the nearest kink are exact up to
    rounding."""
    nlat, L, M, N = 12, 8, 6, 4
    rng = np.random.default_rng(7)
    ens = np.stack([synth.coefficients(40 + e, 1, 2, L, M) for e in range(N)])
    obs = synth.coefficients(50, 1, 2, L, M)
    g = S.spectral_crps_grad(ens, obs, nlat, fair=fair)
    h = 1e-7
    for _ in range(12):
        idx = (int(rng.integers(N)), 0, int(rng.integers(2)), int(rng.integers(1, L)), int(rng.integers(M)))
        for part in (1.0, 1j):
            d = np.zeros_like(ens)
            d[idx] = part * h
            fd = (S.spectral_crps(ens + d, obs, nlat, fair).sum() - S.spectral_crps(ens - d, obs, nlat, fair).sum()) / (2 * h)
            ref = g[idx].real if part == 1.0 else g[idx].imag
            assert fd == pytest.approx(ref, abs=1e-6)
    nlon = 16
    ens_g = rng.standard_normal((N, 2, nlat, nlon))
    obs_g = rng.standard_normal((2, nlat, nlon))
    gg = S.spatial_crps_grad(ens_g, obs_g, 0, fair)
    for _ in range(12):
        idx = tuple(int(rng.integers(s)) for s in ens_g.shape)
        d = np.zeros_like(ens_g)
        d[idx] = h
        fd = (S.spatial_crps(ens_g + d, obs_g, 0, fair).sum() - S.spatial_crps(ens_g - d, obs_g, 0, fair).sum()) / (2 * h)
        assert fd == pytest.approx(gg[idx], abs=1e-8)
