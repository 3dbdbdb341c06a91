"""Pins for the oracle's SHT / ISHT / adjoints / channel mix (App. B.3-B.4).

Anchors, none of which re-types the oracle's formula:
* closed-form coefficients of low-degree fields (tests/golden/
  closed_form_coefficients.json, worked by hand from eq. sht);
* analysis after synthesis is the identity on Gauss-Legendre grids with
  lmax <= nlat (exactness to degree 2 nlat - 1, App. B.1), and on the
  pole-inclusive Clenshaw-Curtis grid with band limit lmax <= (nlat+1)/2;
* Parseval on Gauss-Legendre grids;
* the literal quadruple sums of eq. sht and eq. isht (over -l <= m <= l) on
  tiny grids;
* the DFT shift theorem in longitude;
* dot-product tests and dense explicit transposes for the adjoints;
* the chain rule against central finite differences;
* planted mistakes (a dropped weight, a wrong sign, a missing c_m, a wrong
  normalisation) that each fail at least one of the pins above.
"""
import json
import os
from math import pi, sqrt  # noqa: F401  (eval of golden strings)

import numpy as np
import pytest

import oracle
import synth
from oracle import transforms as T

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_form_coefficients.json")


def _fields(th, nlon):
    p = 2 * np.pi * np.arange(nlon) / nlon
    c, s = np.cos(th)[:, None], np.sin(th)[:, None]
    one = np.ones((th.size, nlon))
    return {
        "one": one,
        "cos_t": c * one,
        "sin_t_cos_p": s * np.cos(p)[None, :],
        "sin_t_sin_p": s * np.sin(p)[None, :],
        "3cos2_t_minus_1": (3 * c * c - 1) * one,
    }


@pytest.mark.parametrize("kind,nlat,nlon", [(1, 8, 16), (0, 9, 16), (1, 32, 64), (0, 33, 64)])
def test_closed_form_coefficients(kind, nlat, nlon):
    gold = json.load(open(GOLD))["fields"]
    th, _, _ = oracle.grid(nlat, kind)
    L = 4
    for name, u in _fields(th, nlon).items():
        a = oracle.sht(u, L, L, kind)
        ref = np.zeros((L, L), dtype=complex)
        g = gold[name]
        ref[g["l"], g["m"]] = eval(g["re"]) + 1j * eval(g["im"])
        np.testing.assert_allclose(a, ref, atol=1e-14, err_msg=name)


@pytest.mark.parametrize("nlat,nlon,L", [(8, 16, 8), (32, 64, 32), (45, 96, 40), (32, 64, 17)])
def test_gauss_round_trip_is_identity(nlat, nlon, L):
    a = synth.coefficients(0, 2, 3, L, L)
    u = oracle.isht(a, nlat, nlon, 1)
    np.testing.assert_allclose(oracle.sht(u, L, L, 1), a, atol=1e-13)
    # and synthesis after analysis on the band-limited field
    np.testing.assert_allclose(oracle.isht(oracle.sht(u, L, L, 1), nlat, nlon, 1), u, atol=1e-13)


@pytest.mark.parametrize("nlat,nlon", [(33, 64), (65, 128), (181, 360)])
def test_cc_round_trip_within_exactness(nlat, nlon):
    L = (nlat + 1) // 2
    a = synth.coefficients(1, 1, 2, L, L)
    u = oracle.isht(a, nlat, nlon, 0)
    np.testing.assert_allclose(oracle.sht(u, L, L, 0), a, atol=1e-13)


def test_cc_round_trip_beyond_exactness_is_not_identity():
    # Clenshaw-Curtis on nlat rings integrates P^_l P^_l' exactly only for
    # l + l' <= nlat - 1; at lmax = nlat - 1 the round trip is visibly inexact
    nlat, nlon, L = 33, 64, 32
    a = synth.coefficients(1, 1, 2, L, L)
    b = oracle.sht(oracle.isht(a, nlat, nlon, 0), L, L, 0)
    assert np.linalg.norm(b - a) / np.linalg.norm(a) > 1e-4


@pytest.mark.parametrize("nlat,nlon,L", [(16, 32, 16), (24, 50, 20)])
def test_parseval_gauss(nlat, nlon, L):
    a = synth.coefficients(2, 1, 2, L, L)
    u = oracle.isht(a, nlat, nlon, 1)
    _, _, w = oracle.grid(nlat, 1)
    lhs = np.sum((2 * np.pi / nlon) * w[None, :, None] * u[0] ** 2, axis=(-2, -1))
    cm = np.full(L, 2.0)
    cm[0] = 1.0
    rhs = np.sum(cm[None, None, :] * np.abs(a[0]) ** 2, axis=(-2, -1))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)


@pytest.mark.parametrize("kind,nlat,nlon,L,M", [(1, 6, 12, 5, 4), (0, 7, 12, 4, 4), (2, 5, 10, 3, 3)])
def test_bruteforce_sums(kind, nlat, nlon, L, M):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((2, nlat, nlon))
    np.testing.assert_allclose(oracle.sht(u, L, M, kind), oracle.sht_bruteforce(u, L, M, kind), atol=1e-14)
    a = synth.coefficients(3, 1, 2, L, M)
    a[..., 0] += 1j * 0.5  # imaginary m = 0 parts must be ignored by both
    np.testing.assert_allclose(oracle.isht(a, nlat, nlon, kind), oracle.isht_bruteforce(a, nlat, nlon, kind),
                               atol=1e-14)


def test_longitude_shift_theorem():
    nlat, nlon, L = 12, 24, 10
    rng = np.random.default_rng(5)
    u = rng.standard_normal((nlat, nlon))
    a = oracle.sht(u, L, L, 1)
    b = oracle.sht(np.roll(u, 1, axis=-1), L, L, 1)
    m = np.arange(L)
    np.testing.assert_allclose(b, a * np.exp(-2j * np.pi * m / nlon)[None, :], atol=1e-14)


def _rdot(a, b):
    return float(np.sum(np.real(np.conj(a) * b)))


@pytest.mark.parametrize("kind,nlat,nlon,L,M", [(1, 16, 32, 16, 16), (0, 17, 32, 16, 12), (2, 9, 20, 7, 5)])
def test_adjoint_dot_products(kind, nlat, nlon, L, M):
    rng = np.random.default_rng(11)
    u = rng.standard_normal((2, nlat, nlon))
    g = rng.standard_normal((2, L, M)) + 1j * rng.standard_normal((2, L, M))
    # <SHT u, g> = <u, SHT^T g>
    assert abs(_rdot(oracle.sht(u, L, M, kind), g) - _rdot(u, oracle.sht_T(g, nlat, nlon, kind))) < 1e-12
    # <ISHT g, u> = <g, ISHT^T u>
    assert abs(_rdot(oracle.isht(g, nlat, nlon, kind), u) - _rdot(g, oracle.isht_T(u, L, M, kind))) < 1e-12


def _dense_real_matrix(fn, n_in, in_complex, in_shape):
    cols = []
    for i in range(n_in * (2 if in_complex else 1)):
        e = np.zeros(n_in * (2 if in_complex else 1))
        e[i] = 1.0
        if in_complex:
            v = (e[:n_in] + 1j * e[n_in:]).reshape(in_shape)
        else:
            v = e.reshape(in_shape)
        out = fn(v)
        if np.iscomplexobj(out):
            out = np.concatenate([out.real.ravel(), out.imag.ravel()])
        cols.append(out.ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("kind", [0, 1])
def test_adjoints_equal_explicit_transposes(kind):
    nlat, nlon, L, M = 6, 12, 5, 4
    A = _dense_real_matrix(lambda v: oracle.sht(v, L, M, kind), nlat * nlon, False, (nlat, nlon))
    AT = _dense_real_matrix(lambda v: oracle.sht_T(v, nlat, nlon, kind), L * M, True, (L, M))
    np.testing.assert_allclose(AT, A.T, atol=1e-14)
    B = _dense_real_matrix(lambda v: oracle.isht(v, nlat, nlon, kind), L * M, True, (L, M))
    BT = _dense_real_matrix(lambda v: oracle.isht_T(v, L, M, kind), nlat * nlon, False, (nlat, nlon))
    np.testing.assert_allclose(BT, B.T, atol=1e-14)


def test_channel_mix_pins():
    B, C, L, M = 2, 5, 6, 4
    x = synth.coefficients(4, B, C, L, M)
    # W_l = s_l * I scales degree l by s_l (the isotropic filter of eq. s2_spectral_conv)
    s = np.arange(1, L + 1) * (1 + 0.5j)
    W = s[:, None, None] * np.eye(C)[None]
    np.testing.assert_allclose(oracle.channel_mix(x, W), x * s[None, None, :, None], atol=1e-15)
    # a channel permutation permutes channels
    perm = np.array([2, 0, 4, 1, 3])
    Wp = np.repeat(np.eye(C)[perm][None], L, axis=0)
    np.testing.assert_allclose(oracle.channel_mix(x, Wp), x[:, perm], atol=0)
    # dot test for the adjoint
    W = synth.mix_weights(5, L, C)
    g = synth.coefficients(6, B, C, L, M)
    assert abs(_rdot(oracle.channel_mix(x, W), g) - _rdot(x, oracle.channel_mix_T(g, W))) < 1e-12


def test_chain_gradient_against_finite_differences():
    # L(x) = <r, ISHT(mix(SHT(x)))>; its gradient by the adjoints
    # SHT^T(mix^T(ISHT^T(r))) against central differences (h = 1e-3)
    nlat, nlon, Lm, B, C = 12, 24, 12, 2, 3
    rng = np.random.default_rng(9)
    x = rng.standard_normal((B, C, nlat, nlon))
    r = rng.standard_normal((B, C, nlat, nlon))
    W = synth.mix_weights(4, Lm, C)

    def loss(v):
        return float(np.sum(r * oracle.isht(oracle.channel_mix(oracle.sht(v, Lm, Lm, 1), W), nlat, nlon, 1)))

    grad = oracle.sht_T(oracle.channel_mix_T(oracle.isht_T(r, Lm, Lm, 1), W), nlat, nlon, 1)
    h = 1e-3
    for i in range(6):
        v = rng.standard_normal(x.shape)
        fd = (loss(x + h * v) - loss(x - h * v)) / (2 * h)
        assert abs(fd - np.sum(grad * v)) <= 1e-9 * np.linalg.norm(grad) * np.linalg.norm(v)


def test_channel_mix_weight_gradient_pins():
    """dW = channel_mix_dW(g, x) pinned without its own matrix products:
    (a) the exact directional derivative of the linear loss
    L(W) = Re <G, mix_W(x)> along V equals Re <dW, V> (the forward mix is a
    separate code path); (b) brute-force loops on a tiny case; (c) entries
    with m > l (where the filter does not act) contribute nothing."""
    B, C, L, M = 2, 4, 6, 5
    x = synth.coefficients(11, B, C, L, M)            # zero for l < m
    G = synth.coefficients(12, B, C, L, M)
    dW = oracle.channel_mix_dW(G, x)
    rng = np.random.default_rng(13)
    for _ in range(4):
        V = rng.standard_normal((L, C, C)) + 1j * rng.standard_normal((L, C, C))
        assert abs(_rdot(G, oracle.channel_mix(x, V)) - _rdot(dW, V)) < 1e-12
    ref = np.zeros((L, C, C), complex)
    for l in range(L):
        for co in range(C):
            for ci in range(C):
                for b in range(B):
                    for m in range(min(l + 1, M)):
                        ref[l, co, ci] += G[b, co, l, m] * np.conj(x[b, ci, l, m])
    np.testing.assert_allclose(dW, ref, atol=1e-13)
    x2, G2 = x.copy(), G.copy()
    for l in range(L):
        x2[:, :, l, l + 1:] = 7.0 + 3.0j
        G2[:, :, l, l + 1:] = -5.0 + 1.0j
    np.testing.assert_allclose(oracle.channel_mix_dW(G2, x2), dW, atol=0)


def test_weight_gradient_pins_catch_planted_mistakes():
    """Plausible mistakes in the weight gradient, planted in copies on the
    CPU: each must break the directional-derivative identity or the mask."""
    B, C, L, M = 2, 3, 5, 4
    x = synth.coefficients(31, B, C, L, M)
    G = synth.coefficients(32, B, C, L, M)
    rng = np.random.default_rng(33)
    V = rng.standard_normal((L, C, C)) + 1j * rng.standard_normal((L, C, C))
    x2, G2 = x.copy(), G.copy()
    for l in range(L):
        x2[:, :, l, l + 1:] = 2.0 - 1.0j
        G2[:, :, l, l + 1:] = 1.0 + 4.0j

    def all_m(g, xx):  # no m <= l restriction
        return np.einsum("bclm,bdlm->lcd", g, np.conj(xx))

    def m_below_l(g, xx):  # m < l instead of m <= l
        out = np.zeros((L, C, C), complex)
        for l in range(L):
            out[l] = np.einsum("bcm,bdm->cd", g[:, :, l, :min(l, M)], np.conj(xx[:, :, l, :min(l, M)]))
        return out

    wrong = {
        "conj on g": lambda g, xx: np.conj(oracle.channel_mix_dW(g, xx)),
        "transposed": lambda g, xx: np.transpose(oracle.channel_mix_dW(g, xx), (0, 2, 1)),
        "all m": all_m,
        "m < l": m_below_l,
    }
    for name, f in wrong.items():
        identity = abs(_rdot(G, oracle.channel_mix(x, V)) - _rdot(f(G, x), V)) < 1e-12
        masked = np.allclose(f(G2, x2), f(G, x))
        assert not (identity and masked), name


def test_weight_gradient_of_the_chain_against_finite_differences():
    # L(W) = <r, ISHT(mix_W(SHT(x)))>: dL/dW = channel_mix_dW(ISHT^T(r), SHT(x))
    # in PyTorch's convention (dL/dRe W + i dL/dIm W), against central
    # differences along random complex directions (h = 1e-3; L is linear in W)
    nlat, nlon, Lm, B, C = 12, 24, 12, 2, 3
    rng = np.random.default_rng(21)
    x = rng.standard_normal((B, C, nlat, nlon))
    r = rng.standard_normal((B, C, nlat, nlon))
    W = synth.mix_weights(4, Lm, C)
    xh = oracle.sht(x, Lm, Lm, 1)

    def loss(Wv):
        return float(np.sum(r * oracle.isht(oracle.channel_mix(xh, Wv), nlat, nlon, 1)))

    dW = oracle.channel_mix_dW(oracle.isht_T(r, Lm, Lm, 1), xh)
    h = 1e-3
    for _ in range(6):
        V = rng.standard_normal(W.shape) + 1j * rng.standard_normal(W.shape)
        fd = (loss(W + h * V) - loss(W - h * V)) / (2 * h)
        assert abs(fd - _rdot(dW, V)) <= 1e-9 * np.linalg.norm(dW) * np.linalg.norm(V)


def test_input_validation():
    u = np.zeros((8, 16))
    with pytest.raises(ValueError):
        oracle.sht(u, 4, 9, 1)   # mmax > nlon/2
    with pytest.raises(ValueError):
        oracle.sht(u, 3, 4, 1)   # mmax > lmax


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by at least one pin above
# ---------------------------------------------------------------------------

def _pins_pass():
    """A compact subset of the pins above; True when all hold."""
    try:
        test_closed_form_coefficients(1, 8, 16)
        test_closed_form_coefficients(0, 9, 16)
        test_gauss_round_trip_is_identity(8, 16, 8)
        test_adjoint_dot_products(1, 16, 32, 16, 16)
        test_bruteforce_sums(1, 6, 12, 5, 4)
        test_longitude_shift_theorem()
    except AssertionError:
        return False
    return True


def test_pins_pass_unmodified():
    assert _pins_pass()


@pytest.mark.parametrize("mutation", ["drop_weight", "wrong_phase", "no_cm", "wrong_norm",
                                      "transposed_dft_sign", "sht_T_cm"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "drop_weight":
        orig = T.grid
        monkeypatch.setattr(T, "grid", lambda n, k: (lambda t: (t[0], t[1], np.ones_like(t[2]) * 2 / n))(orig(n, k)))
    elif mutation == "wrong_phase":
        orig = T.iter_orders

        def flipped(lmax, mmax, x, s):
            for m, rows in orig(lmax, mmax, x, s):
                yield m, rows * (-1.0) ** m
        monkeypatch.setattr(T, "iter_orders", flipped)
    elif mutation == "no_cm":
        monkeypatch.setattr(T, "_ring_synth", lambda Y, nlon, c: nlon * np.fft.irfft(
            np.concatenate([Y, np.zeros(Y.shape[:-1] + (nlon // 2 + 1 - Y.shape[-1],))], -1) * 0.5, n=nlon))
    elif mutation == "wrong_norm":
        orig = T._ring_dft
        monkeypatch.setattr(T, "_ring_dft", lambda u, mmax: orig(u, mmax) / u.shape[-1])
    elif mutation == "transposed_dft_sign":
        monkeypatch.setattr(T, "_ring_dft", lambda u, mmax: np.conj(np.fft.rfft(u, axis=-1)[..., :mmax]))
    elif mutation == "sht_T_cm":
        orig = T._ring_synth
        monkeypatch.setattr(T, "_ring_synth", lambda Y, nlon, c: orig(Y, nlon, 2.0))
    assert not _pins_pass()
