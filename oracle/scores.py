"""Ensemble scores and spectra on the sphere (oracle, FP64; test infrastructure only).

* CRPS of a real observable against an ensemble (App. D.4):
  - ``crps_integral``: the definition eq. crps, the integral over the real
    line of (F_ens(u) - 1(u* <= u))^2 with the ensemble's empirical CDF,
    evaluated exactly (the integrand is piecewise constant between the
    sorted members and the observation);
  - ``crps_sorted``: the rank form eq. ensemble_crps_cdf on the sorted
    members, with weights (2e - 1)/N^2 below the observation and
    (2N + 1 - 2e)/N^2 above it;
  - ``crps_spread_skill``: eq. spread_skill_crps, the mean absolute error of
    the members minus half the mean absolute difference of all member pairs;
    with ``fair=True`` the pair sum is divided by 2N(N-1) instead of 2N^2
    (eq. fair_spread_skill_crps).
* ``spectral_crps``: the spectral loss term eq. spectral_loss (App. E.1): the
  CRPS of every spherical harmonic coefficient over the ensemble, summed over
  degrees 1 <= l <= l_hi and orders |m| <= l.
* ``spatial_crps``: the spatial loss term eq. spatial_loss: the point-wise
  CRPS averaged over the sphere, (1/4 pi) times the quadrature sum with
  weights (2 pi / nlon) w_k (App. B.1).
* ``psd``: the angular power spectral density eq. psd (App. F.7),
  PSD(l) = sum over |m| <= l of |u^_l^m|^2.
* ``zonal_psd``: eq. zonal_psd, 2 pi sin(t) |integral of u e^{-i m p} dp|^2
  at every ring, the integral taken as the longitude quadrature sum
  (2 pi / nlon) sum_j.
* ``*_grad``: derivatives of the spread-skill CRPS and of both loss terms
  with respect to the members (each |.| differentiated as sign(.), with
  sign(0) = 0), for the backward pass of a training loss.

Readings of the paper (where it is silent or garbled):
* A spectral coefficient is complex; its CRPS is that of its real part plus
  that of its imaginary part (two real marginals).  m = 0 coefficients of
  real fields have a zero imaginary part, which adds nothing.
* Negative orders of a real field satisfy u^_l^{-m} = (-1)^m conj(u^_l^m);
  the sign flips the observation and every member alike and CRPS is
  invariant under u -> -u, so the sum over |m| <= l counts each stored order
  m >= 1 twice and m = 0 once (the multiplicity weighting the paper
  describes).  The same holds for |u^|^2 in the PSD.
* The printed degree range of the spectral loss is 1 <= l <= nlat/2; with
  counts lmax (l < lmax) it is l = 1 .. min(lmax - 1, nlat // 2), the
  default of ``l_hi`` here.
* The observation in eq. spectral_loss is printed as u*(x, t_n); it is read
  as the coefficient u*^_l^m of the observation.
"""
import numpy as np

from .grids import grid


def _as_ens(ens, obs):
    ens = np.asarray(ens, dtype=np.float64)
    obs = np.asarray(obs, dtype=np.float64)
    if ens.shape[1:] != obs.shape:
        raise ValueError("ensemble must be [N, ...] with obs [...]")
    return ens, obs


def crps_integral(ens, obs):
    """eq. crps with the empirical ensemble CDF: the exact integral of
    (F_ens(u) - 1(obs <= u))^2 over u.  ens: [N, ...], obs: [...]."""
    ens, obs = _as_ens(ens, obs)
    n = ens.shape[0]
    # breakpoints of the piecewise constant integrand, per point
    pts = np.sort(np.concatenate([ens, obs[None]], axis=0), axis=0)    # [N+1, ...]
    out = np.zeros(obs.shape)
    for i in range(n):                      # interval [pts[i], pts[i+1])
        lo, hi = pts[i], pts[i + 1]
        mid = 0.5 * (lo + hi)
        F = np.sum(ens <= mid[None], axis=0) / n
        H = (obs <= mid).astype(np.float64)
        out += (F - H) ** 2 * (hi - lo)
    return out


def crps_sorted(ens, obs):
    """eq. ensemble_crps_cdf: members sorted ascending, u_1 .. u_e* at or
    below the observation, the rest above it."""
    ens, obs = _as_ens(ens, obs)
    n = ens.shape[0]
    s = np.sort(ens, axis=0)
    e = np.arange(1, n + 1, dtype=np.float64).reshape((n,) + (1,) * obs.ndim)
    below = s <= obs[None]
    w_below = (2.0 * e - 1.0) / n ** 2
    w_above = (2.0 * n + 1.0 - 2.0 * e) / n ** 2
    return np.sum(np.where(below, w_below * (obs[None] - s), w_above * (s - obs[None])), axis=0)


def crps_spread_skill(ens, obs, fair=False):
    """eq. spread_skill_crps (fair=False) or eq. fair_spread_skill_crps
    (fair=True): mean |u_e - u*| minus the pair term sum |u_e - u_i| divided
    by 2 N^2 (or 2 N (N - 1))."""
    ens, obs = _as_ens(ens, obs)
    n = ens.shape[0]
    skill = np.mean(np.abs(ens - obs[None]), axis=0)
    pairs = np.zeros(obs.shape)
    for e in range(n):
        pairs += np.sum(np.abs(ens[e][None] - ens), axis=0)
    denom = 2.0 * n * (n - 1) if fair else 2.0 * n * n
    if fair and n < 2:
        raise ValueError("the fair CRPS needs at least two members")
    return skill - pairs / denom


def _order_weights(mmax):
    """Multiplicity of a stored order m >= 0 in a sum over |m| <= l."""
    c = np.full(mmax, 2.0)
    c[0] = 1.0
    return c


def spectral_crps(ens_coeffs, obs_coeffs, nlat, fair=False, l_hi=None):
    """eq. spectral_loss per field: ens_coeffs complex [N, ..., lmax, mmax]
    (members first), obs_coeffs complex [..., lmax, mmax].  Returns [...]:
    sum over 1 <= l <= l_hi, m <= min(l, mmax - 1) of
    c_m (CRPS(Re) + CRPS(Im)), c_0 = 1, c_m = 2."""
    ens = np.asarray(ens_coeffs, dtype=np.complex128)
    obs = np.asarray(obs_coeffs, dtype=np.complex128)
    lmax, mmax = obs.shape[-2], obs.shape[-1]
    if l_hi is None:
        l_hi = min(lmax - 1, nlat // 2)
    score = crps_spread_skill(ens.real, obs.real, fair) + crps_spread_skill(ens.imag, obs.imag, fair)
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    mask = (l >= 1) & (l <= l_hi) & (m <= l)
    w = np.where(mask, _order_weights(mmax)[None, :], 0.0)
    return np.sum(score * w, axis=(-2, -1))


def spatial_crps(ens_fields, obs_field, kind, fair=False):
    """eq. spatial_loss per field: (1/4 pi) sum_k sum_j (2 pi / nlon) w_k
    CRPS at (k, j).  ens_fields [N, ..., nlat, nlon], obs_field [..., nlat, nlon]."""
    ens = np.asarray(ens_fields, dtype=np.float64)
    obs = np.asarray(obs_field, dtype=np.float64)
    nlat, nlon = obs.shape[-2], obs.shape[-1]
    _, _, w = grid(nlat, kind)
    score = crps_spread_skill(ens, obs, fair)
    quad = (2.0 * np.pi / nlon) * w[:, None] * np.ones((1, nlon))
    return np.sum(score * quad, axis=(-2, -1)) / (4.0 * np.pi)


def psd(coeffs):
    """eq. psd: PSD(l) = sum over |m| <= l of |u^_l^m|^2 for a real field whose
    orders m >= 0 are stored.  coeffs complex [..., lmax, mmax] -> [..., lmax]."""
    a = np.asarray(coeffs, dtype=np.complex128)
    lmax, mmax = a.shape[-2], a.shape[-1]
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    w = np.where(m <= l, _order_weights(mmax)[None, :], 0.0)
    return np.sum(np.abs(a) ** 2 * w, axis=-1)


def zonal_psd(u, kind, mmax):
    """eq. zonal_psd at every ring k and order m < mmax:
    2 pi sin(t_k) |(2 pi / nlon) sum_j u[k, j] e^{-2 pi i j m / nlon}|^2.
    u: [..., nlat, nlon] -> [..., nlat, mmax]."""
    u = np.asarray(u, dtype=np.float64)
    nlat, nlon = u.shape[-2], u.shape[-1]
    theta, _, _ = grid(nlat, kind)
    X = (2.0 * np.pi / nlon) * np.fft.rfft(u, axis=-1)[..., :mmax]
    return 2.0 * np.pi * np.sin(theta)[:, None] * np.abs(X) ** 2


def crps_spread_skill_grad(ens, obs, fair=False):
    """Derivative of ``crps_spread_skill`` with respect to every member:
    sign(u_e - u*) / N - sum_i sign(u_e - u_i) / N^2 (fair: / N(N - 1)),
    each |.| differentiated as sign(.) with sign(0) = 0."""
    ens, obs = _as_ens(ens, obs)
    n = ens.shape[0]
    g = np.sign(ens - obs[None]) / n
    pair = np.zeros_like(ens)
    for i in range(n):
        pair += np.sign(ens - ens[i][None])
    return g - pair / (n * (n - 1) if fair else n * n)


def spectral_crps_grad(ens_coeffs, obs_coeffs, nlat, fair=False, l_hi=None):
    """Gradient of sum(spectral_crps(...)) with respect to the ensemble
    coefficients in PyTorch's complex convention, dL/dRe + i dL/dIm:
    complex [N, ..., lmax, mmax]."""
    ens = np.asarray(ens_coeffs, dtype=np.complex128)
    obs = np.asarray(obs_coeffs, dtype=np.complex128)
    lmax, mmax = obs.shape[-2], obs.shape[-1]
    if l_hi is None:
        l_hi = min(lmax - 1, nlat // 2)
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    w = np.where((l >= 1) & (l <= l_hi) & (m <= l), _order_weights(mmax)[None, :], 0.0)
    return w * (crps_spread_skill_grad(ens.real, obs.real, fair)
                + 1j * crps_spread_skill_grad(ens.imag, obs.imag, fair))


def spatial_crps_grad(ens_fields, obs_field, kind, fair=False):
    """Gradient of sum(spatial_crps(...)) with respect to the members' grid
    values: [N, ..., nlat, nlon]."""
    ens = np.asarray(ens_fields, dtype=np.float64)
    obs = np.asarray(obs_field, dtype=np.float64)
    nlat, nlon = obs.shape[-2], obs.shape[-1]
    _, _, w = grid(nlat, kind)
    quad = (2.0 * np.pi / nlon) * w[:, None] * np.ones((1, nlon)) / (4.0 * np.pi)
    return quad * crps_spread_skill_grad(ens, obs, fair)
