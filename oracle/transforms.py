"""SHT, ISHT and their adjoints (oracle, FP64; test infrastructure only).

Definitions (App. B.3):

* eq. sht: u^_l^m = integral of u conj(Y_l^m) over the sphere.  On a grid it
  is the quadrature sum
      u^[l, m] = sum_k sum_j (2 pi / nlon) w_k u[k, j] P^_l^m(x_k) e^{-2 pi i j m / nlon}
  for m <= l < lmax, m < mmax, and 0 for l < m.  lmax and mmax are counts
  (degrees l < lmax, orders m < mmax), as in the mode truncation
  xf[..., :mmax] of Alg. 1.  The longitude sum is the "2 pi * FFT_1D_R2C"
  step of Alg. 1 with the forward 1/nlon normalisation (the longitude
  quadrature spacing 2 pi / nlon).
* eq. isht: u = sum_l sum_{|m| <= l} u^_l^m Y_l^m.  For a real field
  u^_l^{-m} = (-1)^m conj(u^_l^m), so with stored orders m >= 0 only
      u[k, j] = sum_{m < mmax} c_m Re(e^{2 pi i j m / nlon} sum_{l=m}^{lmax-1} P^_l^m(x_k) u^[l, m])
  with c_0 = 1 and c_m = 2 for m >= 1; Im(u^[l, 0]) and entries l < m do not
  enter.
* Adjoints under the real inner product <a, b> = Re sum conj(a) b (which is
  PyTorch's gradient convention for complex tensors):
      sht_T : g_u[k, j] = (2 pi / nlon) w_k sum_m Re(e^{2 pi i j m / nlon} sum_l P^ g[l, m])
              (weight 1 for every m, m = 0 included)
      isht_T: g^[l, m] = c_m sum_k P^_l^m(x_k) sum_j g[k, j] e^{-2 pi i j m / nlon}   (l >= m)

Arrays are float64 [..., nlat, nlon] (grid) and complex128 [..., lmax, mmax]
(spectral, m fastest), matching the B x C x H x W and B x C x lmax x mmax
layouts of Alg. 1.  The Legendre step is one plain matrix product per order m;
the longitude step is numpy's real FFT.  Nothing is folded, blocked or fused.
"""
import numpy as np

from .grids import grid
from .legendre import iter_orders, legendre_table


def _ring_dft(u, mmax):
    """sum_j u[..., k, j] e^{-2 pi i j m / nlon} for m < mmax (unnormalised)."""
    return np.fft.rfft(u, axis=-1)[..., :mmax]


def _ring_synth(Y, nlon, c_rest):
    """sum_m c_m Re(Y[..., k, m] e^{2 pi i j m / nlon}), c_0 = 1, c_m = c_rest.

    numpy's irfft of a half spectrum H of length nlon//2+1 returns
    (1/nlon)(Re H_0 + 2 sum_{m>=1} Re(H_m e^{...})) when the Nyquist bin is
    zero, so H_0 = Y_0 and H_m = (c_rest / 2) Y_m reproduce the sum exactly."""
    mmax = Y.shape[-1]
    if 2 * mmax > nlon:
        raise ValueError("mmax must not reach the Nyquist bin")
    H = np.zeros(Y.shape[:-1] + (nlon // 2 + 1,), dtype=np.complex128)
    H[..., 0] = Y[..., 0]
    H[..., 1:mmax] = 0.5 * c_rest * Y[..., 1:mmax]
    return nlon * np.fft.irfft(H, n=nlon, axis=-1)


def _legendre_analysis(X, lmax, x, sin_t):
    """out[..., l, m] = sum_k P^_l^m(x_k) X[..., k, m] for l >= m, else 0.

    The data are moved once to order-major layout so that each order's
    product reads contiguous memory; the arithmetic is one matrix product
    per order m."""
    lead = X.shape[:-2]
    nlat, mmax = X.shape[-2], X.shape[-1]
    Xr = np.ascontiguousarray(np.moveaxis(X.real.reshape(-1, nlat, mmax), -1, 0))  # (mmax, F, nlat)
    Xi = np.ascontiguousarray(np.moveaxis(X.imag.reshape(-1, nlat, mmax), -1, 0))
    F = Xr.shape[1]
    out = np.zeros((mmax, F, lmax), dtype=np.complex128)
    for m, rows in iter_orders(lmax, mmax, x, sin_t):
        if rows.shape[0] == 0:
            continue
        # (F, nlat) @ (nlat, lmax - m)
        out[m, :, m:].real = Xr[m] @ rows.T
        out[m, :, m:].imag = Xi[m] @ rows.T
    # returned in C order ([..., l, m], m fastest): later per-degree slicing
    # of a strided view would touch one memory page per element
    return np.ascontiguousarray(np.moveaxis(out, 0, -1).reshape(lead + (lmax, mmax)))


def _legendre_synthesis(a, nlat, x, sin_t):
    """Y[..., k, m] = sum_{l=m}^{lmax-1} P^_l^m(x_k) a[..., l, m] (one matrix
    product per order m, on order-major data)."""
    lead = a.shape[:-2]
    lmax, mmax = a.shape[-2], a.shape[-1]
    ar = np.ascontiguousarray(np.moveaxis(a.real.reshape(-1, lmax, mmax), -1, 0))  # (mmax, F, lmax)
    ai = np.ascontiguousarray(np.moveaxis(a.imag.reshape(-1, lmax, mmax), -1, 0))
    F = ar.shape[1]
    Y = np.zeros((mmax, F, nlat), dtype=np.complex128)
    for m, rows in iter_orders(lmax, mmax, x, sin_t):
        if rows.shape[0] == 0:
            continue
        # (F, lmax - m) @ (lmax - m, nlat)
        Y[m].real = ar[m, :, m:] @ rows
        Y[m].imag = ai[m, :, m:] @ rows
    return np.moveaxis(Y, 0, -1).reshape(lead + (nlat, mmax))


def _check_spec(lmax, mmax, nlon):
    if lmax < 1 or mmax < 1 or mmax > lmax:
        raise ValueError("need 1 <= mmax <= lmax")
    if 2 * mmax > nlon:
        raise ValueError("need mmax <= nlon/2 (the Nyquist bin is never used)")


def sht(u, lmax, mmax, kind):
    """Forward transform (eq. sht as a quadrature sum).  u: [..., nlat, nlon]."""
    u = np.asarray(u, dtype=np.float64)
    nlat, nlon = u.shape[-2], u.shape[-1]
    _check_spec(lmax, mmax, nlon)
    theta, x, w = grid(nlat, kind)
    X = _ring_dft(u, mmax) * (2.0 * np.pi / nlon)
    X = X * w[:, None]
    return _legendre_analysis(X, lmax, x, np.sin(theta))


def isht(a, nlat, nlon, kind):
    """Inverse transform (eq. isht with real-field symmetry).  a: [..., lmax, mmax]."""
    a = np.asarray(a, dtype=np.complex128)
    lmax, mmax = a.shape[-2], a.shape[-1]
    _check_spec(lmax, mmax, nlon)
    theta, x, _ = grid(nlat, kind)
    Y = _legendre_synthesis(a, nlat, x, np.sin(theta))
    return _ring_synth(Y, nlon, 2.0)


def sht_T(g, nlat, nlon, kind):
    """Adjoint of ``sht``: [..., lmax, mmax] complex -> [..., nlat, nlon] real."""
    g = np.asarray(g, dtype=np.complex128)
    lmax, mmax = g.shape[-2], g.shape[-1]
    _check_spec(lmax, mmax, nlon)
    theta, x, w = grid(nlat, kind)
    Y = _legendre_synthesis(g, nlat, x, np.sin(theta))
    u = _ring_synth(Y, nlon, 1.0)
    return u * ((2.0 * np.pi / nlon) * w)[:, None]


def isht_T(g, lmax, mmax, kind):
    """Adjoint of ``isht``: [..., nlat, nlon] real -> [..., lmax, mmax] complex."""
    g = np.asarray(g, dtype=np.float64)
    nlat, nlon = g.shape[-2], g.shape[-1]
    _check_spec(lmax, mmax, nlon)
    theta, x, _ = grid(nlat, kind)
    X = _ring_dft(g, mmax)
    out = _legendre_analysis(X, lmax, x, np.sin(theta))
    out[..., 1:] *= 2.0
    return out


def sht_bruteforce(u, lmax, mmax, kind):
    """The literal quadruple sum of eq. sht on a grid, for tiny grids only:
    every (l, m) coefficient is summed point by point over (k, j)."""
    u = np.asarray(u, dtype=np.float64)
    nlat, nlon = u.shape[-2], u.shape[-1]
    theta, _, w = grid(nlat, kind)
    P = legendre_table(lmax, mmax, theta)
    phi = 2.0 * np.pi * np.arange(nlon) / nlon
    lead = u.shape[:-2]
    uu = u.reshape(-1, nlat, nlon)
    out = np.zeros((uu.shape[0], lmax, mmax), dtype=np.complex128)
    for f in range(uu.shape[0]):
        for l in range(lmax):
            for m in range(min(l + 1, mmax)):
                acc = 0.0 + 0.0j
                for k in range(nlat):
                    for j in range(nlon):
                        conj_y = P[m, l, k] * complex(np.cos(m * phi[j]), -np.sin(m * phi[j]))
                        acc += uu[f, k, j] * conj_y * w[k] * (2.0 * np.pi / nlon)
                out[f, l, m] = acc
    return out.reshape(lead + (lmax, mmax))


def isht_bruteforce(a, nlat, nlon, kind):
    """The literal sum of eq. isht over l and -l <= m <= l, for tiny grids
    only, with negative orders filled in from the real-field symmetry
    u^_l^{-m} = (-1)^m conj(u^_l^m) and Y_l^{-m} = (-1)^m conj(Y_l^m).
    Im(u^_l^0) is treated as zero (a real field has a real m = 0 column)."""
    a = np.asarray(a, dtype=np.complex128)
    lmax, mmax = a.shape[-2], a.shape[-1]
    theta, _, _ = grid(nlat, kind)
    P = legendre_table(lmax, mmax, theta)
    phi = 2.0 * np.pi * np.arange(nlon) / nlon
    lead = a.shape[:-2]
    aa = a.reshape(-1, lmax, mmax).copy()
    aa[:, :, 0] = aa[:, :, 0].real
    out = np.zeros((aa.shape[0], nlat, nlon), dtype=np.float64)
    for f in range(aa.shape[0]):
        for k in range(nlat):
            for j in range(nlon):
                acc = 0.0 + 0.0j
                for l in range(lmax):
                    for m in range(-min(l, mmax - 1), min(l, mmax - 1) + 1):
                        mm = abs(m)
                        y_pos = P[mm, l, k] * complex(np.cos(mm * phi[j]), np.sin(mm * phi[j]))
                        if m >= 0:
                            acc += aa[f, l, mm] * y_pos
                        else:
                            sgn = -1.0 if (mm % 2) else 1.0
                            acc += (sgn * np.conj(aa[f, l, mm])) * (sgn * np.conj(y_pos))
                out[f, k, j] = acc.real
    return out.reshape(lead + (nlat, nlon))
