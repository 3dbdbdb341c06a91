"""Orthonormal associated Legendre functions (oracle, FP64; test infrastructure only).

App. B.3, eq. spherical_harmonics: Y_l^m(t, p) = P^_l^m(cos t) e^{i m p} with
P^_l^m = (-1)^m c_l^m P_l^m and c_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
P_l^m is read as the associated Legendre function *without* the
Condon-Shortley phase, so P^_l^m carries the factor (-1)^m; Y_l^m are then
orthonormal on the sphere (the orthonormality relation stated after
eq. spherical_harmonics).

The values are produced by the textbook three-term recurrence for fully
normalised functions, in float64, one order m at a time:

    P^_0^0           = 1/sqrt(4 pi)
    P^_m^m           = -sqrt((2m+1)/(2m)) sin t P^_{m-1}^{m-1}
    P^_{m+1}^m       = sqrt(2m+3) x P^_m^m
    P^_l^m           = a_lm (x P^_{l-1}^m - b_lm P^_{l-2}^m)
    a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1))

Tiny starting values that underflow in float64 near the poles at high m are
flushed to zero; none of them can grow back to a significant size before
l = 720 on the grids used here.
"""
import numpy as np


def legendre_order(m, lmax, x, sin_t, pmm):
    """Rows P^_l^m(x) for l = m..lmax-1 (shape (lmax-m, len(x))), given the
    diagonal start pmm = P^_m^m(x)."""
    n = lmax - m
    out = np.zeros((max(n, 0), x.shape[0]), dtype=np.float64)
    if n <= 0:
        return out
    out[0] = pmm
    if n > 1:
        out[1] = np.sqrt(2.0 * m + 3.0) * x * pmm
    for i in range(2, n):
        l = m + i
        a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
        out[i] = a * (x * out[i - 1] - b * out[i - 2])
    return out


def iter_orders(lmax, mmax, x, sin_t):
    """Yield (m, rows) for m = 0..mmax-1, where rows[i] = P^_{m+i}^m(x)."""
    pmm = np.full(x.shape[0], 1.0 / np.sqrt(4.0 * np.pi))
    for m in range(mmax):
        if m > 0:
            pmm = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sin_t * pmm
        yield m, legendre_order(m, lmax, x, sin_t, pmm)


def legendre_table(lmax, mmax, theta):
    """Dense P^[m, l, k] (zeros for l < m) at colatitudes theta.  For small
    grids only: the 721-ring, lmax 720 table would need 3 GB."""
    x = np.cos(theta)
    s = np.sin(theta)
    tab = np.zeros((mmax, lmax, theta.shape[0]), dtype=np.float64)
    for m, rows in iter_orders(lmax, mmax, x, s):
        tab[m, m:lmax] = rows
    return tab
