"""Latitude grids and quadrature weights (oracle, FP64; test infrastructure only).

Conventions (App. B.1):

* Rings are ordered from the north pole (colatitude 0) southwards.
* ``x`` is cos(colatitude); ``w`` are the latitude weights, normalised so that
  sum(w) approximates the integral of sin(t) dt over [0, pi], i.e. 2.  The full
  sphere weight of grid point (k, j) is w[k] * 2*pi/nlon (the longitudinal
  spacing, eq. latlon_quad_weights).
* Equiangular grids include both poles: t_k = pi*k/(nlat-1).  The printed form
  t_i = pi*i/n_lat of eq. latlon_grid cannot hold both poles of an odd,
  pole-inclusive grid such as the 721-ring 0.25 degree grid, so it is read as
  spacing pi/(nlat-1).
"""
import numpy as np

GRID_EQUIANGULAR = 0            # poles included, Clenshaw-Curtis weights
GRID_GAUSS = 1                  # Gauss-Legendre nodes and weights
GRID_EQUIANGULAR_TRAPEZOID = 2  # poles included, sin(t)*dt weights


def equiangular_nodes(nlat):
    """Colatitudes t_k = pi*k/(nlat-1), k = 0..nlat-1, and x_k = cos t_k.

    Follows eq. latlon_grid with both poles on the grid (see module note)."""
    if nlat < 2:
        raise ValueError("nlat must be >= 2")
    theta = np.pi * np.arange(nlat, dtype=np.float64) / (nlat - 1)
    return theta, np.cos(theta)


def clenshaw_curtis_weights(nlat):
    """Clenshaw-Curtis weights on the pole-inclusive equiangular grid.

    The rule (Clenshaw and Curtis 1960, cited in the footnote to
    eq. latlon_quad_weights) integrates every polynomial of degree <= N in
    x = cos t exactly, N = nlat-1.  Written out as the cosine series

        w_k = (c_k / N) * (1 - sum_{j=1}^{floor(N/2)} b_j cos(2 j t_k) / (4 j^2 - 1))

    with c_k = 1 at the poles and 2 elsewhere, b_j = 1 for j = N/2 (N even)
    and 2 otherwise.  It follows from integrating the degree-N interpolant in
    the Chebyshev basis: int_{-1}^{1} T_{2j}(x) dx = -2/(4j^2-1), odd T
    integrate to zero.
    """
    theta, _ = equiangular_nodes(nlat)
    N = nlat - 1
    s = np.ones(nlat, dtype=np.float64)
    for j in range(1, N // 2 + 1):
        b = 1.0 if (2 * j == N) else 2.0
        s -= b * np.cos(2.0 * j * theta) / (4.0 * j * j - 1.0)
    c = np.full(nlat, 2.0)
    c[0] = c[N] = 1.0
    return c * s / N


def trapezoid_weights(nlat):
    """Weights sin(t_k) * dt with dt = pi/(nlat-1): the latitude factor of
    eq. latlon_quad_weights on the pole-inclusive grid.  They sum only
    approximately to 2."""
    theta, _ = equiangular_nodes(nlat)
    return np.sin(theta) * (np.pi / (nlat - 1))


def _legendre_p_and_dp(n, x):
    """P_n(x) and P_n'(x) by the Bonnet recurrence (plain, unnormalised)."""
    p0 = np.ones_like(x)
    p1 = x.copy()
    if n == 0:
        return p0, np.zeros_like(x)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative: (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    dp = n * (p0 - x * p1) / ((1.0 - x) * (1.0 + x))
    return p1, dp


def gauss_legendre(nlat, iters=100):
    """Gauss-Legendre nodes x_k (roots of P_nlat, descending: north to south)
    and weights w_k = 2 / ((1 - x_k^2) P'_nlat(x_k)^2).

    The roots are found by Newton's method on P_nlat, started from the
    asymptotic guess cos(pi (k + 3/4) / (nlat + 1/2)).  The rule is exact for
    polynomials of degree <= 2*nlat - 1 in x (App. B.1, Gaussian grids)."""
    if nlat < 1:
        raise ValueError("nlat must be >= 1")
    k = np.arange(nlat, dtype=np.float64)
    x = np.cos(np.pi * (k + 0.75) / (nlat + 0.5))
    for _ in range(iters):
        p, dp = _legendre_p_and_dp(nlat, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = _legendre_p_and_dp(nlat, x)
    w = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp)
    return np.arccos(x), x, w


def grid(nlat, kind):
    """(theta, x, w) for a grid type: 0 equiangular + Clenshaw-Curtis,
    1 Gauss-Legendre, 2 equiangular + trapezoid weights."""
    if kind == GRID_EQUIANGULAR:
        theta, x = equiangular_nodes(nlat)
        return theta, x, clenshaw_curtis_weights(nlat)
    if kind == GRID_GAUSS:
        return gauss_legendre(nlat)
    if kind == GRID_EQUIANGULAR_TRAPEZOID:
        theta, x = equiangular_nodes(nlat)
        return theta, x, trapezoid_weights(nlat)
    raise ValueError(f"unknown grid kind {kind}")
