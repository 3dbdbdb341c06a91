"""Spherical diffusion noise (oracle, FP64; test infrastructure only).

App. B.7, eq. spherical_diffusion: an AR(1) process in the spectral domain,
    z_n = phi z_{n-1} + sum_{l >= 1} sum_{|m| <= l} sigma_l eta_l^m Y_l^m,
    phi = e^{-lambda},  sigma_l = F_0 e^{-(k_T / 2) l (l + 1)},
    F_0 = sigma sqrt(2 pi (1 - phi^2) / sum_{l > 0} (2 l + 1) e^{-k_T l (l + 1)}),
with the length scales k_T of Table 1 (lambda = 1, sigma = 1), synthesised
to the grid by the ISHT (eq. isht).

Readings of the paper (where it is silent or garbled):
* eta is printed with the degree index only; it is read as independent
  standard normal draws per coefficient (l, m), otherwise the field would not
  be isotropic.
* A real field stores m >= 0: for m >= 1 the coefficient is
  sigma_l (eta_re + i eta_im), for m = 0 it is real, sqrt(2) sigma_l eta_re,
  so that E|a_l^m|^2 = 2 sigma_l^2 for every m (isotropy).  With the F_0 of
  the paper the stationary point-wise variance is then exactly sigma^2
  (addition theorem: sum_m |Y_l^m|^2 = (2l + 1) / 4 pi), the variance the
  paper says sigma sets.
* Degrees start at l = 1 (the sum defining F_0 runs over l > 0) and end at
  lmax - 1 (the degrees the transform represents); F_0's sum is taken over
  the same degrees, so the truncated field keeps variance sigma^2.
* The process starts from its stationary law: the first state is
  sigma_l / sqrt(1 - phi^2) times the draw.

Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011), a counter-based generator, written
here from its published definition: ten rounds of
    (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
with the key bumped by the Weyl constants after every round.  Coefficient
(f, l, m) of step n (f = member * channels + channel) takes counter
(index, n, 0, 0) with index = (f * lmax + l) * mmax + m and key (seed, 0);
the first two outputs become two uniforms u = (x >> 11) 2^-53 and, by the
Box-Muller transform (Box & Muller 1958), the pair
    eta_re = sqrt(-2 ln(1 - u0)) cos(2 pi u1),  eta_im = sqrt(-2 ln(1 - u0)) sin(2 pi u1).
"""
import numpy as np

M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1

# Table 1: the eight noise length scales, lambda = 1, sigma = 1
TABLE1_KT = (3.08e-5, 1.23e-4, 4.93e-4, 1.97e-3, 7.89e-3, 3.16e-2, 1.26e-1, 5.05e-1)


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: counter (4 x uint64), key (2 x uint64) as
    Python ints -> 4 x uint64 (Python ints)."""
    x = [int(c) & _MASK for c in counter]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for _ in range(10):
        p0 = M0 * x[0]
        p1 = M1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k0, p1 & _MASK, (p0 >> 64) ^ x[3] ^ k1, p0 & _MASK]
        k0 = (k0 + W0) & _MASK
        k1 = (k1 + W1) & _MASK
    return x


def _mulhilo(a, b):
    """64 x 64 -> (hi, lo) for uint64 arrays, from 32-bit halves."""
    a_lo, a_hi = a & np.uint64(0xFFFFFFFF), a >> np.uint64(32)
    b_lo, b_hi = b & np.uint64(0xFFFFFFFF), b >> np.uint64(32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> np.uint64(32)) + (lh & np.uint64(0xFFFFFFFF)) + (hl & np.uint64(0xFFFFFFFF))
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = a * b
    return hi, lo


def philox4x64_10_array(c0, c1, c2, c3, k0, k1):
    """The same block function, vectorised over uint64 arrays (the form the
    noise uses); pinned against the scalar form above."""
    x = [np.asarray(c, dtype=np.uint64).copy() for c in (c0, c1, c2, c3)]
    k0 = np.uint64(k0)
    k1 = np.uint64(k1)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(np.uint64(M0), x[0])
            hi1, lo1 = _mulhilo(np.uint64(M1), x[2])
            x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
            k0 = k0 + np.uint64(W0)
            k1 = k1 + np.uint64(W1)
    return x


def normal_pairs(index, step, seed):
    """(eta_re, eta_im) standard normal pairs for coefficient indices `index`
    (uint64 array) at time step `step`."""
    index = np.asarray(index, dtype=np.uint64)
    zeros = np.zeros_like(index)
    x = philox4x64_10_array(index, np.full_like(index, np.uint64(step)), zeros, zeros, seed, 0)
    u0 = (x[0] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u1 = (x[1] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(1.0 - u0))
    return r * np.cos(2.0 * np.pi * u1), r * np.sin(2.0 * np.pi * u1)


def diffusion_params(lmax, kT, lam, sigma):
    """(phi, sigma_l[lmax]) of eq. spherical_diffusion; sigma_0 = 0."""
    l = np.arange(lmax, dtype=np.float64)
    phi = np.exp(-lam)
    q = np.exp(-kT * l * (l + 1.0))
    F0 = sigma * np.sqrt(2.0 * np.pi * (1.0 - phi * phi) / np.sum((2.0 * l[1:] + 1.0) * q[1:]))
    s = F0 * np.exp(-0.5 * kT * l * (l + 1.0))
    s[0] = 0.0
    return phi, s


def diffusion_step(state, step, seed, kT, lam, sigma):
    """One step of eq. spherical_diffusion for every member and channel.

    state: complex [B, C, lmax, mmax] (z_{n-1}'s coefficients; ignored at
    step 0, where the stationary start is drawn).  kT, lam, sigma: per
    channel, length C.  Returns the new coefficients (complex128)."""
    state = np.asarray(state, dtype=np.complex128)
    B, C, lmax, mmax = state.shape
    out = np.zeros_like(state)
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    live = (l >= 1) & (m <= l)
    for b in range(B):
        for c in range(C):
            phi, s = diffusion_params(lmax, kT[c], lam[c], sigma[c])
            f = b * C + c
            index = (np.uint64(f) * np.uint64(lmax) + l.astype(np.uint64)) * np.uint64(mmax) + m.astype(np.uint64)
            er, ei = normal_pairs(index, step, seed)
            draw = np.where(m == 0, np.sqrt(2.0) * er + 0j, er + 1j * ei) * s[:, None]
            if step == 0:
                new = draw / np.sqrt(1.0 - phi * phi)
            else:
                new = phi * state[b, c] + draw
            out[b, c] = np.where(live, new, 0.0)
    return out
