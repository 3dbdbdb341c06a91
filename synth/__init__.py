"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Random draws and masks only: none of the transform's arithmetic
lives here.

Recipe (one numpy Generator per seed, C-order draws):

* ``coefficients``: spectral coefficients a[b, c, l, m] with Re and Im drawn
  i.i.d. N(0, 1) as ``standard_normal((B, C, lmax, mmax, 2))``, scaled by
  1/(l+1) (a red spectrum standing in for the decaying spectra of atmospheric
  fields), Im(a[l, 0]) = 0 and a = 0 for l < m.
* ``white_noise``: N(0, 1) * amplitude on the grid (the aliasing probe).
* ``mix_weights``: per-degree complex C x C weights with Re and Im i.i.d.
  N(0, 1/(2C)), so E|W|^2 = 1/C.
* ``grid_normal``: N(0, 1) grid arrays (cotangents, directions).
"""
import numpy as np


def coefficients(seed, batch, channels, lmax, mmax):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((batch, channels, lmax, mmax, 2))
    a = np.empty((batch, channels, lmax, mmax), dtype=np.complex128)
    a.real = z[..., 0]
    a.imag = z[..., 1]
    del z
    scale = 1.0 / (np.arange(lmax, dtype=np.float64) + 1.0)
    a *= scale[None, None, :, None]
    a[..., 0].imag = 0.0
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    a *= (l >= m)
    return a


def white_noise(seed, shape, amplitude=1e-3):
    rng = np.random.default_rng(seed)
    return amplitude * rng.standard_normal(shape)


def mix_weights(seed, lmax, channels):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((lmax, channels, channels, 2)) * np.sqrt(1.0 / (2.0 * channels))
    return z[..., 0] + 1j * z[..., 1]


def grid_normal(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape)
