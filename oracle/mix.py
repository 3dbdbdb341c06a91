"""Per-degree complex channel mix (oracle, FP64; test infrastructure only).

A multi-channel form of the spectral convolution of App. B.4
(eq. s2_spectral_conv): the filter acts on each degree l with the same
weight for every order m, here a complex C x C matrix W_l:

    y[b, c', l, m] = sum_c W[l, c', c] x[b, c, l, m]

Adjoint under the real inner product Re sum conj(a) b:
    g_x[b, c, l, m] = sum_c' conj(W[l, c', c]) g_y[b, c', l, m]

The single-channel form of the same theorem, one isotropic filter k[c, l]
per channel ((u * k)^_l^m = u^_l^m k^_l^0), is ``isotropic_filter``.
"""
import numpy as np


def channel_mix(x, W):
    """x: complex [B, C, lmax, mmax]; W: complex [lmax, C, C] -> [B, C, lmax, mmax]."""
    x = np.asarray(x, dtype=np.complex128)
    W = np.asarray(W, dtype=np.complex128)
    B, C, lmax, mmax = x.shape
    y = np.empty_like(x)
    for l in range(lmax):
        # (C', C) @ (C, B*mmax)
        xl = np.transpose(x[:, :, l, :], (1, 0, 2)).reshape(C, B * mmax)
        yl = W[l] @ xl
        y[:, :, l, :] = np.transpose(yl.reshape(C, B, mmax), (1, 0, 2))
    return y


def channel_mix_T(g, W):
    """Adjoint of ``channel_mix`` with respect to x."""
    W = np.asarray(W, dtype=np.complex128)
    return channel_mix(g, np.conj(np.transpose(W, (0, 2, 1))))


def channel_mix_dW(g, x, degrees=None):
    """Gradient of a real loss with respect to the weights of ``channel_mix``,
    in PyTorch's complex convention (dL/dRe W + i dL/dIm W), from the gradient
    g = dL/dRe y + i dL/dIm y of y = channel_mix(x, W):

        dW[l, c', c] = sum_b sum_{m <= l} g[b, c', l, m] conj(x[b, c, l, m])

    i.e. per degree the product G_l X_l^H of the (channels x (b, m)) matrices,
    over the stored orders m <= min(l, mmax - 1) to which the filter of
    eq. s2_spectral_conv applies (entries l < m of a spectrum are zero).
    g, x: complex [B, C, lmax, mmax] -> dW: complex [lmax, C, C] (with
    ``degrees``, a list of l: only those, complex [len(degrees), C, C])."""
    g = np.asarray(g, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    B, C, lmax, mmax = x.shape
    ls = range(lmax) if degrees is None else list(degrees)
    dW = np.zeros((len(ls), C, C), dtype=np.complex128)
    for i, l in enumerate(ls):
        mc = min(l + 1, mmax)
        gl = np.transpose(g[:, :, l, :mc], (1, 0, 2)).reshape(C, B * mc)
        xl = np.transpose(x[:, :, l, :mc], (1, 0, 2)).reshape(C, B * mc)
        dW[i] = gl @ np.conj(xl).T
    return dW


def isotropic_filter(x, k):
    """The spectral convolution of eq. s2_spectral_conv with one isotropic
    filter per channel: y[b, c, l, m] = k[c, l] x[b, c, l, m] (the filter
    depends on the degree only).  x complex [B, C, lmax, mmax], k complex
    [C, lmax]."""
    x = np.asarray(x, dtype=np.complex128)
    k = np.asarray(k, dtype=np.complex128)
    return k[None, :, :, None] * x


def isotropic_filter_T(g, k):
    """Adjoint of ``isotropic_filter`` with respect to x: conj(k) g."""
    return isotropic_filter(g, np.conj(np.asarray(k, dtype=np.complex128)))


def isotropic_filter_dk(g, x):
    """Gradient of a real loss with respect to the filter of
    ``isotropic_filter`` (PyTorch's complex convention):
    dk[c, l] = sum_b sum_{m <= min(l, mmax - 1)} g[b, c, l, m] conj(x[b, c, l, m])."""
    g = np.asarray(g, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    lmax, mmax = x.shape[-2], x.shape[-1]
    mask = (np.arange(mmax)[None, :] <= np.arange(lmax)[:, None])
    return np.sum(g * np.conj(x) * mask, axis=(0, 3))
