"""Per-degree complex channel mix (oracle, FP64; test infrastructure only).

A multi-channel form of the spectral convolution of App. B.4
(eq. s2_spectral_conv): the filter acts on each degree l with the same
weight for every order m, here a complex C x C matrix W_l:

    y[b, c', l, m] = sum_c W[l, c', c] x[b, c, l, m]

Adjoint under the real inner product Re sum conj(a) b:
    g_x[b, c, l, m] = sum_c' conj(W[l, c', c]) g_y[b, c', l, m]
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
