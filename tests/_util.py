"""Shared helpers for the test suite (no transform arithmetic here)."""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    """Load the built library; build it only if nothing is built yet."""
    from paper_2507_12144_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2507_12144_amd import build
        build.build()
    return _lib.load()


def rel_l2(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    return float(np.linalg.norm((a - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def per_degree_errors(a, ref):
    """rel-L2 over (b, c, m) and max|diff| / max|ref| for every degree l of
    spectral arrays [..., lmax, mmax]."""
    a = np.asarray(a).reshape(-1, *a.shape[-2:])
    ref = np.asarray(ref).reshape(-1, *ref.shape[-2:])
    d = a - ref
    num = np.sqrt(np.sum(np.abs(d) ** 2, axis=(0, 2)))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(0, 2)))
    rel = num / np.maximum(den, 1e-300)
    mx = np.max(np.abs(d), axis=(0, 2)) / np.maximum(np.max(np.abs(ref), axis=(0, 2)), 1e-300)
    return rel, mx
