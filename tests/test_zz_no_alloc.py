"""The allocation-free spectral CRPS entry point (sht_spectral_crps_noalloc)
through the C ABI, against the plan-based sht_spectral_crps on the same
inputs: loss and gradient, two calls in a row, the second with a smaller
input (the static scratch keeps the first call's contents)."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from _util import ensure_built

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    print(*a, file=sys.__stderr__, flush=True)


def _inputs(N, C, L, M, seed):
    obs = synth.coefficients(seed, 1, C, L, M)[0]
    ens = np.stack([obs + 0.5 * synth.coefficients(seed + 1 + e, 1, C, L, M)[0] for e in range(N)])
    return (torch.from_numpy(ens.astype(np.complex64)).cuda(), torch.from_numpy(obs.astype(np.complex64)).cuda())


@pytest.mark.parametrize("fair", [False, True])
def test_noalloc_crps_matches_plan_entry_point(fair):
    lib = ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_12144_amd as P
    from paper_2507_12144_amd import _lib
    lib.sht_spectral_crps_noalloc.argtypes = [ctypes.POINTER(_lib.ShtDesc)] + [ctypes.c_void_p] * 2 + \
        [ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 3
    lib.sht_spectral_crps_noalloc.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # first a larger call, then a smaller one: 256 x 72 degrees of rows, then 40 x 3
    for (nlat, nlon, L, M, N, C, seed) in ((181, 360, 180, 180, 8, 72, 1), (48, 96, 40, 33, 3, 3, 2)):
        _say("noalloc crps", (nlat, nlon, L, M, N, C), "fair" if fair else "biased")
        ens, obs = _inputs(N, C, L, M, seed)
        plan = P.Plan(dict(nlat=nlat, nlon=nlon, lmax=L, mmax=M, grid="equiangular", batch=N, channels=C))
        ref_loss, ref_g = plan.spectral_crps(ens, obs, fair=fair, grad=True)
        loss = torch.full((C,), float("nan"), device="cuda")
        g = torch.full_like(ens, float("nan"))
        desc = _lib.ShtDesc(nlat, nlon, L, M, 0, N, C)
        _lib.check(lib.sht_spectral_crps_noalloc(ctypes.byref(desc), ctypes.c_void_p(ens.data_ptr()),
                                                 ctypes.c_void_p(obs.data_ptr()), 1 if fair else 0, 0,
                                                 ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                                 stream))
        torch.cuda.synchronize()
        el = float(((loss - ref_loss).abs() / ref_loss.abs()).max())
        eg = float((g - ref_g).abs().max() / ref_g.abs().max())
        _say(f"  loss rel err {el:.3e}, gradient max err {eg:.3e}")
        assert el <= 1e-5 and eg <= 1e-6
        plan.close()


def test_noalloc_crps_rejects_oversized_shapes():
    lib = ensure_built()
    from paper_2507_12144_amd import _lib
    lib.sht_spectral_crps_noalloc.restype = ctypes.c_int
    desc = _lib.ShtDesc(721, 1440, 720, 720, 0, 4, 400)   # 400 x 720 rows > 262144 floats
    rc = lib.sht_spectral_crps_noalloc(ctypes.byref(desc), ctypes.c_void_p(16), ctypes.c_void_p(32), 0, 0,
                                       ctypes.c_void_p(64), None, None)
    assert rc == 2 and b"static scratch" in lib.sht_last_error()
