"""ctypes declarations of the C ABI in include/sht.h (libsht.so)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsht.so")

SHT_OK = 0
STATUS = {0: "SHT_OK", 1: "SHT_ERR_INVALID_ARG", 2: "SHT_ERR_UNSUPPORTED",
          3: "SHT_ERR_OUT_OF_MEMORY", 4: "SHT_ERR_HIP", 5: "SHT_ERR_INTERNAL"}

GRIDS = {"equiangular": 0, "gauss": 1, "equiangular_trapezoid": 2}
PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x2": 2, "bf16x3": 3}

# every symbol include/sht.h declares
EXPORTS = ["sht_plan", "sht_plan_destroy", "sht_plan_segment", "sht_plan_sizes", "sht_plan_grid",
           "sht_forward", "isht_forward", "sht_backward", "isht_backward", "sht_channel_mix",
           "sht_channel_mix_weight_grad", "sht_isotropic_filter", "sht_isotropic_filter_grad", "sht_graph_create", "sht_graph_launch", "sht_graph_destroy", "sht_plan_tune",
           "sht_plan_set_schedule", "sht_plan_get_schedule", "sht_measure_peak",
           "sht_plan_timing", "sht_plan_timing_read", "sht_psd", "sht_zonal_psd", "sht_spectral_crps",
           "sht_spectral_crps_noalloc", "sht_spatial_crps", "sht_noise_create", "sht_noise_step", "sht_noise_set_step", "sht_noise_destroy",
           "sht_status_string", "sht_last_error"]

OPS = {"sht": 0, "isht": 1, "sht_T": 2, "isht_T": 3}

TIMING_KINDS = ["dft_forward", "dft_inverse", "legendre_analysis", "legendre_synthesis", "zero_fill",
                "channel_mix", "scores", "noise", "transpose", "stage"]


class ShtDesc(ctypes.Structure):
    _fields_ = [("nlat", ctypes.c_int), ("nlon", ctypes.c_int), ("lmax", ctypes.c_int),
                ("mmax", ctypes.c_int), ("grid", ctypes.c_int), ("batch", ctypes.c_int),
                ("channels", ctypes.c_int)]


class ShtError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


_lib = None


def load():
    """Load libsht.so from the package directory.  There is no fallback: a
    missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2507_12144_amd.build.build()")
    _lib = open_library(LIB_PATH)
    return _lib


def open_library(path):
    """A separately loaded copy of a build of the library (e.g. the
    race-check build libsht_debug.so) with the C ABI's signatures declared;
    its plans live in that copy only."""
    lib = ctypes.CDLL(path)
    vp, ip, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.sht_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ShtDesc), ip, ip, vp]
    lib.sht_plan_destroy.argtypes = [vp]
    lib.sht_plan_segment.argtypes = [vp, ip, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.sht_plan_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.sht_plan_grid.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    for name in ("sht_forward", "isht_forward", "sht_backward", "isht_backward"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    lib.sht_channel_mix.argtypes = [vp, vp, vp, vp, ip, vp]
    lib.sht_channel_mix_weight_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.sht_isotropic_filter.argtypes = [vp, vp, vp, vp, ip, vp]
    lib.sht_isotropic_filter_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.sht_plan_timing.argtypes = [vp, ip]
    lib.sht_plan_set_schedule.argtypes = [vp, ip, ip, ip, ip]
    lib.sht_measure_peak.argtypes = [ip, sz, ctypes.POINTER(ctypes.c_double), vp]
    ipp = ctypes.POINTER(ctypes.c_int)
    lib.sht_plan_get_schedule.argtypes = [vp, ipp, ipp, ipp, ipp]
    lib.sht_plan_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong), ip]
    lib.sht_psd.argtypes = [vp, vp, vp, vp]
    lib.sht_zonal_psd.argtypes = [vp, vp, vp, vp]
    lib.sht_spectral_crps.argtypes = [vp, vp, vp, ip, ip, vp, vp, vp]
    lib.sht_spatial_crps.argtypes = [vp, vp, vp, ip, vp, vp, vp]
    lib.sht_spectral_crps_noalloc.argtypes = [ctypes.POINTER(ShtDesc), vp, vp, ip, ip, vp, vp, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.sht_noise_create.argtypes = [vp, dp, dp, dp, ctypes.c_ulonglong, ctypes.POINTER(vp)]
    lib.sht_noise_step.argtypes = [vp, vp, vp, vp]
    lib.sht_noise_set_step.argtypes = [vp, ctypes.c_ulonglong]
    lib.sht_noise_destroy.argtypes = [vp]
    for name in EXPORTS[:-2]:
        getattr(lib, name).restype = ctypes.c_int
    lib.sht_status_string.argtypes = [ip]
    lib.sht_status_string.restype = ctypes.c_char_p
    lib.sht_last_error.argtypes = []
    lib.sht_last_error.restype = ctypes.c_char_p
    return lib


def check(status):
    if status != SHT_OK:
        detail = load().sht_last_error().decode(errors="replace")
        raise ShtError(status, detail)
