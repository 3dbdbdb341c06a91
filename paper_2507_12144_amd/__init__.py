"""MI355X-native real spherical harmonic transform (SHT / ISHT and adjoints).

Thin Python layer over libsht.so (include/sht.h): argument marshalling and
torch.autograd wiring only.  Every step of the transform runs in the HIP
kernels of the library; torch supplies device memory and the current stream.
There is no CPU fallback: without the built library, or without a GPU, calls
raise.
"""
import ctypes

import torch

from . import _lib
from ._lib import GRIDS, PRECISIONS, ShtError

__all__ = ["Plan", "SHT", "ISHT", "ChannelMix", "IsotropicFilter", "SpectralCRPS", "SpatialCRPS", "Noise", "ShtError", "GRIDS",
           "PRECISIONS"]


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A transform plan for one or more (nlat, nlon, lmax, mmax, grid, batch,
    channels) shapes.  With one shape, tensors keep their natural shapes
    [batch, channels, nlat, nlon] (float32) and [batch, channels, lmax, mmax]
    (complex64).  With several shapes (the batching form) tensors are flat
    concatenations; ``segment(i)`` gives each shape's offsets."""

    def __init__(self, descs, precision="fp32", device=None, library=None):
        # library: a handle from _lib.open_library (e.g. the race-check build),
        # default the package's libsht.so
        lib = self._lib = library if library is not None else _lib.load()
        if isinstance(descs, dict):
            descs = [descs]
        self.descs = [dict(d) for d in descs]
        arr = (_lib.ShtDesc * len(self.descs))()
        for i, d in enumerate(self.descs):
            grid = d.get("grid", "equiangular")
            grid = GRIDS[grid] if isinstance(grid, str) else int(grid)
            arr[i] = _lib.ShtDesc(int(d["nlat"]), int(d["nlon"]), int(d["lmax"]), int(d["mmax"]), grid,
                                  int(d.get("batch", 1)), int(d.get("channels", 1)))
        self.precision = precision
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._status(lib.sht_plan(ctypes.byref(self._h), arr, len(self.descs), prec,
                                    _stream_ptr(self.device)))
        g, s = ctypes.c_size_t(), ctypes.c_size_t()
        self._status(lib.sht_plan_sizes(self._h, ctypes.byref(g), ctypes.byref(s)))
        self.grid_elems, self.spec_elems = g.value, s.value

    def _status(self, status):
        if status != _lib.SHT_OK:
            raise _lib.ShtError(status, self._lib.sht_last_error().decode(errors="replace"))

    # ------------------------------------------------------------------ info
    def segment(self, i):
        g, s = ctypes.c_size_t(), ctypes.c_size_t()
        self._status(self._lib.sht_plan_segment(self._h, i, ctypes.byref(g), ctypes.byref(s)))
        return g.value, s.value

    def grid(self, i=0):
        """(x_k, w_k) of segment i as float64 host tensors."""
        n = self.descs[i]["nlat"]
        x = (ctypes.c_double * n)()
        w = (ctypes.c_double * n)()
        self._status(self._lib.sht_plan_grid(self._h, i, x, w))
        return torch.tensor(list(x), dtype=torch.float64), torch.tensor(list(w), dtype=torch.float64)

    def grid_shape(self):
        if len(self.descs) == 1:
            d = self.descs[0]
            return (d.get("batch", 1), d.get("channels", 1), d["nlat"], d["nlon"])
        return (self.grid_elems,)

    def spec_shape(self):
        if len(self.descs) == 1:
            d = self.descs[0]
            return (d.get("batch", 1), d.get("channels", 1), d["lmax"], d["mmax"])
        return (self.spec_elems,)

    # ------------------------------------------------------------- transforms
    def _check(self, t, dtype, shape, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _call(self, fn, src, sdt, sshape, dst, ddt, dshape):
        self._check(src, sdt, sshape, "input")
        if dst is None:
            dst = torch.empty(dshape, dtype=ddt, device=self.device)
        self._check(dst, ddt, dshape, "output")
        self._status(fn(self._h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                      _stream_ptr(self.device)))
        return dst

    def sht(self, x, out=None):
        """Forward SHT: float32 grid -> complex64 spectrum."""
        return self._call(self._lib.sht_forward, x, torch.float32, self.grid_shape(), out,
                          torch.complex64, self.spec_shape())

    def isht(self, y, out=None):
        """Inverse SHT: complex64 spectrum -> float32 grid."""
        return self._call(self._lib.isht_forward, y, torch.complex64, self.spec_shape(), out,
                          torch.float32, self.grid_shape())

    def sht_T(self, gy, out=None):
        """Adjoint of ``sht`` (sht_backward)."""
        return self._call(self._lib.sht_backward, gy, torch.complex64, self.spec_shape(), out,
                          torch.float32, self.grid_shape())

    def isht_T(self, gx, out=None):
        """Adjoint of ``isht`` (isht_backward)."""
        return self._call(self._lib.isht_backward, gx, torch.float32, self.grid_shape(), out,
                          torch.complex64, self.spec_shape())

    def mix(self, W, x, adjoint=False, out=None):
        """Per-degree channel mix out[b,c',l,m] = sum_c W[l,c',c] x[b,c,l,m]
        (adjoint: W_l^H).  W: complex64 [lmax, channels, channels]."""
        d = self.descs[0]
        C = d.get("channels", 1)
        self._check(W, torch.complex64, (d["lmax"], C, C), "W")
        self._check(x, torch.complex64, self.spec_shape(), "input")
        if out is None:
            out = torch.empty(self.spec_shape(), dtype=torch.complex64, device=self.device)
        self._check(out, torch.complex64, self.spec_shape(), "output")
        self._status(self._lib.sht_channel_mix(self._h, ctypes.c_void_p(W.data_ptr()),
                                               ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                               1 if adjoint else 0, _stream_ptr(self.device)))
        return out

    def mix_weight_grad(self, g, x, out=None):
        """Weight gradient of ``mix``: dW[l,c',c] = sum over b and m <= l of
        g[b,c',l,m] conj(x[b,c,l,m]) (complex64 [lmax, channels, channels])."""
        d = self.descs[0]
        C = d.get("channels", 1)
        self._check(g, torch.complex64, self.spec_shape(), "g")
        self._check(x, torch.complex64, self.spec_shape(), "x")
        if out is None:
            out = torch.empty((d["lmax"], C, C), dtype=torch.complex64, device=self.device)
        self._check(out, torch.complex64, (d["lmax"], C, C), "dW")
        self._status(self._lib.sht_channel_mix_weight_grad(self._h, ctypes.c_void_p(g.data_ptr()),
                                                           ctypes.c_void_p(x.data_ptr()),
                                                           ctypes.c_void_p(out.data_ptr()),
                                                           _stream_ptr(self.device)))
        return out

    def filter(self, k, x, adjoint=False, out=None):
        """Isotropic filter out[b,c,l,m] = k[c,l] x[b,c,l,m] (adjoint:
        conj(k)).  k: complex64 [channels, lmax]."""
        d = self.descs[0]
        C = d.get("channels", 1)
        self._check(k, torch.complex64, (C, d["lmax"]), "k")
        self._check(x, torch.complex64, self.spec_shape(), "input")
        if out is None:
            out = torch.empty(self.spec_shape(), dtype=torch.complex64, device=self.device)
        self._check(out, torch.complex64, self.spec_shape(), "output")
        self._status(self._lib.sht_isotropic_filter(self._h, ctypes.c_void_p(k.data_ptr()),
                                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                    1 if adjoint else 0, _stream_ptr(self.device)))
        return out

    def filter_grad(self, g, x, out=None):
        """Filter gradient dk[c,l] = sum over b and m <= l of g conj(x)."""
        d = self.descs[0]
        C = d.get("channels", 1)
        self._check(g, torch.complex64, self.spec_shape(), "g")
        self._check(x, torch.complex64, self.spec_shape(), "x")
        if out is None:
            out = torch.empty((C, d["lmax"]), dtype=torch.complex64, device=self.device)
        self._check(out, torch.complex64, (C, d["lmax"]), "dk")
        self._status(self._lib.sht_isotropic_filter_grad(self._h, ctypes.c_void_p(g.data_ptr()),
                                                         ctypes.c_void_p(x.data_ptr()),
                                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(self.device)))
        return out

    # ------------------------------------------------- scores and spectra
    def psd(self, y, out=None):
        """Angular power spectral density sum_{|m| <= l} |y_l^m|^2:
        float32 [batch, channels, lmax]."""
        d = self.descs[0]
        self._check(y, torch.complex64, self.spec_shape(), "y")
        shape = (d.get("batch", 1), d.get("channels", 1), d["lmax"])
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        self._check(out, torch.float32, shape, "out")
        self._status(self._lib.sht_psd(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       _stream_ptr(self.device)))
        return out

    def zonal_psd(self, x, out=None):
        """Zonal power spectral density 2 pi sin(t_k) |(2 pi/nlon) DFT_m|^2 of
        every ring: float32 [batch, channels, nlat, mmax]."""
        d = self.descs[0]
        self._check(x, torch.float32, self.grid_shape(), "x")
        shape = (d.get("batch", 1), d.get("channels", 1), d["nlat"], d["mmax"])
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        self._check(out, torch.float32, shape, "out")
        self._status(self._lib.sht_zonal_psd(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             _stream_ptr(self.device)))
        return out

    def spectral_crps(self, ens, obs, fair=False, l_hi=0, grad=False):
        """Spectral CRPS loss per channel over the ensemble (the plan's batch):
        returns loss float32 [channels] (and its gradient with respect to ens,
        complex64 like ens, when grad=True)."""
        d = self.descs[0]
        C = d.get("channels", 1)
        self._check(ens, torch.complex64, self.spec_shape(), "ens")
        self._check(obs, torch.complex64, (C, d["lmax"], d["mmax"]), "obs")
        loss = torch.empty(C, dtype=torch.float32, device=self.device)
        g = torch.empty_like(ens) if grad else None
        self._status(self._lib.sht_spectral_crps(self._h, ctypes.c_void_p(ens.data_ptr()),
                                                 ctypes.c_void_p(obs.data_ptr()), 1 if fair else 0, int(l_hi),
                                                 ctypes.c_void_p(loss.data_ptr()),
                                                 ctypes.c_void_p(g.data_ptr() if grad else None),
                                                 _stream_ptr(self.device)))
        return (loss, g) if grad else loss

    def spatial_crps(self, ens, obs, fair=False, grad=False):
        """Spatial CRPS loss per channel (quadrature average over the sphere)."""
        d = self.descs[0]
        C = d.get("channels", 1)
        self._check(ens, torch.float32, self.grid_shape(), "ens")
        self._check(obs, torch.float32, (C, d["nlat"], d["nlon"]), "obs")
        loss = torch.empty(C, dtype=torch.float32, device=self.device)
        g = torch.empty_like(ens) if grad else None
        self._status(self._lib.sht_spatial_crps(self._h, ctypes.c_void_p(ens.data_ptr()),
                                                ctypes.c_void_p(obs.data_ptr()), 1 if fair else 0,
                                                ctypes.c_void_p(loss.data_ptr()),
                                                ctypes.c_void_p(g.data_ptr() if grad else None),
                                                _stream_ptr(self.device)))
        return (loss, g) if grad else loss

    # ----------------------------------------------------- batching helpers
    def tune(self, cache=None):
        """Autotune the work schedule (sht_plan_tune); returns (candidate, ms),
        ms = -1.0 when the choice came from the cache file."""
        chosen, ms = ctypes.c_int(), ctypes.c_double()
        path = None if cache is None else str(cache).encode()
        self._status(self._lib.sht_plan_tune(self._h, path, ctypes.byref(chosen), ctypes.byref(ms)))
        return chosen.value, ms.value

    def set_schedule(self, chunk=8, policy=0, ncb=2, staged=1):
        """Set the work schedule explicitly (results do not change)."""
        self._status(self._lib.sht_plan_set_schedule(self._h, int(chunk), int(policy), int(ncb), int(staged)))

    def schedule(self):
        """(orders per chunk, XCD policy, field groups per workgroup, staged
        analysis output) in use."""
        c, p, n, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._status(self._lib.sht_plan_get_schedule(self._h, ctypes.byref(c), ctypes.byref(p), ctypes.byref(n),
                                                     ctypes.byref(st)))
        return c.value, p.value, n.value, st.value

    def graph(self, ops):
        """Capture a sequence [(op, input, output), ...] (op in "sht", "isht",
        "sht_T", "isht_T") into a replayable HIP graph (sht_graph_create)."""
        return Graph(self, ops)

    # ------------------------------------------------------------ diagnostics
    def set_timing(self, enable):
        """Record HIP events around every kernel launch of later calls."""
        self._status(self._lib.sht_plan_timing(self._h, 1 if enable else 0))

    def read_timing(self):
        """{kernel kind: (total ms, launches)} since the last read (synchronises)."""
        n = len(_lib.TIMING_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        self._status(self._lib.sht_plan_timing_read(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.TIMING_KINDS)}

    # --------------------------------------------------------------- lifetime
    def close(self):
        """Free the plan (raises ShtError while graphs of the plan exist)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            self._status(self._lib.sht_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_peaks(copy_bytes=1 << 30, iters=4096):
    """Measured machine peaks on the current GPU: HBM copy GB/s (read +
    written; the library's copy kernel and torch's device copy, the larger
    taken as the measured HBM peak), FP32 and BF16 matrix-core TFLOP/s
    (sht_measure_peak)."""
    lib = _lib.load()
    st = _stream_ptr(torch.cuda.current_device())
    out = {}
    for name, kind, size, scale in (("hbm_copy_GBs", 0, copy_bytes, 1e9), ("fp32_mfma_TFs", 1, iters, 1e12),
                                    ("bf16_mfma_TFs", 2, iters, 1e12)):
        r = ctypes.c_double()
        _lib.check(lib.sht_measure_peak(kind, size, ctypes.byref(r), st))
        out[name] = round(r.value / scale, 1)
    # torch's own device-to-device copy of the same size, for comparison
    a = torch.empty(copy_bytes // 4, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    e1.synchronize()
    out["torch_copy_GBs"] = round(2 * copy_bytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    out["hbm_measured_GBs"] = max(out["hbm_copy_GBs"], out["torch_copy_GBs"])
    del a, b
    return out


class SHT(torch.autograd.Function):
    """y = SHT(x); backward applies the hand-written adjoint (sht_backward)."""

    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.sht(x.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return ctx.plan.sht_T(gy.contiguous()), None


class ISHT(torch.autograd.Function):
    """x = ISHT(y); backward applies the hand-written adjoint (isht_backward)."""

    @staticmethod
    def forward(ctx, y, plan):
        ctx.plan = plan
        return plan.isht(y.contiguous())

    @staticmethod
    def backward(ctx, gx):
        return ctx.plan.isht_T(gx.contiguous()), None


class ChannelMix(torch.autograd.Function):
    """y = mix_W(x) per degree; backward gives the input gradient W_l^H g and,
    when W requires it, the weight gradient sum_{b, m <= l} g x^H."""

    @staticmethod
    def forward(ctx, x, W, plan):
        ctx.plan = plan
        x = x.contiguous()
        ctx.save_for_backward(W, x)
        return plan.mix(W, x)

    @staticmethod
    def backward(ctx, g):
        W, x = ctx.saved_tensors
        g = g.contiguous()
        gx = ctx.plan.mix(W, g, adjoint=True) if ctx.needs_input_grad[0] else None
        gW = ctx.plan.mix_weight_grad(g, x) if ctx.needs_input_grad[1] else None
        return gx, gW, None


class IsotropicFilter(torch.autograd.Function):
    """y = k_l x per channel and degree; backward gives conj(k) g and, when k
    requires it, the filter gradient sum_{b, m <= l} g conj(x)."""

    @staticmethod
    def forward(ctx, x, k, plan):
        ctx.plan = plan
        x = x.contiguous()
        ctx.save_for_backward(k, x)
        return plan.filter(k, x)

    @staticmethod
    def backward(ctx, g):
        k, x = ctx.saved_tensors
        g = g.contiguous()
        gx = ctx.plan.filter(k, g, adjoint=True) if ctx.needs_input_grad[0] else None
        gk = ctx.plan.filter_grad(g, x) if ctx.needs_input_grad[1] else None
        return gx, gk, None


class SpectralCRPS(torch.autograd.Function):
    """loss[c] = spectral CRPS of the ensemble spectra against the observed
    spectrum; backward scales the kernel's gradient by the incoming one."""

    @staticmethod
    def forward(ctx, ens, obs, plan, fair=False):
        loss, g = plan.spectral_crps(ens.contiguous(), obs.contiguous(), fair=fair, grad=True)
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        return g * gl.to(torch.complex64)[None, :, None, None], None, None, None


class SpatialCRPS(torch.autograd.Function):
    """loss[c] = spatial CRPS of the ensemble fields against the observed field."""

    @staticmethod
    def forward(ctx, ens, obs, plan, fair=False):
        loss, g = plan.spatial_crps(ens.contiguous(), obs.contiguous(), fair=fair, grad=True)
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        return g * gl[None, :, None, None], None, None, None


class Noise:
    """Spherical diffusion noise generator (sht_noise_*) on a single-segment
    plan: per channel length scale kT, time scale lam and amplitude sigma.
    step() advances the spectral state and returns (state, field)."""

    def __init__(self, plan, kT, lam, sigma, seed=0):
        d = plan.descs[0]
        C = d.get("channels", 1)
        arr = lambda v: (ctypes.c_double * C)(*[float(t) for t in (v if hasattr(v, "__len__") else [v] * C)])
        self.plan = plan
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().sht_noise_create(plan._h, arr(kT), arr(lam), arr(sigma), int(seed),
                                                ctypes.byref(self._h)))
        self.state = torch.zeros(plan.spec_shape(), dtype=torch.complex64, device=plan.device)

    def step(self, field=True, out=None):
        if field and out is None:
            out = torch.empty(self.plan.grid_shape(), dtype=torch.float32, device=self.plan.device)
        _lib.check(_lib.load().sht_noise_step(self._h, ctypes.c_void_p(self.state.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr() if field else None),
                                              _stream_ptr(self.plan.device)))
        return self.state, out

    def set_step(self, n):
        _lib.check(_lib.load().sht_noise_set_step(self._h, int(n)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().sht_noise_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured sequence of transforms on fixed buffers (sht_graph_*).  The
    tensors stay referenced by the graph; replay with launch()."""

    def __init__(self, plan, ops):
        lib = _lib.load()
        shapes = {"sht": ((torch.float32, plan.grid_shape()), (torch.complex64, plan.spec_shape())),
                  "isht": ((torch.complex64, plan.spec_shape()), (torch.float32, plan.grid_shape())),
                  "sht_T": ((torch.complex64, plan.spec_shape()), (torch.float32, plan.grid_shape())),
                  "isht_T": ((torch.float32, plan.grid_shape()), (torch.complex64, plan.spec_shape()))}
        n = len(ops)
        codes = (ctypes.c_int * n)()
        ins = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        self._keep = []
        for i, (op, src, dst) in enumerate(ops):
            if op not in _lib.OPS:
                raise ValueError(f"unknown op {op!r}")
            (sdt, sshape), (ddt, dshape) = shapes[op]
            plan._check(src, sdt, sshape, "input")
            plan._check(dst, ddt, dshape, "output")
            codes[i] = _lib.OPS[op]
            ins[i] = src.data_ptr()
            outs[i] = dst.data_ptr()
            self._keep += [src, dst]
        self.plan = plan
        self._h = ctypes.c_void_p()
        with torch.cuda.device(plan.device):
            _lib.check(lib.sht_graph_create(plan._h, n, codes, ins, outs, ctypes.byref(self._h)))

    def launch(self):
        _lib.check(_lib.load().sht_graph_launch(self._h, _stream_ptr(self.plan.device)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().sht_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
