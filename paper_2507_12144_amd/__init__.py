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

__all__ = ["Plan", "SHT", "ISHT", "ChannelMix", "ShtError", "GRIDS", "PRECISIONS"]


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A transform plan for one or more (nlat, nlon, lmax, mmax, grid, batch,
    channels) shapes.  With one shape, tensors keep their natural shapes
    [batch, channels, nlat, nlon] (float32) and [batch, channels, lmax, mmax]
    (complex64).  With several shapes (the batching form) tensors are flat
    concatenations; ``segment(i)`` gives each shape's offsets."""

    def __init__(self, descs, precision="fp32", device=None):
        lib = _lib.load()
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
            _lib.check(lib.sht_plan(ctypes.byref(self._h), arr, len(self.descs), prec,
                                    _stream_ptr(self.device)))
        g, s = ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(lib.sht_plan_sizes(self._h, ctypes.byref(g), ctypes.byref(s)))
        self.grid_elems, self.spec_elems = g.value, s.value

    # ------------------------------------------------------------------ info
    def segment(self, i):
        g, s = ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(_lib.load().sht_plan_segment(self._h, i, ctypes.byref(g), ctypes.byref(s)))
        return g.value, s.value

    def grid(self, i=0):
        """(x_k, w_k) of segment i as float64 host tensors."""
        n = self.descs[i]["nlat"]
        x = (ctypes.c_double * n)()
        w = (ctypes.c_double * n)()
        _lib.check(_lib.load().sht_plan_grid(self._h, i, x, w))
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
        _lib.check(fn(self._h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                      _stream_ptr(self.device)))
        return dst

    def sht(self, x, out=None):
        """Forward SHT: float32 grid -> complex64 spectrum."""
        return self._call(_lib.load().sht_forward, x, torch.float32, self.grid_shape(), out,
                          torch.complex64, self.spec_shape())

    def isht(self, y, out=None):
        """Inverse SHT: complex64 spectrum -> float32 grid."""
        return self._call(_lib.load().isht_forward, y, torch.complex64, self.spec_shape(), out,
                          torch.float32, self.grid_shape())

    def sht_T(self, gy, out=None):
        """Adjoint of ``sht`` (sht_backward)."""
        return self._call(_lib.load().sht_backward, gy, torch.complex64, self.spec_shape(), out,
                          torch.float32, self.grid_shape())

    def isht_T(self, gx, out=None):
        """Adjoint of ``isht`` (isht_backward)."""
        return self._call(_lib.load().isht_backward, gx, torch.float32, self.grid_shape(), out,
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
        _lib.check(_lib.load().sht_channel_mix(self._h, ctypes.c_void_p(W.data_ptr()),
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
        _lib.check(_lib.load().sht_channel_mix_weight_grad(self._h, ctypes.c_void_p(g.data_ptr()),
                                                           ctypes.c_void_p(x.data_ptr()),
                                                           ctypes.c_void_p(out.data_ptr()),
                                                           _stream_ptr(self.device)))
        return out

    # ----------------------------------------------------- batching helpers
    def tune(self, cache=None):
        """Autotune the work schedule (sht_plan_tune); returns (candidate, ms),
        ms = -1.0 when the choice came from the cache file."""
        chosen, ms = ctypes.c_int(), ctypes.c_double()
        path = None if cache is None else str(cache).encode()
        _lib.check(_lib.load().sht_plan_tune(self._h, path, ctypes.byref(chosen), ctypes.byref(ms)))
        return chosen.value, ms.value

    def graph(self, ops):
        """Capture a sequence [(op, input, output), ...] (op in "sht", "isht",
        "sht_T", "isht_T") into a replayable HIP graph (sht_graph_create)."""
        return Graph(self, ops)

    # ------------------------------------------------------------ diagnostics
    def set_timing(self, enable):
        """Record HIP events around every kernel launch of later calls."""
        _lib.check(_lib.load().sht_plan_timing(self._h, 1 if enable else 0))

    def read_timing(self):
        """{kernel kind: (total ms, launches)} since the last read (synchronises)."""
        n = len(_lib.TIMING_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        _lib.check(_lib.load().sht_plan_timing_read(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.TIMING_KINDS)}

    # --------------------------------------------------------------- lifetime
    def close(self):
        """Free the plan (raises ShtError while graphs of the plan exist)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().sht_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
