"""MI355X MOFF direct imager: Python binding of the HIP library (include/moff.h).

`Plan` marshals a geometry and torch device tensors into the C ABI; every step
of the imaging path (calibration, gridding, the padded 2-D FFT, squaring,
accumulation and self-power removal) runs in the gfx950 kernels of libmoff.so.
Shapes, dtypes and devices are checked here before any pointer is passed on,
since the C side cannot see the extent of a device buffer.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (MOFF_AUTOCORR_NONE, MOFF_AUTOCORR_UV, MOFF_IN_C64, MOFF_IN_CI4, MOFF_MFMA_BF16,  # noqa: F401
                   MOFF_MFMA_F16, MOFF_NORM_PAIRS, MoffError, moff_geometry)

__all__ = ["Plan", "MoffError", "MOFF_IN_C64", "MOFF_IN_CI4", "MOFF_AUTOCORR_NONE", "MOFF_NORM_PAIRS",
           "MOFF_MFMA_F16", "MOFF_MFMA_BF16", "MOFF_AUTOCORR_UV", "library_path", "moff_image_autograd"]


def library_path():
    return _lib.LIB_PATH


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Plan:
    """A MOFF plan on one device (device < 0: host-only, for queries)."""

    def __init__(self, ant_xy, ktype_k, ktype_vals, ant_ktype, freq_hz, grid_n, cell_m=0.0, flags=0, device=0):
        self._xy = np.ascontiguousarray(ant_xy, dtype=np.float64).reshape(-1, 2)
        self._k = np.ascontiguousarray(ktype_k, dtype=np.int32).reshape(-1)
        tabs = [np.ascontiguousarray(t, dtype=np.complex64) for t in ktype_vals]
        for k, t in zip(self._k, tabs):
            if t.shape != (k, k):
                raise ValueError(f"kernel table shape {t.shape} does not match k={k}")
        if len(tabs) != len(self._k):
            raise ValueError("one table per kernel type is required")
        self._vals = np.ascontiguousarray(np.concatenate([t.reshape(-1) for t in tabs]).view(np.float32))
        self._types = np.ascontiguousarray(ant_ktype, dtype=np.int32).reshape(-1)
        self._freq = np.ascontiguousarray(freq_hz, dtype=np.float64).reshape(-1)
        if self._types.shape[0] != self._xy.shape[0]:
            raise ValueError("ant_ktype must have one entry per antenna")
        g = moff_geometry()
        g.n_ant = self._xy.shape[0]
        g.ant_xy_m = _ptr(self._xy, ctypes.c_double)
        g.n_ktypes = self._k.shape[0]
        g.ktype_k = _ptr(self._k, ctypes.c_int32)
        g.ktype_vals = _ptr(self._vals, ctypes.c_float)
        g.ant_ktype = _ptr(self._types, ctypes.c_int32)
        g.n_chan = self._freq.shape[0]
        g.freq_hz = _ptr(self._freq, ctypes.c_double)
        g.grid_n = int(grid_n)
        g.cell_m = float(cell_m)
        g.flags = int(flags)
        self.device = int(device)
        self.flags = int(flags)
        self.n_ant = int(g.n_ant)
        self.n_chan = int(g.n_chan)
        self.n_ktypes = int(g.n_ktypes)
        self.N = int(grid_n)
        self.handle = None
        self.handle = _lib.moff_plan_create(g, self.device)

    @classmethod
    def from_geometry(cls, geom, device=0, extra_flags=0):
        """Build from any object with the fields of the C geometry (ant_xy, ktype_k,
        ktype_vals, ant_ktype, freq_hz, grid_n, cell_m, flags); extra_flags are
        OR-ed into flags (e.g. MOFF_MFMA_F16)."""
        return cls(geom.ant_xy, geom.ktype_k, geom.ktype_vals, geom.ant_ktype, geom.freq_hz, geom.grid_n,
                   geom.cell_m, int(geom.flags) | int(extra_flags), device)

    # ---- lifetime --------------------------------------------------------
    def close(self):
        if self.handle:
            _lib.moff_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- host queries ----------------------------------------------------
    @property
    def ci4(self):
        return bool(self.flags & MOFF_IN_CI4)

    def cells(self):
        out = np.zeros((self.n_ant, 2), np.int32)
        _lib.moff_plan_query(self.handle, _ptr(out, ctypes.c_int32), None, None, None)
        return out

    def cell_m(self):
        v = ctypes.c_double()
        _lib.moff_plan_query(self.handle, None, ctypes.byref(v), None, None)
        return v.value

    def lm_per_pixel(self):
        out = np.zeros(self.n_chan, np.float64)
        _lib.moff_plan_query(self.handle, None, None, _ptr(out, ctypes.c_double), None)
        return out

    def power_pattern(self, ktype):
        out = np.zeros((self.N, self.N), np.float64)
        _lib.moff_plan_power_pattern(self.handle, int(ktype), _ptr(out, ctypes.c_double))
        return out

    def gather_program(self, w, variant=0):
        """(entries uint32 [prog_len, n_threads, 2], weights complex64, sizes) of class w."""
        sizes = [ctypes.c_int32() for _ in range(5)]
        _lib.moff_plan_gather_program(self.handle, int(variant), 0, None, None, *[ctypes.byref(s) for s in sizes])
        plen, nt, ncls, pitch, nw = (s.value for s in sizes)
        out = np.zeros((plen, nt, 2), np.uint32)
        wts = np.zeros(2 * nw, np.float32)
        _lib.moff_plan_gather_program(self.handle, int(variant), int(w), _ptr(out, ctypes.c_uint32),
                                      _ptr(wts, ctypes.c_float), *[ctypes.byref(s) for s in sizes])
        return out, wts.view(np.complex64), dict(prog_len=plen, n_threads=nt, n_classes=ncls, row_pitch=pitch)

    def mfma_tables(self):
        """(gather entries uint32 [prog_len, n_threads, 2], phase-factor operand bit
        patterns uint16 [2, N/64, 2, N/64, 2, 64, 8], sizes) of a MOFF_MFMA_* plan."""
        sizes = [ctypes.c_int32() for _ in range(5)]
        _lib.moff_plan_mfma_tables(self.handle, None, None, *[ctypes.byref(s) for s in sizes])
        plen, nt, pitch, base, ndft = (s.value for s in sizes)
        prog = np.zeros((plen, nt, 2), np.uint32)
        dft = np.zeros(ndft, np.uint16)
        _lib.moff_plan_mfma_tables(self.handle, _ptr(prog, ctypes.c_uint32), _ptr(dft, ctypes.c_uint16),
                                   *[ctypes.byref(s) for s in sizes])
        N = self.N
        return prog, dft.reshape(2, N // 64, 2, N // 64, 2, 64, 8), dict(prog_len=plen, n_threads=nt, row_pitch=pitch,
                                                                     grid_base=base)

    def autotune(self, E, gains=None, stream=None):
        """Time every launch configuration on this input and keep the fastest."""
        pE, T = self._E(E)
        _lib.moff_plan_autotune(self.handle, pE, T, self._gains(gains), self._stream(stream))
        return self.config(T)

    def set_config(self, variant=0, slices=0):
        _lib.moff_plan_set_config(self.handle, int(variant), int(slices))

    def config(self, n_time):
        return _lib.moff_plan_get_config(self.handle, int(n_time))

    def set_timing(self, enable=True):
        _lib.moff_plan_set_timing(self.handle, enable)

    def last_kernel_ms(self):
        return _lib.moff_plan_last_kernel_ms(self.handle)

    # ---- device calls ----------------------------------------------------
    def _torch(self):
        import torch
        return torch

    def _dev(self, t, name, shape, dtype):
        torch = self._torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must live on cuda:{self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr()

    def _stream(self, stream):
        torch = self._torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return s.cuda_stream

    def _E(self, E):
        torch = self._torch()
        if E.dim() != 3:
            raise ValueError("E must be [n_time, n_chan, n_ant]")
        T = E.shape[0]
        dt = torch.uint8 if self.ci4 else torch.complex64
        return self._dev(E, "E", (T, self.n_chan, self.n_ant), dt), T

    def _gains(self, gains):
        if gains is None:
            return None
        return self._dev(gains, "gains", (self.n_chan, self.n_ant), self._torch().complex64)

    def _new(self, shape, dtype):
        torch = self._torch()
        return torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")

    def image(self, E, gains=None, out=None, stream=None):
        """Fused path: time-averaged image float32 [n_chan, N, N]."""
        torch = self._torch()
        pE, T = self._E(E)
        if out is None:
            out = self._new((self.n_chan, self.N, self.N), torch.float32)
        po = self._dev(out, "out", (self.n_chan, self.N, self.N), torch.float32)
        _lib.moff_image(self.handle, pE, T, self._gains(gains), po, self._stream(stream))
        return out

    def image_noalloc(self, E, gains=None, out=None, stream=None):
        """As image(), with every scratch buffer in the library's fixed per-GPU
        array (moff_image_noalloc); `out` must be given when nothing may be allocated."""
        torch = self._torch()
        pE, T = self._E(E)
        if out is None:
            out = self._new((self.n_chan, self.N, self.N), torch.float32)
        po = self._dev(out, "out", (self.n_chan, self.N, self.N), torch.float32)
        _lib.moff_image_noalloc(self.handle, pE, T, self._gains(gains), po, self._stream(stream))
        return out

    def accumulate(self, E, S, A, gains=None, stream=None):
        torch = self._torch()
        pE, T = self._E(E)
        pS = self._dev(S, "S", (self.n_chan, self.N, self.N), torch.float32)
        pA = self._dev(A, "A", (self.n_chan, self.n_ktypes), torch.float64)
        _lib.moff_accumulate(self.handle, pE, T, self._gains(gains), pS, pA, self._stream(stream))

    def finalize(self, S, A, n_time_total, out=None, stream=None):
        torch = self._torch()
        pS = self._dev(S, "S", (self.n_chan, self.N, self.N), torch.float32)
        pA = self._dev(A, "A", (self.n_chan, self.n_ktypes), torch.float64)
        if out is None:
            out = self._new((self.n_chan, self.N, self.N), torch.float32)
        po = self._dev(out, "out", (self.n_chan, self.N, self.N), torch.float32)
        _lib.moff_finalize(self.handle, pS, pA, int(n_time_total), po, self._stream(stream))
        return out

    def grid(self, E, gains=None, out=None, stream=None):
        torch = self._torch()
        pE, T = self._E(E)
        L = self.N // 2
        if out is None:
            out = self._new((T, self.n_chan, L, L), torch.complex64)
        po = self._dev(out, "out", (T, self.n_chan, L, L), torch.complex64)
        _lib.moff_grid(self.handle, pE, T, self._gains(gains), po, self._stream(stream))
        return out

    def self_power(self, E, A, gains=None, stream=None):
        torch = self._torch()
        pE, T = self._E(E)
        pA = self._dev(A, "A", (self.n_chan, self.n_ktypes), torch.float64)
        _lib.moff_self_power(self.handle, pE, T, self._gains(gains), pA, self._stream(stream))

    def fft2(self, eg, out=None, stream=None):
        torch = self._torch()
        L = self.N // 2
        lead = tuple(eg.shape[:-2])
        F = int(np.prod(lead)) if lead else 1
        if tuple(eg.shape[-2:]) != (L, L):
            raise ValueError(f"eg must end in ({L}, {L})")
        pe = self._dev(eg, "eg", tuple(eg.shape), torch.complex64)
        if out is None:
            out = self._new(lead + (self.N, self.N), torch.complex64)
        po = self._dev(out, "out", lead + (self.N, self.N), torch.complex64)
        _lib.moff_fft2(self.handle, pe, F, po, self._stream(stream))
        return out

    def detect_accumulate(self, Y, S, stream=None):
        torch = self._torch()
        T = Y.shape[0]
        pY = self._dev(Y, "Y", (T, self.n_chan, self.N, self.N), torch.complex64)
        pS = self._dev(S, "S", (self.n_chan, self.N, self.N), torch.float32)
        _lib.moff_detect_accumulate(self.handle, pY, T, pS, self._stream(stream))

    def image_staged(self, E, gains=None, out=None, stream=None):
        """Staged path (each step through HBM): same result as image()."""
        torch = self._torch()
        pE, T = self._E(E)
        if out is None:
            out = self._new((self.n_chan, self.N, self.N), torch.float32)
        po = self._dev(out, "out", (self.n_chan, self.N, self.N), torch.float32)
        _lib.moff_image_staged(self.handle, pE, T, self._gains(gains), po, self._stream(stream))
        return out

    def set_adjoint_waves(self, waves_per_simd):
        """Register budget of the fused gain adjoint: waves per SIMD (1, or 2 at grid 256)."""
        _lib.moff_plan_set_adjoint_waves(self.handle, int(waves_per_simd))

    def adjoint_waves(self):
        """(waves per SIMD in use, largest available) for the fused gain adjoint."""
        w, m = ctypes.c_int32(), ctypes.c_int32()
        _lib.moff_plan_get_adjoint_waves(self.handle, ctypes.byref(w), ctypes.byref(m))
        return w.value, m.value

    def image_fx(self, E, gains=None, out=None, stream=None):
        """Visibility-route (FX) image of the same integration: pair
        cross-products gridded with the tables' pair responses and transformed
        once; equals image() to rounding (zero spacings as for image())."""
        torch = self._torch()
        pE, T = self._E(E)
        if out is None:
            out = self._new((self.n_chan, self.N, self.N), torch.float32)
        po = self._dev(out, "out", (self.n_chan, self.N, self.N), torch.float32)
        _lib.moff_image_fx(self.handle, pE, T, self._gains(gains), po, self._stream(stream))
        return out

    def gain_vjp(self, E, gains, dL_dimage, out=None, stream=None, staged=False):
        """dL/dRe(g) + i dL/dIm(g) (complex64 [n_chan, n_ant]) for R = dL/dI
        (staged=True: the HBM-staged form of the same computation)."""
        torch = self._torch()
        pE, T = self._E(E)
        pR = self._dev(dL_dimage, "dL_dimage", (self.n_chan, self.N, self.N), torch.float32)
        if out is None:
            out = self._new((self.n_chan, self.n_ant), torch.complex64)
        po = self._dev(out, "out", (self.n_chan, self.n_ant), torch.complex64)
        fn = _lib.moff_gain_vjp_staged if staged else _lib.moff_gain_vjp
        fn(self.handle, pE, T, self._gains(gains), pR, po, self._stream(stream))
        return out


def _make_autograd():
    import torch

    class MoffImage(torch.autograd.Function):
        """Differentiable MOFF image: I = MoffImage.apply(plan, E, gains).

        Forward runs the fused imaging kernel; backward runs the gain adjoint
        (moff_gain_vjp) and returns dL/dgains in torch's complex convention.  E is
        not differentiated (raw antenna samples)."""

        @staticmethod
        def forward(ctx, plan, E, gains):
            ctx.plan = plan
            ctx.save_for_backward(E, gains)
            return plan.image(E, gains.detach().contiguous())

        @staticmethod
        def backward(ctx, grad_out):
            E, gains = ctx.saved_tensors
            g = None
            if ctx.needs_input_grad[2]:
                g = ctx.plan.gain_vjp(E, gains.detach().contiguous(), grad_out.contiguous().float())
            return None, None, g

    return MoffImage


_autograd_cls = None


def moff_image_autograd(plan, E, gains):
    """I = MOFF image of E with gains `gains` (a complex64 tensor that may require grad)."""
    global _autograd_cls
    if _autograd_cls is None:
        _autograd_cls = _make_autograd()
    return _autograd_cls.apply(plan, E, gains)
