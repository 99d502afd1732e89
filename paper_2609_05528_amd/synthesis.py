"""Representation synthesis Q_d (Sec. 3.2 eq. (5)-(8), Sec. 7) and the rank audit of A Q_d.

Argument marshalling only over synthesis_* / synth_* of ``include/rtt.h``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import Geometry, _check, _dev_ptr, _nvec, _stream, require_native

RTT_SYNTH_DCT, RTT_SYNTH_HATS = 0, 1


class rtt_synthesis_spec(ctypes.Structure):
    _fields_ = [("n_radial", ctypes.c_int32), ("m_max", ctypes.c_int32), ("n_temporal", ctypes.c_int32),
                ("temporal", ctypes.c_int32), ("t_lo", ctypes.c_double), ("t_hi", ctypes.c_double),
                ("reserved", ctypes.c_int32 * 4)]


class Synthesis:
    """Q_d on the coefficient nodes of geometry ``g`` of a handle (S_224: the defaults)."""

    def __init__(self, geom: Geometry, g: int = 0, n_radial: int = 4, m_max: int = 3, n_temporal: int = 8,
                 temporal: str = "dct", window=None):
        lib = require_native()
        if temporal not in ("dct", "hats"):
            raise ValueError("temporal must be 'dct' or 'hats'")
        t_lo, t_hi = (0.0, 0.0) if window is None else (float(window[0]), float(window[1]))
        spec = rtt_synthesis_spec(n_radial, m_max, n_temporal, RTT_SYNTH_DCT if temporal == "dct" else RTT_SYNTH_HATS,
                                  t_lo, t_hi)
        h = ctypes.c_void_p()
        _check(lib.synthesis_create(geom.handle, int(g), ctypes.byref(spec), ctypes.byref(h)))
        self._h = h
        d, n = ctypes.c_int32(), ctypes.c_int64()
        _check(lib.synthesis_info(h, ctypes.byref(d), ctypes.byref(n), None))
        self.d, self.n_cols, self.member = d.value, n.value, int(g)
        self.n_temporal = int(n_temporal)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("synthesis was freed")
        return self._h

    def expand(self, c, x=None, stream=None):
        """x = Q c: c float32 CUDA [..., d] -> x [..., n_cols]."""
        import torch
        nvec = _nvec(c, self.d)
        if x is None:
            x = torch.empty(c.shape[:-1] + (self.n_cols,), dtype=torch.float32, device=c.device)
        _check(require_native().synth_expand(self.handle, _dev_ptr(c, nvec * self.d, "c"),
                                             _dev_ptr(x, nvec * self.n_cols, "x"), nvec, _stream(stream)))
        return x

    def project(self, x, c=None, stream=None):
        """c = Q^T x: x float32 CUDA [..., n_cols] -> c [..., d]."""
        import torch
        nvec = _nvec(x, self.n_cols)
        if c is None:
            c = torch.empty(x.shape[:-1] + (self.d,), dtype=torch.float32, device=x.device)
        _check(require_native().synth_project(self.handle, _dev_ptr(x, nvec * self.n_cols, "x"),
                                              _dev_ptr(c, nvec * self.d, "c"), nvec, _stream(stream)))
        return c

    def audit(self, geom: Geometry, order_mask: int = 0, rel_tol: float = 1e-6, stream=None):
        """Exactly zero columns, singular values and numerical rank (at rel_tol * sigma_1) of A Q."""
        sigma = np.zeros(self.d)
        zero = np.zeros(self.d, dtype=np.uint8)
        _check(require_native().synthesis_audit(geom.handle, self.handle, int(order_mask),
                                                sigma.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                zero.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _stream(stream)))
        rank = int(np.sum(sigma > rel_tol * sigma[0])) if sigma[0] > 0 else 0
        return dict(zero_columns=[int(c) for c in np.nonzero(zero)[0]], sigma=sigma, rank=rank)

    def age_fisher(self, geom: Geometry, ages, h: float = 3.0, order_mask: int = 0, stream=None):
        """M(a) of eq. (14) for the localised probes built on this synthesis' spatial functions:
        numpy [n_ages][L][L], L = n_radial (2 m_max + 1)."""
        ages = np.ascontiguousarray(ages, dtype=np.float64)
        L = self.d // self.n_temporal
        out = np.zeros((ages.size, L, L))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(require_native().age_fisher(geom.handle, self.handle, ages.ctypes.data_as(dp), ages.size, float(h),
                                           int(order_mask), out.ctypes.data_as(dp), _stream(stream)))
        return out

    def free(self):
        from . import _lib
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.synthesis_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
