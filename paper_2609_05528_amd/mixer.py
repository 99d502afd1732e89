"""Order mixers L of Sec. 3.1 eq. (4): the unresolved spatial image and the total-flux readout.

Argument marshalling only; the gather sums run in the HIP library (mixer_* / mix_* of
``include/rtt.h``).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import Geometry, _check, _dev_ptr, _nvec, _stream, require_native

RTT_MIX_UNRESOLVED, RTT_MIX_TOTAL_FLUX = 0, 1
KINDS = {"unresolved": RTT_MIX_UNRESOLVED, "total_flux": RTT_MIX_TOTAL_FLUX}


class rtt_mixer_info(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_geometries", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("n_src_rows", ctypes.c_int64), ("reserved", ctypes.c_int32 * 4)]


class Mixer:
    """Device gather tables of one order mixer over every geometry of a handle.

    ``kind``: "unresolved" or "total_flux".  ``pixels`` (unresolved only): one integer array per
    ray map, in the order the maps were loaded (geometry 0's orders first), giving the image pixel
    of each ray; indices are local to a geometry.
    """

    def __init__(self, geom: Geometry, kind: str, pixels=None):
        lib = require_native()
        if kind not in KINDS:
            raise ValueError("kind must be one of %s" % (tuple(KINDS),))
        arrays = None
        ptrs = None
        if pixels is not None:
            arrays = [np.ascontiguousarray(p, dtype=np.int64) for p in pixels]
            n_maps = sum(m["n_orders"] for m in geom.members)
            if len(arrays) != n_maps:
                raise ValueError("need one pixel array per ray map (%d), got %d" % (n_maps, len(arrays)))
            want = [n for m in geom.members for n in m["rays_per_order"]]
            for i, (a, n) in enumerate(zip(arrays, want)):
                if a.shape != (n,):
                    raise ValueError("pixel array %d has shape %s, expected (%d,)" % (i, a.shape, n))
            ptrs = (ctypes.POINTER(ctypes.c_int64) * len(arrays))(
                *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for a in arrays])
        h = ctypes.c_void_p()
        _check(lib.mixer_create(geom.handle, KINDS[kind], ptrs, ctypes.byref(h)))
        self._h = h
        self.kind = kind
        info = rtt_mixer_info()
        _check(lib.mixer_info(h, ctypes.byref(info)))
        self.n_rows = info.n_rows
        self.n_src_rows = info.n_src_rows
        self.n_geometries = info.n_geometries
        self.members = []
        for gi in range(self.n_geometries):
            off, n, n_out = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            _check(lib.mixer_member(h, gi, ctypes.byref(off), ctypes.byref(n), ctypes.byref(n_out)))
            self.members.append(dict(row_offset=off.value, n_rows=n.value, n_out=n_out.value))

    def set_variant(self, apply=-1, adjoint=-1):
        """Pin vectors per wave (1, 2, 4, 8; 0 = automatic) of the forward and transposed kernels."""
        _check(require_native().mixer_set_variant(self.handle, apply, adjoint))

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("mixer was freed")
        return self._h

    def free(self):
        from . import _lib
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.mixer_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mixer_create(geom: Geometry, kind: str, pixels=None) -> Mixer:
    return Mixer(geom, kind, pixels)


def mix_apply(mixer: Mixer, y, d=None, stream=None):
    """d = (L kron I) y.  y: [..., n_src_rows] float32 CUDA; returns d [..., n_rows]."""
    import torch
    nvec = _nvec(y, mixer.n_src_rows)
    if d is None:
        d = torch.empty(y.shape[:-1] + (mixer.n_rows,), dtype=torch.float32, device=y.device)
    _check(require_native().mix_apply(mixer.handle, _dev_ptr(y, nvec * mixer.n_src_rows, "y"),
                                      _dev_ptr(d, nvec * mixer.n_rows, "d"), nvec, _stream(stream)))
    return d


def mix_apply_noalloc(mixer: Mixer, y, d, stream=None):
    """d = (L kron I) y into the caller's d, through the library entry point that allocates no
    device memory (partial rows in a fixed per-GPU scratch array; see include/rtt.h)."""
    nvec = _nvec(y, mixer.n_src_rows)
    _check(require_native().mix_apply_noalloc(mixer.handle, _dev_ptr(y, nvec * mixer.n_src_rows, "y"),
                                              _dev_ptr(d, nvec * mixer.n_rows, "d"), nvec, _stream(stream)))
    return d


def mix_adjoint(mixer: Mixer, d, y=None, stream=None):
    """y = (L^T kron I) d.  d: [..., n_rows] float32 CUDA; returns y [..., n_src_rows]."""
    import torch
    nvec = _nvec(d, mixer.n_rows)
    if y is None:
        y = torch.empty(d.shape[:-1] + (mixer.n_src_rows,), dtype=torch.float32, device=d.device)
    _check(require_native().mix_adjoint(mixer.handle, _dev_ptr(d, nvec * mixer.n_rows, "d"),
                                        _dev_ptr(y, nvec * mixer.n_src_rows, "y"), nvec, _stream(stream)))
    return y


def mix_covariance(mixer: Mixer, var, out=None, stream=None):
    """Diagonal of C_L = (L kron I) diag(var) (L^T kron I).  var: [n_src_rows] float32 CUDA."""
    import torch
    if out is None:
        out = torch.empty(mixer.n_rows, dtype=torch.float32, device=var.device)
    _check(require_native().mix_covariance(mixer.handle, _dev_ptr(var, mixer.n_src_rows, "var"),
                                           _dev_ptr(out, mixer.n_rows, "var_out"), _stream(stream)))
    return out
