"""Age-localised probes and historical reach (Sec. 3.3, 3.5, 4.4; eq. (10)-(13), (17), (29)-(30), (35)).

Argument marshalling only over the age_* / reference_response calls of ``include/rtt.h``.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import Geometry, _check, _dev_ptr, _stream, require_native

_dp = ctypes.POINTER(ctypes.c_double)


class rtt_reach(ctypes.Structure):
    _fields_ = [("t_reach", ctypes.c_double), ("l_anchor", ctypes.c_double), ("longest", ctypes.c_double),
                ("j_old", ctypes.c_double), ("anchor", ctypes.c_int32), ("n_pass", ctypes.c_int32)]


def reference_response(geom: Geometry, stream=None):
    """s_ref of eq. (17) for every geometry of the handle (numpy [G])."""
    out = np.zeros(geom.n_geometries)
    _check(require_native().reference_response(geom.handle, out.ctypes.data_as(_dp), _stream(stream)))
    return out


def age_information(geom: Geometry, ages, h: float = 3.0, mixer=None, var=None, stream=None):
    """Squared probe responses of eq. (12)/(29): numpy [n_ages][G][8] per order, or [n_ages][G]
    through an order mixer (var: per-datum variances, float32 CUDA [n_rows], default 1)."""
    ages = np.ascontiguousarray(ages, dtype=np.float64)
    G = geom.n_geometries
    out = np.zeros((ages.size, G) if mixer is not None else (ages.size, G, 8))
    vp = None if var is None else _dev_ptr(var, geom.n_rows, "var")
    _check(require_native().age_information(geom.handle, ages.ctypes.data_as(_dp), ages.size, float(h),
                                            None if mixer is None else mixer.handle, vp,
                                            out.ctypes.data_as(_dp), _stream(stream)))
    return out


def age_window(geom: Geometry, g: int = 0, order_mask: int = 0, h: float = 3.0, q: float = 0.999):
    """(a_min, a_max, A_{0,q}): fully supported ages (eq. (13)) and the direct throughput boundary."""
    a0, a1, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(require_native().age_window(geom.handle, g, order_mask, float(h), float(q), ctypes.byref(a0),
                                       ctypes.byref(a1), ctypes.byref(b)))
    return a0.value, a1.value, b.value


def age_reach(ages, info, rho: float = 1.0, a_min: float = -math.inf, a_max: float = math.inf,
              boundary: float = math.nan):
    """Threshold statistics on an age grid: dict(mask, t_reach, anchor, l_anchor, longest, j_old, n_pass);
    NaN / None where a statistic does not exist."""
    ages = np.ascontiguousarray(ages, dtype=np.float64)
    info = np.ascontiguousarray(info, dtype=np.float64)
    if info.shape != ages.shape:
        raise ValueError("ages and info differ in shape")
    mask = np.zeros(ages.size, dtype=np.uint8)
    r = rtt_reach()
    _check(require_native().age_reach(ages.ctypes.data_as(_dp), info.ctypes.data_as(_dp), ages.size, float(rho),
                                      float(a_min), float(a_max), float(boundary),
                                      mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(r)))

    def opt(v):
        return None if math.isnan(v) else v

    return dict(mask=mask.astype(bool), t_reach=opt(r.t_reach), anchor=None if r.anchor < 0 else r.anchor,
                l_anchor=opt(r.l_anchor), longest=opt(r.longest), j_old=opt(r.j_old), n_pass=r.n_pass)


def age_window_error(geom: Geometry, x_hat, x, ages, half_width: float = 2.0, eta: float = 1e-12, stream=None):
    """E(a) of eq. (32): numpy [nvec][G][n_ages] (x_hat, x: float32 CUDA [nvec][n_cols])."""
    from . import _nvec
    ages = np.ascontiguousarray(ages, dtype=np.float64)
    nvec = _nvec(x, geom.n_cols)
    out = np.zeros((nvec, geom.n_geometries, ages.size))
    _check(require_native().age_window_error(geom.handle, _dev_ptr(x_hat, nvec * geom.n_cols, "x_hat"),
                                             _dev_ptr(x, nvec * geom.n_cols, "x"), nvec, ages.ctypes.data_as(_dp),
                                             ages.size, float(half_width), float(eta), out.ctypes.data_as(_dp),
                                             _stream(stream)))
    return out


def noise_add(y, seed: int, sigma: float, stream=None):
    """y += sigma * N(0, 1) seeded draws (Philox-4x32-10 + Box-Muller; see include/rtt.h), in place."""
    _check(require_native().noise_add(_dev_ptr(y, None, "y"), y.numel(), int(seed) & (2 ** 64 - 1), float(sigma),
                                      _stream(stream)))
    return y
