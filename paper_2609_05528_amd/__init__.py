"""Python binding of librtt (MI355X retarded-time tomography operator).

Argument marshalling only: every step of the operator, the spectral drivers
and the solvers runs in the HIP library.  Tensors are torch CUDA (ROCm)
tensors; their device memory and the current stream are passed through the
C ABI of ``include/rtt.h``.  The binding fails loudly when the library has
not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtt.so")

RTT_OK, RTT_EINVAL, RTT_ENOMEM, RTT_EDEVICE, RTT_ENOCONV, RTT_ESTATE = 0, -1, -2, -3, -4, -5
RTT_SVD_RSVD, RTT_SVD_BLOCK_LANCZOS = 0, 1
RTT_SOLVE_ASYNC = 1
RTT_SOLVE_NORMAL_RHS = 2
RTT_EACH_GEOMETRY = -2

EXPORTED = ("geometry_load", "geometry_free", "geometry_info", "geometry_member", "geometry_set_variant",
            "geometry_set_batch_mode", "variant_name", "geometry_tune", "op_apply", "op_apply_shared", "op_apply_adjoint", "rsvd", "svd_free", "svd_get",
            "svd_converged", "tsvd_solve", "ridge_solve", "mixer_create", "mixer_free", "mixer_info", "mixer_member", "mixer_set_variant",
            "mix_apply", "mix_apply_noalloc", "mix_adjoint", "mix_covariance", "reference_response", "age_information", "age_window",
            "age_reach", "age_window_error", "tsvd_project", "noise_add", "synthesis_create", "synthesis_free",
            "synthesis_info", "synth_expand", "synth_project", "synthesis_audit", "age_fisher", "last_error")


class RttError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rtt error %d: %s" % (code, msg))
        self.code = code


class NoConvergence(RttError):
    pass


# ----------------------------------------------------------------------------------- C structs
class rtt_grid(ctypes.Structure):
    _fields_ = [("n_orders", ctypes.c_int32), ("n_frames", ctypes.c_int32),
                ("t0", ctypes.c_double), ("dt_obs", ctypes.c_double),
                ("n_r", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("n_hat", ctypes.c_int32), ("s0", ctypes.c_double), ("dt_src", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)


class rtt_raymap(ctypes.Structure):
    _fields_ = [("n_rays", ctypes.c_int64), ("r_src", _dp), ("phi_src", _dp), ("delay", _dp),
                ("weight", _dp), ("pixel_area", _dp)]


class rtt_load_opts(ctypes.Structure):
    _fields_ = [("sigma_omega", ctypes.c_double), ("drop_invalid", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class rtt_geometry_info(ctypes.Structure):
    _fields_ = [("n_geometries", ctypes.c_int32), ("n_rows", ctypes.c_int64),
                ("n_cols", ctypes.c_int64), ("n_rays", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("batch_apply_mode", ctypes.c_int32), ("batch_adjoint_mode", ctypes.c_int32),
                ("apply_launches", ctypes.c_int32), ("adjoint_launches", ctypes.c_int32)]


class rtt_member_info(ctypes.Structure):
    _fields_ = [("grid", rtt_grid), ("row_offset", ctypes.c_int64), ("n_rows", ctypes.c_int64),
                ("col_offset", ctypes.c_int64), ("n_cols", ctypes.c_int64),
                ("rays_per_order", ctypes.c_int64 * 8), ("apply_variant", ctypes.c_int32),
                ("adjoint_variant", ctypes.c_int32), ("digest", ctypes.c_uint64)]


class rtt_svd_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("k", ctypes.c_int32), ("p", ctypes.c_int32),
                ("q", ctypes.c_int32), ("block", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("order_mask", ctypes.c_uint32), ("geometry", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("keep_u", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class rtt_cg_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_float), ("maxit", ctypes.c_int32), ("order_mask", ctypes.c_uint32),
                ("flags", ctypes.c_int32), ("resid_dev", ctypes.c_void_p), ("reserved", ctypes.c_int32 * 2)]


class rtt_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_float), ("reserved", ctypes.c_int32)]


# ----------------------------------------------------------------------------------- loading
_lib = None


def lib_available() -> bool:
    return os.path.exists(LIB_PATH)


def require_native():
    """Load librtt.so or raise: the product path has no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librtt.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2609_05528_amd.build_lib)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
    sig = {
        "geometry_load": [ctypes.POINTER(rtt_grid), ctypes.POINTER(rtt_raymap), i32,
                          ctypes.POINTER(rtt_load_opts), ctypes.POINTER(vp)],
        "geometry_free": [vp],
        "geometry_info": [vp, ctypes.POINTER(rtt_geometry_info)],
        "geometry_member": [vp, i32, ctypes.POINTER(rtt_member_info)],
        "geometry_set_variant": [vp, i32, i32, i32],
        "geometry_set_batch_mode": [vp, i32, i32],
        "geometry_tune": [vp, i32, i32, ctypes.c_char_p, vp],
        "op_apply": [vp, vp, vp, i32, u32, vp],
        "op_apply_shared": [vp, vp, vp, i32, u32, vp],
        "op_apply_adjoint": [vp, vp, vp, i32, u32, vp],
        "rsvd": [vp, ctypes.POINTER(rtt_svd_opts), vp, ctypes.POINTER(vp), vp],
        "svd_free": [vp],
        "svd_get": [vp, ctypes.POINTER(i32), _dp, ctypes.POINTER(vp), ctypes.POINTER(vp), _dp],
        "svd_converged": [vp, ctypes.c_double, ctypes.POINTER(i32)],
        "tsvd_solve": [vp, vp, vp, i32, i32, ctypes.c_double, vp, vp],
        "ridge_solve": [vp, vp, i32, ctypes.c_float, ctypes.POINTER(rtt_cg_opts), vp,
                        ctypes.POINTER(rtt_solve_info), vp],
        "mixer_create": [vp, i32, vp, ctypes.POINTER(vp)],
        "mixer_free": [vp],
        "mixer_info": [vp, vp],
        "mixer_member": [vp, i32, vp, vp, vp],
        "mixer_set_variant": [vp, i32, i32],
        "mix_apply": [vp, vp, vp, i32, vp],
        "mix_apply_noalloc": [vp, vp, vp, i32, vp],
        "mix_adjoint": [vp, vp, vp, i32, vp],
        "mix_covariance": [vp, vp, vp, vp],
        "reference_response": [vp, _dp, vp],
        "age_information": [vp, _dp, i32, ctypes.c_double, vp, vp, _dp, vp],
        "age_window": [vp, i32, u32, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp],
        "age_reach": [_dp, _dp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                      ctypes.POINTER(ctypes.c_uint8), vp],
        "age_window_error": [vp, vp, vp, i32, _dp, i32, ctypes.c_double, ctypes.c_double, _dp, vp],
        "tsvd_project": [vp, vp, vp, i32, i32, ctypes.c_double, vp, vp],
        "noise_add": [vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, vp],
        "synthesis_create": [vp, i32, vp, ctypes.POINTER(vp)],
        "synthesis_free": [vp],
        "synthesis_info": [vp, vp, vp, vp],
        "synth_expand": [vp, vp, vp, i32, vp],
        "synth_project": [vp, vp, vp, i32, vp],
        "synthesis_audit": [vp, vp, u32, vp, vp, vp],
        "age_fisher": [vp, vp, _dp, i32, ctypes.c_double, u32, _dp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.variant_name.argtypes = [i32, i32]
    lib.variant_name.restype = ctypes.c_char_p
    lib.last_error.argtypes = []
    lib.last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != RTT_OK:
        msg = require_native().last_error().decode(errors="replace")
        if rc == RTT_ENOCONV:
            raise NoConvergence(rc, msg)
        raise RttError(rc, msg)


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, n_expected=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n_expected is not None and t.numel() != n_expected:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n_expected))
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------------- geometry
class Geometry:
    """Device ray tables of one geometry or of a block-diagonal batch of geometries.

    ``geoms``: one object or a list of objects with ``.grid`` (fields of
    rtt_grid) and ``.maps`` (per order: r, phi, delay, weight arrays, optional
    pixel_area).
    """

    def __init__(self, geoms, sigma_omega=0.0, drop_invalid=False):
        lib = require_native()
        if not isinstance(geoms, (list, tuple)):
            geoms = [geoms]
        grids = (rtt_grid * len(geoms))()
        maps_list = []
        keep = []
        for gi, geo in enumerate(geoms):
            g = geo.grid
            grids[gi] = rtt_grid(g.n_orders, g.n_frames, g.t0, g.dt_obs, g.n_r, g.n_phi, g.r_in,
                                 g.r_out, g.n_hat, g.s0, g.dt_src)
            if len(geo.maps) != g.n_orders:
                raise ValueError("need one ray map per order")
            for m in geo.maps:
                arrs = [np.ascontiguousarray(getattr(m, a), dtype=np.float64) for a in ("r", "phi", "delay", "weight")]
                area = getattr(m, "pixel_area", None)
                area = None if area is None else np.ascontiguousarray(area, dtype=np.float64)
                keep.extend(arrs + ([area] if area is not None else []))
                ptr = lambda a: a.ctypes.data_as(_dp)
                maps_list.append(rtt_raymap(arrs[0].shape[0], ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]),
                                            ptr(arrs[3]), ptr(area) if area is not None else None))
        maps = (rtt_raymap * len(maps_list))(*maps_list)
        opts = rtt_load_opts(float(sigma_omega), int(bool(drop_invalid)))
        h = ctypes.c_void_p()
        _check(lib.geometry_load(grids, maps, len(geoms), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        info = rtt_geometry_info()
        _check(lib.geometry_info(h, ctypes.byref(info)))
        self.n_geometries = info.n_geometries
        self.n_rows = info.n_rows
        self.n_cols = info.n_cols
        self.n_rays = info.n_rays
        self.table_bytes = info.table_bytes
        self._read_members()

    def _read_members(self):
        lib = require_native()
        self.members = []
        for gi in range(self.n_geometries):
            mi = rtt_member_info()
            _check(lib.geometry_member(self._h, gi, ctypes.byref(mi)))
            self.members.append(dict(row_offset=mi.row_offset, n_rows=mi.n_rows,
                                     col_offset=mi.col_offset, n_cols=mi.n_cols,
                                     n_frames=mi.grid.n_frames, n_orders=mi.grid.n_orders,
                                     rays_per_order=list(mi.rays_per_order)[: mi.grid.n_orders],
                                     apply_variant=mi.apply_variant, adjoint_variant=mi.adjoint_variant,
                                     digest=mi.digest))

    def set_variant(self, apply=-1, adjoint=-1, member=-1):
        """Pin kernel variants (indices as in variant_names())."""
        _check(require_native().geometry_set_variant(self.handle, member, apply, adjoint))
        self._read_members()

    def set_batch_mode(self, apply=-1, adjoint=-1):
        """Launch mode of whole-operator calls on several geometries (0, 1, 2; see include/rtt.h)."""
        _check(require_native().geometry_set_batch_mode(self.handle, apply, adjoint))

    @property
    def launches(self):
        """Kernel launches of one whole-operator (op_apply, op_apply_adjoint) call."""
        info = rtt_geometry_info()
        _check(require_native().geometry_info(self.handle, ctypes.byref(info)))
        return info.apply_launches, info.adjoint_launches

    @property
    def batch_mode(self):
        info = rtt_geometry_info()
        _check(require_native().geometry_info(self.handle, ctypes.byref(info)))
        return info.batch_apply_mode, info.batch_adjoint_mode

    def tune(self, nvec=1, reps=5, cache_path=None, stream=None):
        """Autotune the kernel variants of every member and the batch launch mode (see include/rtt.h)."""
        cp = None if cache_path is None else str(cache_path).encode()
        _check(require_native().geometry_tune(self.handle, nvec, reps, cp, _stream(stream)))
        self._read_members()
        return [(m["apply_variant"], m["adjoint_variant"]) for m in self.members]

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("geometry was freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.geometry_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def variant_names(adjoint: bool):
    lib = require_native()
    out = []
    while True:
        n = lib.variant_name(int(bool(adjoint)), len(out))
        if n is None:
            return out
        out.append(n.decode())


def geometry_load(geoms, sigma_omega=0.0, drop_invalid=False) -> Geometry:
    return Geometry(geoms, sigma_omega=sigma_omega, drop_invalid=drop_invalid)


def _nvec(t, n):
    if t.numel() % n:
        raise ValueError("tensor size is not a multiple of %d" % n)
    return t.numel() // n


def op_apply(geom: Geometry, x, y=None, order_mask: int = 0, stream=None):
    """y = A x.  x: [..., n_cols] float32 CUDA; returns y [..., n_rows].

    The library leaves the rows of orders outside ``order_mask`` unwritten; a y allocated here
    for a masked call therefore starts at zero, so those rows read as the masked operator's
    (zero) rows.
    """
    import torch
    nvec = _nvec(x, geom.n_cols)
    if y is None:
        alloc = torch.zeros if order_mask else torch.empty
        y = alloc(x.shape[:-1] + (geom.n_rows,), dtype=torch.float32, device=x.device)
    _check(require_native().op_apply(geom.handle, _dev_ptr(x, nvec * geom.n_cols, "x"),
                                     _dev_ptr(y, nvec * geom.n_rows, "y"), nvec, order_mask, _stream(stream)))
    return y


def op_apply_shared(geom: Geometry, x, y=None, order_mask: int = 0, stream=None):
    """y = A x with one coefficient block shared by every geometry of the handle (see
    include/rtt.h).  x: [..., n_cols / n_geometries]; returns y [..., n_rows]."""
    import torch
    ncg = geom.members[0]["n_cols"]
    nvec = _nvec(x, ncg)
    if y is None:
        alloc = torch.zeros if order_mask else torch.empty
        y = alloc(x.shape[:-1] + (geom.n_rows,), dtype=torch.float32, device=x.device)
    _check(require_native().op_apply_shared(geom.handle, _dev_ptr(x, nvec * ncg, "x"),
                                            _dev_ptr(y, nvec * geom.n_rows, "y"), nvec, order_mask,
                                            _stream(stream)))
    return y


def op_apply_adjoint(geom: Geometry, y, x=None, order_mask: int = 0, stream=None):
    """x = A^T y.  y: [..., n_rows] float32 CUDA; returns x [..., n_cols]."""
    import torch
    nvec = _nvec(y, geom.n_rows)
    if x is None:
        x = torch.empty(y.shape[:-1] + (geom.n_cols,), dtype=torch.float32, device=y.device)
    _check(require_native().op_apply_adjoint(geom.handle, _dev_ptr(y, nvec * geom.n_rows, "y"),
                                             _dev_ptr(x, nvec * geom.n_cols, "x"), nvec, order_mask,
                                             _stream(stream)))
    return x


from .svd import SVD, rsvd, tsvd_solve, tsvd_project, ridge_solve  # noqa: E402,F401
from .autograd import RetardedTimeOp, retarded_time_apply  # noqa: E402,F401
from .mixer import Mixer, mixer_create, mix_apply, mix_apply_noalloc, mix_adjoint, mix_covariance  # noqa: E402,F401
from .synthesis import Synthesis  # noqa: E402,F401
from .age import (reference_response, age_information, age_window, age_reach,  # noqa: E402,F401
                  age_window_error, noise_add)
