"""Bindings of the spectral drivers and estimators (rsvd, tsvd_solve, ridge_solve)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import (RTT_EACH_GEOMETRY, RTT_SOLVE_ASYNC, RTT_SOLVE_NORMAL_RHS, RTT_SVD_BLOCK_LANCZOS, RTT_SVD_RSVD, _check, _dev_ptr, _nvec,
               _stream, require_native, rtt_cg_opts, rtt_solve_info, rtt_svd_opts)


class SVD:
    """Singular factors held in device memory by the library (rtt_svd)."""

    def __init__(self, handle, geom, sets=1):
        self._h = handle
        self.geom = geom
        lib = require_native()
        k = ctypes.c_int32()
        _check(lib.svd_get(handle, ctypes.byref(k), None, None, None, None))
        self.k = k.value
        self.sets = sets
        sig = np.zeros(self.k * sets)
        res = np.zeros(self.k * sets)
        _check(lib.svd_get(handle, None, sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None,
                           res.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        # [k] for one operator, [G][k] for factors of every geometry
        self.sigma = sig if sets == 1 else sig.reshape(sets, self.k)
        self.residual = res if sets == 1 else res.reshape(sets, self.k)

    def converged(self, rel_tol=1e-6):
        """Number of singular values whose residual is <= rel_tol * sigma_1 (an int, or one per
        geometry for factors of every geometry); see svd_converged in include/rtt.h."""
        cnt = (ctypes.c_int32 * self.sets)()
        _check(require_native().svd_converged(self._h, float(rel_tol), cnt))
        return cnt[0] if self.sets == 1 else np.array(list(cnt))

    def _ptr(self, which):
        lib = require_native()
        vp = ctypes.c_void_p()
        if which == "V":
            _check(lib.svd_get(self._h, None, None, ctypes.byref(vp), None, None))
        else:
            _check(lib.svd_get(self._h, None, None, None, ctypes.byref(vp), None))
        return vp.value

    @property
    def geom_cols(self):
        return self.geom.n_cols if self._member is None else self.geom.members[self._member]["n_cols"]

    @property
    def geom_rows(self):
        return self.geom.n_rows if self._member is None else self.geom.members[self._member]["n_rows"]

    def block(self, V, g):
        """Geometry g's part of a [k][n_cols] factor of RTT_EACH_GEOMETRY factors."""
        m = self.geom.members[g]
        return V[:, m["col_offset"]:m["col_offset"] + m["n_cols"]]

    _member = None

    def _copy(self, which, n):
        import torch
        addr = self._ptr(which)
        if not addr:
            return None
        out = torch.empty((self.k, n), dtype=torch.float32, device="cuda")
        _d2d(out.data_ptr(), addr, self.k * n * 4)
        return out

    def V(self):
        """Right singular vectors, a new torch tensor [k][n_cols] (device copy)."""
        return self._copy("V", self.geom_cols)

    def U(self):
        """Left singular vectors [k][n_rows] if they were kept, else None."""
        return self._copy("U", self.geom_rows)

    def free(self):
        if getattr(self, "_h", None) is not None:
            require_native().svd_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_hip = None


def _d2d(dst, src, nbytes):
    """Device-to-device copy on the current stream (plumbing for library-owned factors)."""
    import torch
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    rc = _hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError("hipMemcpyAsync failed (%d)" % rc)


def rsvd(geom, k=256, p=8, q=2, omega=None, method="rsvd", block=32, steps=16, order_mask=0,
         geometry=-1, seed=0, keep_u=False, stream=None) -> SVD:
    """Leading singular triplets of A (rSVD or block Lanczos, see include/rtt.h)."""
    lib = require_native()
    opts = rtt_svd_opts()
    opts.method = RTT_SVD_RSVD if method == "rsvd" else RTT_SVD_BLOCK_LANCZOS
    opts.k, opts.p, opts.q = int(k), int(p), int(q)
    opts.block, opts.steps = int(block), int(steps)
    opts.order_mask = int(order_mask)
    opts.geometry = int(geometry)
    opts.seed = int(seed)
    opts.keep_u = int(bool(keep_u))
    n_cols = geom.n_cols if geometry < 0 else geom.members[geometry]["n_cols"]
    om = None
    if omega is not None:
        nv = _nvec(omega, n_cols)
        om = _dev_ptr(omega, nv * n_cols, "omega")
    h = ctypes.c_void_p()
    _check(lib.rsvd(geom.handle, ctypes.byref(opts), om, ctypes.byref(h), _stream(stream)))
    s = SVD(h, geom, sets=geom.n_geometries if geometry == RTT_EACH_GEOMETRY else 1)
    s._member = None if geometry < 0 else int(geometry)
    return s


def tsvd_solve(geom, svd: SVD, y, t=0, sigma_min=0.0, x=None, stream=None):
    """TSVD estimate x = V_t diag(sigma_t^-2) V_t^T A^T y."""
    import torch
    n_rows = svd.geom_rows
    n_cols = svd.geom_cols
    nrhs = _nvec(y, n_rows)
    if x is None:
        x = torch.empty(y.shape[:-1] + (n_cols,), dtype=torch.float32, device=y.device)
    _check(require_native().tsvd_solve(geom.handle, svd._h, _dev_ptr(y, nrhs * n_rows, "y"), nrhs, int(t),
                                       float(sigma_min), _dev_ptr(x, nrhs * n_cols, "x"), _stream(stream)))
    return x


def tsvd_project(geom, svd: SVD, b, t=0, sigma_min=0.0, x=None, stream=None):
    """x = V_t diag(sigma_t^-2) V_t^T b for a coefficient block b (the map tsvd_solve applies after A^T)."""
    import torch
    n_cols = svd.geom_cols
    nrhs = _nvec(b, n_cols)
    if x is None:
        x = torch.empty(b.shape[:-1] + (n_cols,), dtype=torch.float32, device=b.device)
    _check(require_native().tsvd_project(geom.handle, svd._h, _dev_ptr(b, nrhs * n_cols, "b"), nrhs, int(t),
                                         float(sigma_min), _dev_ptr(x, nrhs * n_cols, "x"), _stream(stream)))
    return x


def ridge_solve(geom, y, lam, tol=1e-6, maxit=1000, order_mask=0, x=None, stream=None, raise_on_noconv=True,
                async_mode=False, resid=None, normal_rhs=False):
    """Ridge estimate by CG on (A^T A + lam I) x = A^T y, one CG per (right-hand side, geometry);
    returns (x, info dict).

    async_mode: stream-ordered solve of exactly ``maxit`` iterations with no host
    synchronisation (capturable into a graph once its scratch exists); ``resid``
    (float32 CUDA [nrhs * n_geometries]) then receives the final relative residuals.
    normal_rhs: ``y`` is a coefficient block b and the solve is (A^T A + lam I) x = b.
    """
    import torch
    n_in = geom.n_cols if normal_rhs else geom.n_rows
    nrhs = _nvec(y, n_in)
    if x is None:
        x = torch.empty(y.shape[:-1] + (geom.n_cols,), dtype=torch.float32, device=y.device)
    rp = None if resid is None else _dev_ptr(resid, nrhs * geom.n_geometries, "resid").value
    flags = (RTT_SOLVE_ASYNC if async_mode else 0) | (RTT_SOLVE_NORMAL_RHS if normal_rhs else 0)
    opts = rtt_cg_opts(float(tol), int(maxit), int(order_mask), flags, rp)
    info = rtt_solve_info()
    rc = require_native().ridge_solve(geom.handle, _dev_ptr(y, nrhs * n_in, "y"), nrhs, float(lam),
                                      ctypes.byref(opts), _dev_ptr(x, nrhs * geom.n_cols, "x"),
                                      ctypes.byref(info), _stream(stream))
    out = dict(iterations=info.iterations, converged=info.converged, rel_residual=info.rel_residual)
    if rc != 0 and (raise_on_noconv or rc != -4):
        _check(rc)
    return x, out
