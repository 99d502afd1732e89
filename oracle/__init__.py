"""FP64 CPU oracle for the retarded-time imaging operator and its drivers.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.

* ``forward`` / ``adjoint``: A and A^T of Sec. 3.1 eq. (2)-(3) and App. A.2
  eq. (47), evaluated row by row in FP64 by the plain C code in
  ``rtt_oracle.c``.
* ``dense``: the dense matrix of A, column by column (tiny grids only).
* ``rsvd``: randomized subspace iteration (Halko, Martinsson & Tropp, SIAM
  Review 2011, Alg. 4.4) followed by the direct SVD of the projected matrix
  (their Alg. 5.1), FP64, LAPACK QR/SVD.
* ``block_lanczos``: block Golub-Kahan bidiagonalisation with full
  one-sided reorthogonalisation, FP64.
* ``tsvd_solve``, ``ridge_solve``, ``ridge_gradient``: the TSVD and ridge
  estimators of Sec. 9 and the ridge objective gradient.
* ``s_ref`` and ``operational_rank``: eq. (17)-(18) and eq. (31).
* ``mixer_matrix``, ``mix``, ``mix_adjoint``, ``mix_covariance``: the order mixer
  L of Sec. 3.1 eq. (4) (unresolved image and total flux) and the propagation of
  the data covariance through it, written out as dense matrices.
* ``probe_norm``, ``age_probes``, ``age_energy``, ``supported_ages``,
  ``throughput_age_boundary``, ``reach``: the age-localised probes of Sec. 3.3
  eq. (10)-(13), age information eq. (12)/(29) per observation arm, and the
  threshold statistics T_reach, L_anchor (eq. (30)) and J_old (eq. (35)).
* ``ridge_normal_solve``, ``ridge_data_gradient``, ``tsvd_project``: what the
  derivatives of the Sec. 9 estimators with respect to the data need (dense).
* ``age_window_error``: E(a) of eq. (32).
* ``philox4x32_10``, ``normal_draws``: the counter-based generator behind the
  seeded noise draws, written from its published definition.
* ``localized_probe_norms``, ``age_fisher``: the 28-direction localised probe
  class of eq. (14) and its age-local Fisher matrix M(a) = P^T P.
* ``synthesis_matrix``, ``synthesis_audit``: the representation synthesis Q_d of
  Sec. 3.2 eq. (7)-(8) (radial B-splines x azimuthal modes x DCT-II or compact
  temporal functions) on the coefficient nodes, and the rank audit of A Q_d.

Every function here is pinned by the "not gpu" tests against facts that do
not come from this module (see the tests' docstrings).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_rtt_oracle.so")
_lib = None


class _Grid(ctypes.Structure):
    _fields_ = [("n_orders", ctypes.c_int), ("n_frames", ctypes.c_int),
                ("t0", ctypes.c_double), ("dt_obs", ctypes.c_double),
                ("n_r", ctypes.c_int), ("n_phi", ctypes.c_int),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("n_hat", ctypes.c_int), ("s0", ctypes.c_double), ("dt_src", ctypes.c_double)]


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into oracle/_rtt_oracle.so."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        for name in ("ora_forward", "ora_adjoint"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.POINTER(_Grid), i64p, dp, dp, dp, dp, dp, dp, ctypes.c_uint]
        lib.ora_stencil.restype = ctypes.c_int
        lib.ora_stencil.argtypes = [ctypes.POINTER(_Grid), ctypes.c_double, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_int), dp]
        _lib = lib
    return _lib


def _cgrid(g) -> _Grid:
    return _Grid(g.n_orders, g.n_frames, g.t0, g.dt_obs, g.n_r, g.n_phi, g.r_in, g.r_out,
                 g.n_hat, g.s0, g.dt_src)


class _Packed:
    """Ray maps of a geometry concatenated over orders (caller ray order)."""

    def __init__(self, geom):
        self.grid = geom.grid
        self.counts = np.array(geom.rays_per_order, dtype=np.int64)
        cat = lambda attr: np.ascontiguousarray(
            np.concatenate([getattr(m, attr) for m in geom.maps]) if geom.maps else np.zeros(0))
        self.r, self.phi, self.delay, self.weight = (cat(a) for a in ("r", "phi", "delay", "weight"))
        self.n_rays = int(self.counts.sum())


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _mask(geom, order_mask):
    return (1 << geom.grid.n_orders) - 1 if order_mask is None else int(order_mask)


def host_threads() -> int:
    """Host threads the vector loops use by default: every core this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _each_vector(fn, n, threads):
    """Run fn(b) for b in range(n), on up to ``threads`` host threads.

    The vectors are independent and each one is evaluated by the same serial C loop whatever
    the thread count (ctypes releases the GIL during the call), so the results do not depend
    on ``threads``.
    """
    threads = host_threads() if threads is None else max(1, int(threads))
    if threads == 1 or n <= 1:
        for b in range(n):
            fn(b)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(threads, n)) as ex:
        for _ in ex.map(fn, range(n)):
            pass


def forward(geom, x, order_mask=None, out=None, threads=None):
    """y = A x (FP64).  x: [S*K] or [B][S*K]; y rows (n, p, f), frames fastest.

    Rows of orders outside ``order_mask`` are returned as zeros.  The B vectors are spread over
    ``threads`` host threads (default: host_threads()); each is one serial C evaluation.
    """
    lib = _load()
    pk = _Packed(geom)
    g = pk.grid
    x = np.ascontiguousarray(x, dtype=np.float64)
    single = x.ndim == 1
    xb = x.reshape(1, -1) if single else x
    if xb.shape[1] != g.n_cols:
        raise ValueError("x has wrong length")
    y = np.zeros((xb.shape[0], pk.n_rays * g.n_frames))
    cg = _cgrid(g)
    mask = _mask(geom, order_mask)
    counts = pk.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def one(b):
        xv = np.ascontiguousarray(xb[b])
        rc = lib.ora_forward(ctypes.byref(cg), counts, _ptr(pk.r), _ptr(pk.phi), _ptr(pk.delay),
                             _ptr(pk.weight), _ptr(xv), _ptr(y[b]), mask)
        if rc:
            raise ValueError("oracle forward rejected its inputs")

    _each_vector(one, xb.shape[0], threads)
    return y[0] if single else y


def adjoint(geom, y, order_mask=None, threads=None):
    """x = A^T y (FP64), same layouts as ``forward``; vectors spread over threads as there."""
    lib = _load()
    pk = _Packed(geom)
    g = pk.grid
    y = np.ascontiguousarray(y, dtype=np.float64)
    single = y.ndim == 1
    yb = y.reshape(1, -1) if single else y
    if yb.shape[1] != pk.n_rays * g.n_frames:
        raise ValueError("y has wrong length")
    x = np.zeros((yb.shape[0], g.n_cols))
    cg = _cgrid(g)
    mask = _mask(geom, order_mask)
    counts = pk.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def one(b):
        yv = np.ascontiguousarray(yb[b])
        rc = lib.ora_adjoint(ctypes.byref(cg), counts, _ptr(pk.r), _ptr(pk.phi), _ptr(pk.delay),
                             _ptr(pk.weight), _ptr(yv), _ptr(x[b]), mask)
        if rc:
            raise ValueError("oracle adjoint rejected its inputs")

    _each_vector(one, yb.shape[0], threads)
    return x[0] if single else x


def stencil(grid, r, phi):
    """(cells[4], weights[4]) of the bilinear spatial basis at (r, phi)."""
    lib = _load()
    cells = (ctypes.c_int * 4)()
    w = np.zeros(4)
    lib.ora_stencil(ctypes.byref(_cgrid(grid)), float(r), float(phi), cells, _ptr(w))
    return np.array(list(cells)), w


def dense(geom, order_mask=None):
    """Dense A (rows x cols) built column by column from ``forward``: tiny grids only."""
    n = geom.grid.n_cols
    if n * geom.n_rows > 5e7:
        raise ValueError("dense oracle is for tiny grids")
    eye = np.eye(n)
    return forward(geom, eye, order_mask).T.copy()


# ----------------------------------------------------------------------------------------------
# Linear algebra drivers (FP64)
# ----------------------------------------------------------------------------------------------

def _orth(Y):
    """Orthonormal basis of range(Y): LAPACK Householder QR."""
    q, _ = np.linalg.qr(Y, mode="reduced")
    return q


def rsvd(geom, omega, q=2, order_mask=None, want_u=False):
    """Randomized SVD of A (HMT 2011 Alg. 4.4 + Alg. 5.1), FP64.

    ``omega``: test block [l][S*K] (one row per test vector, the layout of a
    block of coefficient vectors).  Returns (sigma[l], V[l][S*K], U or None),
    where the rows of V (and of U) are right (left) singular vectors.
    """
    Om = np.asarray(omega, dtype=np.float64)
    Q = _orth(forward(geom, Om, order_mask).T)               # rows x l
    for _ in range(q):
        Qt = _orth(adjoint(geom, Q.T, order_mask).T)           # cols x l
        Q = _orth(forward(geom, Qt.T, order_mask).T)
    Bt = adjoint(geom, Q.T, order_mask).T                      # cols x l   (= (Q^T A)^T)
    Qb, Rb = np.linalg.qr(Bt, mode="reduced")                   # B = Rb^T Qb^T
    Ur, s, Wt = np.linalg.svd(Rb.T)                             # Rb^T = Ur diag(s) Wt
    V = Qb @ Wt.T                                               # cols x l
    U = Q @ Ur if want_u else None
    return s, V.T.copy(), (U.T.copy() if want_u else None)


def block_lanczos(geom, start, steps, order_mask=None):
    """Block Golub-Kahan bidiagonalisation, one-sided reorthogonalisation, FP64.

    ``start``: [b][S*K] start block.  With V_1 = orth(start) it runs, for
    j = 1..steps,
        A V_j - U_{j-1} R_{j-1}^T = U_j L_j          (QR, L_j upper triangular)
        A^T U_j - V_j L_j^T       = V_{j+1} R_j      (QR after reorthogonalising
                                                      against every stored V)
    so that A [V_1..V_s] = [U_1..U_s] T with T block upper bidiagonal (L_j on
    the diagonal, R_j^T above it).  Only the right (coefficient-space) basis is
    stored and reorthogonalised (two classical Gram-Schmidt passes); left
    blocks are kept one step back.  Returns (ritz_sigma, ritz_V[m][S*K],
    residual_estimates) with m = b * steps, where the residual of Ritz pair i
    is || R_s (last block of the left singular vector of T) ||, the norm of
    A^T u_i - sigma_i v_i implied by the recurrence.
    """
    X = np.asarray(start, dtype=np.float64).T                   # cols x b
    b = X.shape[1]
    V, _ = np.linalg.qr(X, mode="reduced")
    Vs = [V]
    m = b * steps
    T = np.zeros((m, m))
    U_prev, R_prev = None, None
    for j in range(steps):
        W = forward(geom, Vs[j].T, order_mask).T                  # rows x b
        if U_prev is not None:
            W = W - U_prev @ R_prev.T
        U, L = np.linalg.qr(W, mode="reduced")
        T[j * b:(j + 1) * b, j * b:(j + 1) * b] = L
        Z = adjoint(geom, U.T, order_mask).T - Vs[j] @ L.T        # cols x b
        for _ in range(2):
            for Vo in Vs:
                Z = Z - Vo @ (Vo.T @ Z)
        Vn, Rn = np.linalg.qr(Z, mode="reduced")
        if j + 1 < steps:
            T[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = Rn.T
            Vs.append(Vn)
        U_prev, R_prev = U, Rn
    Vall = np.concatenate(Vs, axis=1)                                # cols x m
    Pu, s, Pvt = np.linalg.svd(T)
    ritz_V = Vall @ Pvt.T
    res = np.linalg.norm(R_prev @ Pu[m - b:, :], axis=0)
    return s, ritz_V.T.copy(), res


def tsvd_solve(geom, V, sigma, y, t, order_mask=None):
    """TSVD estimate x = sum_{i<t} v_i (v_i . A^T y) / sigma_i^2 (rows of V are v_i)."""
    g = adjoint(geom, y, order_mask)
    single = g.ndim == 1
    G = g.reshape(1, -1) if single else g                         # [nrhs][S*K]
    Vt = np.asarray(V, dtype=np.float64)[:t]                      # [t][S*K]
    c = (G @ Vt.T) / (np.asarray(sigma, dtype=np.float64)[:t] ** 2)   # [nrhs][t]
    x = c @ Vt
    return x[0] if single else x


def ridge_gradient(geom, x, y, lam, order_mask=None):
    """Gradient of 1/2 ||A x - y||^2 + lam/2 ||x||^2: A^T (A x - y) + lam x."""
    return adjoint(geom, forward(geom, x, order_mask) - y, order_mask) + lam * np.asarray(x, dtype=np.float64)


def ridge_solve(geom, y, lam, tol=1e-12, maxit=10000, order_mask=None):
    """Ridge estimate: conjugate gradients on (A^T A + lam I) x = A^T y, FP64.

    Stops when ||r|| <= tol * ||A^T y||.  Returns (x, iterations).
    """
    rhs = adjoint(geom, y, order_mask)
    x = np.zeros_like(rhs)
    r = rhs.copy()
    p = r.copy()
    rr = float(r @ r)
    stop = tol * math.sqrt(float(rhs @ rhs))
    it = 0
    while math.sqrt(rr) > stop and it < maxit:
        Ap = adjoint(geom, forward(geom, p, order_mask), order_mask) + lam * p
        alpha = rr / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def s_ref(geom):
    """eq. (17): RMS direct-order response to the constant reference emissivity."""
    ones = np.ones(geom.grid.n_cols)
    y0 = forward(geom, ones, order_mask=1)
    m0 = geom.maps[0].n_rays * geom.grid.n_frames
    return math.sqrt(float(y0[:m0] @ y0[:m0]) / m0)


def operational_rank(sigma, s_reference, snr0=100.0, rho=1.0):
    """eq. (31) with C = sigma_Omega^2 I, sigma_Omega = s_ref/SNR0 (eq. (18))."""
    thr = rho * s_reference / snr0
    return int(np.count_nonzero(np.asarray(sigma) >= thr))


# ------------------------------------------------------------------ order mixer (Sec. 3.1, eq. (4))
MIX_KINDS = ("unresolved", "total_flux")


def mixer_matrix(geom, kind):
    """The order mixer L of eq. (4) for one geometry, written out as a dense 0/1 matrix.

    Columns are the order-resolved rays in data-row order (order 0's rays first, eq. (3)).
    'unresolved': one row per distinct image pixel (ascending pixel index) adding the rays of
    every order that land on that pixel -- the unresolved spatial image; 'total_flux': a single
    row adding every ray -- the total-flux readout.  Returns (L, pixels of the rows or None).
    """
    pix = np.concatenate([np.asarray(m.pixel, dtype=np.int64) for m in geom.maps])
    if kind == "total_flux":
        return np.ones((1, pix.size)), None
    if kind != "unresolved":
        raise ValueError("kind must be one of %s" % (MIX_KINDS,))
    rows = np.unique(pix)
    return (pix[None, :] == rows[:, None]).astype(np.float64), rows


def mix(geom, y, kind):
    """d_L = (L kron I) d_R of eq. (4): y holds order-resolved rows [..., n_rays * F]."""
    L, _ = mixer_matrix(geom, kind)
    F = geom.grid.n_frames
    y = np.asarray(y, dtype=np.float64)
    lead = y.shape[:-1]
    Y = y.reshape(lead + (geom.n_rays, F))
    return np.einsum("or,...rf->...of", L, Y).reshape(lead + (L.shape[0] * F,))


def mix_adjoint(geom, d, kind):
    """(L^T kron I) d: every ray row receives the mixed row it feeds."""
    L, _ = mixer_matrix(geom, kind)
    F = geom.grid.n_frames
    d = np.asarray(d, dtype=np.float64)
    lead = d.shape[:-1]
    D = d.reshape(lead + (L.shape[0], F))
    return np.einsum("or,...of->...rf", L, D).reshape(lead + (geom.n_rays * F,))


def mix_covariance(geom, var, kind):
    """C_L = (L kron I) C_R (L^T kron I) of eq. (4) for a diagonal C_R = diag(var), var being the
    per-datum variances in data-row order.  Returns the full matrix (small cases only)."""
    L, _ = mixer_matrix(geom, kind)
    K = np.kron(L, np.eye(geom.grid.n_frames))
    return K @ np.diag(np.asarray(var, dtype=np.float64)) @ K.T


# ------------------------------------------------------------------ age probes and reach (Sec. 3.3, Sec. 4.4, Sec. 6.5)
def probe_norm(grid, h=3.0):
    """N_h of eq. (11): the L2 norm of the unnormalised probe over the emission annulus
    (area measure r dr dphi) and over all source times."""
    return math.sqrt(math.pi * (grid.r_out ** 2 - grid.r_in ** 2) * h * math.sqrt(math.pi))


def age_probes(grid, ages, h=3.0):
    """The age-localised probes q_a of eq. (10) on the coefficient nodes: every cell node lies in the
    annulus (indicator 1, no azimuthal modulation) and hat k takes the probe's value at its centre
    s_k.  Returns [len(ages), n_cols] (hat index fastest)."""
    ages = np.asarray(ages, dtype=np.float64)
    s_k = grid.s0 + grid.dt_src * np.arange(grid.n_hat)
    X = np.empty((ages.size, grid.n_cells, grid.n_hat))
    for i, a in enumerate(ages):
        X[i, :, :] = np.exp(-((s_k + a) ** 2) / (2.0 * h * h)) / probe_norm(grid, h)
    return X.reshape(ages.size, grid.n_cols)


def age_energy(geom, ages, h=3.0, arm="resolved", var=None):
    """||C^{-1/2} A q_a||^2 of eq. (12)/(29) for every age, at sigma_Omega = 1.

    arm: "direct" (order-0 rows, C = I), "resolved" (every order, C = I), or a mixer kind of eq. (4)
    ("unresolved", "total_flux") whose covariance C_L = (L kron I) diag(var) (L^T kron I) is formed in
    full and solved against (var: per-datum variances of the resolved rows, default 1)."""
    X = age_probes(geom.grid, ages, h)
    if arm in ("direct", "resolved"):
        mask = 1 if arm == "direct" else None
        Y = forward(geom, X, order_mask=mask)
        return np.einsum("ar,ar->a", Y, Y)
    Y = forward(geom, X)
    v = np.ones(Y.shape[1]) if var is None else np.asarray(var, dtype=np.float64)
    D = mix(geom, Y, arm)
    C = mix_covariance(geom, v, arm)
    return np.array([float(d @ np.linalg.solve(C, d)) for d in D])


def supported_ages(geom, ages, h=3.0, order_mask=None):
    """Centres whose operational support |t + a| <= 3h lies inside the source-time window that the
    selected orders reach (eq. (13)), found by brute force over every datum's retarded time
    t_f - Delta of the rays with chi = 1 (non-zero weight, radius inside the annulus)."""
    g = geom.grid
    t_f = g.t0 + g.dt_obs * np.arange(g.n_frames)
    lo, hi = math.inf, -math.inf
    for n, m in enumerate(geom.maps):
        if order_mask is not None and not (int(order_mask) >> n) & 1:
            continue
        for p in range(m.n_rays):
            if m.weight[p] == 0.0 or not (g.r_in <= m.r[p] <= g.r_out):
                continue
            t = t_f - m.delay[p]
            lo, hi = min(lo, float(t.min())), max(hi, float(t.max()))
    ages = np.asarray(ages, dtype=np.float64)
    return np.array([lo <= -a - 3.0 * h and -a + 3.0 * h <= hi for a in ages], dtype=bool)


def throughput_age_boundary(geom, q=0.999):
    """A_{0,q} of eq. (35): the age below which the fraction q of the direct order's throughput lies,
    every direct datum (ray p, frame f) carrying the age Delta_p - t_f and the weight |w_p|."""
    g = geom.grid
    m = geom.maps[0]
    t_f = g.t0 + g.dt_obs * np.arange(g.n_frames)
    age = (m.delay[:, None] - t_f[None, :]).ravel()
    w = np.repeat(np.abs(m.weight), g.n_frames)
    order = np.argsort(age, kind="stable")
    cum = np.cumsum(w[order])
    return float(age[order][np.searchsorted(cum, q * cum[-1])])


def reach(ages, info, rho=1.0, supported=None, boundary=None):
    """Threshold statistics of Sec. 4.4 on an age grid, from the physical information info(a)
    (SNR0^2 times the normalised information).

    mask: info >= rho^2 (eq. (30)); t_reach: the oldest passing centre (None if none passes);
    anchor: the youngest supported centre; l_anchor: extent of the passing run that starts at the
    anchor (None if the anchor fails); longest: extent of the longest passing run; j_old: eq. (35),
    the sum of log(1 + info) over centres older than `boundary`, times the grid step."""
    ages = [float(a) for a in ages]
    info = [float(v) for v in info]
    n = len(ages)
    mask = [v >= rho * rho for v in info]
    passing = [ages[i] for i in range(n) if mask[i]]
    t_reach = max(passing) if passing else None
    anchor = None
    for i in range(n):
        if supported is None or supported[i]:
            anchor = i
            break
    l_anchor = None
    if anchor is not None and mask[anchor]:
        j = anchor
        while j + 1 < n and mask[j + 1]:
            j += 1
        l_anchor = ages[j] - ages[anchor]
    longest = None
    i = 0
    while i < n:
        if mask[i]:
            j = i
            while j + 1 < n and mask[j + 1]:
                j += 1
            ext = ages[j] - ages[i]
            longest = ext if longest is None or ext > longest else longest
            i = j + 1
        else:
            i += 1
    step = ages[1] - ages[0] if n > 1 else 0.0
    j_old = None
    if boundary is not None:
        j_old = 0.0
        for i in range(n):
            if ages[i] > boundary:
                j_old += math.log(1.0 + info[i]) * step
    return dict(mask=mask, t_reach=t_reach, anchor=anchor, l_anchor=l_anchor, longest=longest, j_old=j_old)


# ------------------------------------------------------------------ differentiating through the estimators (Sec. 9)
def ridge_normal_solve(geom, b, lam, order_mask=None):
    """Solves (A^T A + lambda I) x = b for a coefficient-space right-hand side b, with the dense
    matrix of A (tiny grids only)."""
    A = dense(geom, order_mask)
    M = A.T @ A + lam * np.eye(A.shape[1])
    return np.linalg.solve(M, np.asarray(b, dtype=np.float64).T).T


def ridge_data_gradient(geom, g_x, lam, order_mask=None):
    """Gradient with respect to the data y of <g_x, x_hat(y)> for the ridge estimate
    x_hat(y) = (A^T A + lambda I)^{-1} A^T y: A (A^T A + lambda I)^{-1} g_x (the normal matrix is
    symmetric).  Dense, tiny grids only."""
    A = dense(geom, order_mask)
    return (A @ ridge_normal_solve(geom, g_x, lam, order_mask).T).T


def tsvd_project(V, sigma, b, t):
    """V_t diag(sigma_t^-2) V_t^T b with the t leading right singular vectors (rows of V)."""
    Vt = np.asarray(V, dtype=np.float64)[:t]
    s = np.asarray(sigma, dtype=np.float64)[:t]
    b = np.asarray(b, dtype=np.float64)
    c = Vt @ np.atleast_2d(b).T                  # [t][B]
    out = (c / (s * s)[:, None]).T @ Vt          # [B][n]
    return out[0] if b.ndim == 1 else out


def age_window_error(grid, x_hat, x, ages, half_width=2.0, eta=1e-12):
    """E(a) of eq. (32) with W_a keeping the coefficients of every cell at the hats whose centre s_k
    lies in the age window |s_k + a| <= half_width (source time -a): ||W_a (x_hat - x)|| /
    max(||W_a x||, eta).  x_hat, x: [n_cols] or [B][n_cols]; returns [len(ages)] or [B][len(ages)]."""
    xh = np.atleast_2d(np.asarray(x_hat, dtype=np.float64))
    xt = np.atleast_2d(np.asarray(x, dtype=np.float64))
    s_k = grid.s0 + grid.dt_src * np.arange(grid.n_hat)
    out = np.zeros((xh.shape[0], len(ages)))
    for b in range(xh.shape[0]):
        D = (xh[b] - xt[b]).reshape(grid.n_cells, grid.n_hat)
        X = xt[b].reshape(grid.n_cells, grid.n_hat)
        for i, a in enumerate(ages):
            num, den = 0.0, 0.0
            for k in range(grid.n_hat):
                if abs(s_k[k] + a) <= half_width:
                    num += float(np.sum(D[:, k] ** 2))
                    den += float(np.sum(X[:, k] ** 2))
            out[b, i] = math.sqrt(num) / max(math.sqrt(den), eta)
    return out[0] if np.asarray(x_hat).ndim == 1 else out


# ------------------------------------------------------------------ seeded noise draws
_PHILOX_M0, _PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
_PHILOX_W0, _PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(counter, key):
    """Philox-4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11): the S-box round
    multiplies words 0 and 2 by the two round constants, takes the high halves XORed with the
    other words and the key, and the key is bumped by the Weyl constants after every round."""
    c = [int(v) & 0xFFFFFFFF for v in counter]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _PHILOX_M0 * c[0]
        p1 = _PHILOX_M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
        k0 = (k0 + _PHILOX_W0) & 0xFFFFFFFF
        k1 = (k1 + _PHILOX_W1) & 0xFFFFFFFF
    return c


def normal_draws(n, seed):
    """N(0, 1) draws: group i of four uses the Philox-4x32-10 block of counter (i mod 2^32, i >> 32,
    0, 0) and key (seed mod 2^32, seed >> 32); the words map to uniforms (w + 1/2) 2^-32 and pairs
    (u0, u1), (u2, u3) to Box-Muller normals r cos(2 pi u'), r sin(2 pi u'), r = sqrt(-2 ln u).
    FP64 here."""
    out = np.empty(n)
    for i in range((n + 3) // 4):
        w = philox4x32_10([i & 0xFFFFFFFF, i >> 32, 0, 0], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
        u = [(v + 0.5) * 2.0 ** -32 for v in w]
        r0, r1 = math.sqrt(-2.0 * math.log(u[0])), math.sqrt(-2.0 * math.log(u[2]))
        v = [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
             r1 * math.cos(2 * math.pi * u[3]), r1 * math.sin(2 * math.pi * u[3])]
        for t in range(4):
            if 4 * i + t < n:
                out[4 * i + t] = v[t]
    return out


# ------------------------------------------------------------------ representation synthesis (Sec. 3.2, eq. (5)-(8); Sec. 7)
def _radial_bsplines(r, r_in, r_out, n_radial):
    """Clamped cubic B-splines on uniform knots in log r over [r_in, r_out] (scipy's BSpline
    evaluates them): [len(r)][n_radial]."""
    from scipy.interpolate import BSpline
    u = (np.log(r) - math.log(r_in)) / (math.log(r_out) - math.log(r_in))
    inner = [j / (n_radial - 3) for j in range(1, n_radial - 3)]
    t = np.r_[[0.0] * 4, inner, [1.0] * 4]
    out = np.zeros((len(u), n_radial))
    for a in range(n_radial):
        c = np.zeros(n_radial)
        c[a] = 1.0
        out[:, a] = BSpline(t, c, 3, extrapolate=False)(np.clip(u, 0.0, 1.0))
    return np.nan_to_num(out)


def synthesis_matrix(grid, n_radial=4, m_max=3, n_temporal=8, temporal="dct", window=None):
    """Q_d of eq. (7)-(8) evaluated on the coefficient nodes: column (a, b, c) (radial slowest,
    temporal fastest) holds R_a(r_i) Phi_b(phi_j) T_c(s_k) at node (i, j, k).  R_a: clamped cubic
    B-splines on uniform knots in log r; Phi_b: 1, cos m phi, sin m phi (m <= m_max); T_c over the
    source-time window [t_lo, t_hi] (default [s0 - dt/2, s0 + (K - 1/2) dt], where the DCT-II modes
    on the nodes are exactly the discrete DCT-II vectors): "dct" = cos(pi c (t - t_lo)/(t_hi - t_lo)),
    "hats" = degree-one B-splines on n_temporal uniform knots from t_lo to t_hi.  [n_cols][d]."""
    rc = grid.r_in + (np.arange(grid.n_r) + 0.5) * (grid.r_out - grid.r_in) / grid.n_r
    pc = (np.arange(grid.n_phi) + 0.5) * 2.0 * math.pi / grid.n_phi
    sk = grid.s0 + grid.dt_src * np.arange(grid.n_hat)
    t_lo, t_hi = window if window is not None else (grid.s0 - 0.5 * grid.dt_src,
                                                   grid.s0 + (grid.n_hat - 0.5) * grid.dt_src)
    R = _radial_bsplines(rc, grid.r_in, grid.r_out, n_radial)                  # [n_r][n_radial]
    az = [np.ones_like(pc)]
    for m in range(1, m_max + 1):
        az += [np.cos(m * pc), np.sin(m * pc)]
    P = np.stack(az, axis=1)                                                   # [n_phi][2 m_max + 1]
    if temporal == "dct":
        T = np.stack([np.cos(math.pi * c * (sk - t_lo) / (t_hi - t_lo)) for c in range(n_temporal)], axis=1)
    elif temporal == "hats":
        knots = np.linspace(t_lo, t_hi, n_temporal)
        w = (t_hi - t_lo) / (n_temporal - 1)
        T = np.stack([np.maximum(0.0, 1.0 - np.abs(sk - knots[c]) / w) for c in range(n_temporal)], axis=1)
    else:
        raise ValueError("temporal must be 'dct' or 'hats'")
    Q = np.einsum("ia,jb,kc->ijkabc", R, P, T)
    return Q.reshape(grid.n_cols, R.shape[1] * P.shape[1] * T.shape[1])


def synthesis_audit(geom, Q, order_mask=None, rel_tol=1e-7):
    """Rank audit of A^(d) = A Q_d (eq. (7)) restricted to the selected orders' rows: the indices of
    exactly zero columns, the singular values (LAPACK SVD of the dense FP64 product) and the
    numerical rank at rel_tol * sigma_max."""
    A = dense(geom, order_mask)
    AQ = A @ Q
    zero = [int(c) for c in range(AQ.shape[1]) if not np.any(AQ[:, c])]
    s = np.linalg.svd(AQ, compute_uv=False)
    rank = int(np.sum(s > rel_tol * s[0])) if s.size and s[0] > 0 else 0
    return dict(zero_columns=zero, sigma=s, rank=rank)


def localized_probe_norms(grid, n_radial=4, m_max=3, h=3.0):
    """N_{h,l} of eq. (14) for the spatial functions psi_l = R_a Phi_b (l = a (2 m_max + 1) + b): the
    L2 norm of psi_l(r, phi) exp(-(t + a)^2 / (2 h^2)) over the annulus (area measure) and time,
    with the radial integral of the continuum B-spline by adaptive quadrature."""
    from scipy.integrate import quad
    out = []
    for a in range(n_radial):
        rad = quad(lambda r: _radial_bsplines(np.array([r]), grid.r_in, grid.r_out, n_radial)[0, a] ** 2 * r,
                   grid.r_in, grid.r_out, limit=200, epsabs=0.0, epsrel=1e-12)[0]
        for b in range(2 * m_max + 1):
            az = 2.0 * math.pi if b == 0 else math.pi
            out.append(math.sqrt(rad * az * h * math.sqrt(math.pi)))
    return np.array(out)


def age_fisher(geom, ages, h=3.0, n_radial=4, m_max=3, order_mask=None):
    """M(a) = P(a)^T P(a) of eq. (14) for the localised probes q_{a,l} = psi_l g_a / N_{h,l} set on the
    coefficient nodes (psi_l = R_a Phi_b from the synthesis factors, g_a the Gaussian of eq. (10)),
    P(a) = A q_{a,l} column by column (C = I).  Returns [len(ages)][L][L], L = n_radial (2 m_max + 1)."""
    g = geom.grid
    Q = synthesis_matrix(g, n_radial=n_radial, m_max=m_max, n_temporal=1, temporal="dct")   # T_0 = 1
    norms = localized_probe_norms(g, n_radial, m_max, h)
    sk = g.s0 + g.dt_src * np.arange(g.n_hat)
    S = Q.reshape(g.n_cells, g.n_hat, -1)[:, 0, :]                 # psi_l at the cell nodes: [cells][L]
    out = []
    for a in ages:
        gt = np.exp(-((sk + a) ** 2) / (2.0 * h * h))
        X = np.einsum("sl,k->lsk", S, gt).reshape(S.shape[1], g.n_cols) / norms[:, None]
        P = forward(geom, X, order_mask=order_mask)                  # [L][rows]
        out.append(P @ P.T)
    return np.array(out)
