"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* spatial factor: scipy's RegularGridInterpolator (bilinear on the cell-centre
  grid, periodic in phi, constant continuation in r) evaluated at each ray's
  source point (eq. (47), psi_l(r, phi));
* temporal factor: numpy.interp on the hat nodes padded by one zero node on
  each side -- piecewise-linear interpolation is exactly the span of the
  degree-one B-splines of Sec. 7 (eq. (47), tau_k(t_o - Delta));
* Thm 4.1 / Cor 4.2: the blind hats are computed from the footprint eq. (23)
  alone, and the oracle must return exact (bitwise) zeros on them;
* adjoint identity, Gram monotonicity eq. (21), split/merge Gram invariance
  of the whitened rows eq. (16) (paper's criterion 1e-10);
* LAPACK: rSVD and block Lanczos reduce to the SVD when the sketch spans the
  range, TSVD to the truncated pseudo-inverse, ridge CG to a dense solve;
* the ridge gradient against central finite differences of the objective.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth
from tinygeo import tiny_geometry

GEOMS = {
    "ratio1": dict(seed=11, rays=(12, 6, 5)),
    "ratio_half": dict(seed=12, rays=(10, 5, 4), dt_obs=2.0, n_frames=9),
    "ratio2": dict(seed=13, rays=(9, 4, 3), dt_obs=8.0, n_frames=4),
    "direct_only": dict(seed=14, rays=(15,)),
}


def packed(geo):
    r = np.concatenate([m.r for m in geo.maps])
    phi = np.concatenate([m.phi for m in geo.maps])
    delay = np.concatenate([m.delay for m in geo.maps])
    w = np.concatenate([m.weight for m in geo.maps])
    return r, phi, delay, w


def spatial_interp(grid, field, r, phi):
    """Bilinear interpolation of a cell-centred field via scipy (periodic phi, clamped r)."""
    dr = (grid.r_out - grid.r_in) / grid.n_r
    dphi = 2 * math.pi / grid.n_phi
    rc = grid.r_in + (np.arange(grid.n_r) + 0.5) * dr
    pc = (np.arange(grid.n_phi) + 0.5) * dphi
    f2 = field.reshape(grid.n_r, grid.n_phi)
    pcp = np.concatenate([[pc[-1] - 2 * math.pi], pc, [pc[0] + 2 * math.pi]])
    f2p = np.concatenate([f2[:, -1:], f2, f2[:, :1]], axis=1)
    rgi = RegularGridInterpolator((rc, pcp), f2p, method="linear")
    q = np.stack([np.clip(r, rc[0], rc[-1]), np.mod(phi, 2 * math.pi)], axis=1)
    return rgi(q)


def temporal_interp(grid, h, t):
    nodes = grid.s0 + grid.dt_src * np.arange(-1, grid.n_hat + 1)
    vals = np.concatenate([[0.0], h, [0.0]])
    return np.interp(t, nodes, vals, left=0.0, right=0.0)


def frame_times(grid):
    return grid.t0 + grid.dt_obs * np.arange(grid.n_frames)


@pytest.mark.parametrize("name", list(GEOMS))
def test_separable_field_matches_library_interpolation(name):
    geo = tiny_geometry(**GEOMS[name])
    g = geo.grid
    rng = np.random.default_rng(5)
    gs = rng.standard_normal(g.n_cells)
    hk = rng.standard_normal(g.n_hat)
    x = np.outer(gs, hk).ravel()
    y = oracle.forward(geo, x).reshape(geo.n_rays, g.n_frames)
    r, phi, delay, w = packed(geo)
    G = spatial_interp(g, gs, r, phi)
    H = temporal_interp(g, hk, frame_times(g)[None, :] - delay[:, None])
    expect = w[:, None] * G[:, None] * H
    assert np.max(np.abs(y - expect)) <= 1e-13 * np.max(np.abs(expect))


@pytest.mark.parametrize("name", list(GEOMS))
def test_spatial_and_temporal_factors_separately(name):
    geo = tiny_geometry(**GEOMS[name])
    g = geo.grid
    r, phi, delay, w = packed(geo)
    rng = np.random.default_rng(6)
    # spatial only: x constant in time -> hats sum to one inside [s_0, s_{K-1}]
    gs = rng.standard_normal(g.n_cells)
    y = oracle.forward(geo, np.repeat(gs, g.n_hat)).reshape(geo.n_rays, g.n_frames)
    tret = frame_times(g)[None, :] - delay[:, None]
    inside = (tret >= g.s0) & (tret <= g.s0 + (g.n_hat - 1) * g.dt_src)
    expect = (w * spatial_interp(g, gs, r, phi))[:, None] * np.ones_like(tret)
    assert inside.all()
    assert np.max(np.abs(y - expect)) <= 1e-13 * np.max(np.abs(expect))
    # temporal only: x constant over cells -> bilinear weights sum to one
    hk = rng.standard_normal(g.n_hat)
    y = oracle.forward(geo, np.tile(hk, g.n_cells)).reshape(geo.n_rays, g.n_frames)
    expect = w[:, None] * temporal_interp(g, hk, tret)
    assert np.max(np.abs(y - expect)) <= 1e-13 * np.max(np.abs(expect))


def test_partition_of_unity_and_sref_closed_form():
    geo = tiny_geometry(**GEOMS["ratio1"])
    g = geo.grid
    y = oracle.forward(geo, np.ones(g.n_cols)).reshape(geo.n_rays, g.n_frames)
    w = packed(geo)[3]
    assert np.max(np.abs(y - w[:, None])) <= 1e-15
    # eq. (17): with every direct row inside the hat window, s_ref^2 = mean(w_0^2)
    w0 = geo.maps[0].weight
    assert oracle.s_ref(geo) == pytest.approx(math.sqrt(np.mean(w0 ** 2)), rel=1e-14)


def test_window_edges_ramp_like_unclamped_hats():
    """Retarded times beyond the last node ramp down over one hat width."""
    geo = tiny_geometry(seed=21, rays=(20,), delay_hi=10.0, extra_hats=-3)
    g = geo.grid
    y = oracle.forward(geo, np.ones(g.n_cols)).reshape(geo.n_rays, g.n_frames)
    r, phi, delay, w = packed(geo)
    tret = frame_times(g)[None, :] - delay[:, None]
    top = g.s0 + (g.n_hat - 1) * g.dt_src
    ramp = np.clip(1.0 - (tret - top) / g.dt_src, 0.0, 1.0)
    expect = w[:, None] * np.where(tret > top, ramp, 1.0)
    assert (tret > top).any()
    assert np.max(np.abs(y - expect)) <= 1e-14


@pytest.mark.parametrize("name", list(GEOMS))
def test_adjoint_identity(name):
    geo = tiny_geometry(**GEOMS[name])
    rng = np.random.default_rng(7)
    x = rng.standard_normal(geo.grid.n_cols)
    y = rng.standard_normal(geo.n_rows)
    lhs = float(oracle.forward(geo, x) @ y)
    rhs = float(x @ oracle.adjoint(geo, y))
    assert abs(lhs - rhs) <= 1e-13 * (np.linalg.norm(oracle.forward(geo, x)) * np.linalg.norm(y))


def direct_blind_hats(geo):
    """Hats whose open support misses the discrete direct footprint eq. (23)."""
    g = geo.grid
    W0 = (frame_times(g)[None, :] - geo.maps[0].delay[:, None]).ravel()
    sk = g.s0 + g.dt_src * np.arange(g.n_hat)
    return np.array([k for k in range(g.n_hat) if not np.any(np.abs(W0 - sk[k]) < g.dt_src)])


def test_direct_old_epoch_blindness_theorem():
    geo = tiny_geometry(**GEOMS["ratio1"])
    g = geo.grid
    Z0 = direct_blind_hats(geo)
    assert len(Z0) >= 3                      # the old-anchored window has direct-blind hats
    rng = np.random.default_rng(8)
    x = np.zeros((g.n_cells, g.n_hat))
    x[:, Z0] = rng.standard_normal((g.n_cells, len(Z0)))
    y = oracle.forward(geo, x.ravel()).reshape(geo.n_rays, g.n_frames)
    P0 = geo.maps[0].n_rays
    assert np.all(y[:P0] == 0.0)                              # eq. (24): bitwise zero block
    # converse: hats reached by an added order make the stacked column nonzero
    Wr = (frame_times(g)[None, :] - np.concatenate([m.delay for m in geo.maps[1:]])[:, None]).ravel()
    sk = g.s0 + g.dt_src * np.arange(g.n_hat)
    lifted = [k for k in Z0 if np.any(np.abs(Wr - sk[k]) < g.dt_src)]
    assert lifted and np.any(y[P0:] != 0.0)
    # transpose: A_0^T y vanishes on the blind block
    xb = oracle.adjoint(geo, rng.standard_normal(geo.n_rows), order_mask=1).reshape(g.n_cells, g.n_hat)
    assert np.all(xb[:, Z0] == 0.0)
    # Cor. 4.2: nullity(A_0) >= m * d_s
    D0 = oracle.dense(geo, order_mask=1)[: P0 * g.n_frames]
    assert D0.shape[1] - np.linalg.matrix_rank(D0) >= len(Z0) * g.n_cells


def test_zero_columns_are_the_support_based_set():
    """Column (s,k) of A_0 is zero iff no (ray, frame) has psi_s > 0 and tau_k > 0."""
    geo = tiny_geometry(**GEOMS["ratio1"])
    g = geo.grid
    P0 = geo.maps[0].n_rays
    D0 = oracle.dense(geo, order_mask=1)[: P0 * g.n_frames]
    r, phi, delay = geo.maps[0].r, geo.maps[0].phi, geo.maps[0].delay
    psi = np.stack([spatial_interp(g, np.eye(g.n_cells)[s], r, phi) for s in range(g.n_cells)], 1)
    tret = frame_times(g)[None, :] - delay[:, None]
    tau = np.stack([temporal_interp(g, np.eye(g.n_hat)[k], tret) for k in range(g.n_hat)], -1)
    touched = np.einsum("ps,pfk->sk", (psi > 1e-15).astype(float), (tau > 1e-15).astype(float)) > 0
    zero_cols = np.all(D0 == 0.0, axis=0).reshape(g.n_cells, g.n_hat)
    assert np.array_equal(zero_cols, ~touched)


def test_gram_monotonicity_and_order_blocks():
    geo = tiny_geometry(**GEOMS["ratio1"])
    g = geo.grid
    D = oracle.dense(geo)
    P = [m.n_rays * g.n_frames for m in geo.maps]
    prev = None
    for N in range(len(P)):
        DN = D[: sum(P[: N + 1])]
        s = np.linalg.svd(DN, compute_uv=False)
        if prev is not None:
            assert np.all(s[: len(prev)] >= prev[: len(s)] - 1e-14 * s[0])   # eq. (21)
        prev = s
    # masked rows are not produced, unmasked blocks are the stacked blocks of eq. (3)
    x = np.random.default_rng(9).standard_normal(g.n_cols)
    y12 = oracle.forward(geo, x, order_mask=0b110)
    assert np.all(y12[: P[0]] == 0.0)
    assert np.allclose(y12[P[0]:], (D @ x)[P[0]:], rtol=0, atol=1e-15)


def test_split_merge_gram_invariance():
    """eq. (15)-(16): four equal-area children with identical transfer values keep A^T A."""
    geo = tiny_geometry(**GEOMS["ratio1"])
    kids = []
    for m in geo.maps:
        rep = lambda a: np.repeat(a, 4)
        kids.append(synth.RayMap(r=rep(m.r), phi=rep(m.phi), delay=rep(m.delay),
                                 weight=rep(m.weight) * math.sqrt(0.25)))
    geo4 = synth.Geometry(grid=geo.grid, maps=kids)
    D, D4 = oracle.dense(geo), oracle.dense(geo4)
    G, G4 = D.T @ D, D4.T @ D4
    assert np.linalg.norm(G4 - G) / np.linalg.norm(G) <= 1e-10


def test_rsvd_equals_lapack_when_sketch_spans_range():
    geo = tiny_geometry(**GEOMS["ratio1"])
    D = oracle.dense(geo)
    s_ref_ = np.linalg.svd(D, compute_uv=False)
    om = np.random.default_rng(10).standard_normal((D.shape[1], D.shape[1]))
    s, V, U = oracle.rsvd(geo, om, q=2, want_u=True)
    k = int(np.sum(s_ref_ > 1e-12 * s_ref_[0]))
    assert np.max(np.abs(s[:k] - s_ref_[:k])) <= 1e-12 * s_ref_[0]
    # the factors reproduce A on the numerical range
    approx = (U[:k].T * s[:k]) @ V[:k]
    assert np.linalg.norm(approx - D) <= 1e-11 * np.linalg.norm(D)


def test_rsvd_partial_sketch_converges_with_power_iterations():
    """A partial sketch: Ritz values lie below the true ones and approach them as q grows.

    The tiny operator's spectrum is flat (sigma_1/sigma_40 ~ 1.4), so the error
    decays like (sigma_{l+1}/sigma_j)^(2q+1) (HMT 2011, Sec. 10.4) and needs q ~ 16.
    """
    geo = tiny_geometry(seed=15, rays=(40, 12, 10), n_r=6, n_phi=8, n_frames=10)
    D = oracle.dense(geo)
    s_true = np.linalg.svd(D, compute_uv=False)
    om = np.random.default_rng(16).standard_normal((40, D.shape[1]))
    errs = []
    for q in (0, 2, 8, 16):
        s, V, _ = oracle.rsvd(geo, om, q=q)
        assert np.all(s <= s_true[: len(s)] * (1 + 1e-12))
        errs.append(abs(s[0] - s_true[0]) / s_true[0])
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 1e-8


def test_block_lanczos_equals_lapack_when_space_exhausted():
    geo = tiny_geometry(**GEOMS["ratio_half"])
    D = oracle.dense(geo)
    s_true = np.linalg.svd(D, compute_uv=False)
    b = 4
    steps = D.shape[0] // b
    start = np.random.default_rng(17).standard_normal((b, D.shape[1]))
    s, V, res = oracle.block_lanczos(geo, start, steps)
    k = int(np.sum(s_true > 1e-10 * s_true[0]))
    assert np.max(np.abs(s[:k] - s_true[:k])) <= 1e-10 * s_true[0]
    assert np.max(res[:k]) <= 1e-8 * s_true[0]
    # Ritz vectors are right singular vectors: ||A v|| = sigma
    Av = D @ V[:k].T
    assert np.allclose(np.linalg.norm(Av, axis=0), s[:k], rtol=1e-9, atol=1e-12 * s[0])


def test_tsvd_is_truncated_pseudoinverse():
    geo = tiny_geometry(**GEOMS["ratio1"])
    D = oracle.dense(geo)
    U, s, Vt = np.linalg.svd(D, full_matrices=False)
    y = np.random.default_rng(18).standard_normal(D.shape[0])
    for t in (1, 5, 20):
        expect = Vt[:t].T @ ((U[:, :t].T @ y) / s[:t])
        got = oracle.tsvd_solve(geo, Vt, s, y, t)
        assert np.linalg.norm(got - expect) <= 1e-10 * np.linalg.norm(expect)


def test_ridge_cg_matches_dense_solve():
    geo = tiny_geometry(**GEOMS["ratio_half"])
    D = oracle.dense(geo)
    y = np.random.default_rng(19).standard_normal(D.shape[0])
    lam = 1e-3
    expect = np.linalg.solve(D.T @ D + lam * np.eye(D.shape[1]), D.T @ y)
    got, it = oracle.ridge_solve(geo, y, lam, tol=1e-13)
    assert np.linalg.norm(got - expect) <= 1e-9 * np.linalg.norm(expect)


def test_ridge_gradient_against_finite_differences():
    geo = tiny_geometry(**GEOMS["ratio1"])
    g = geo.grid
    rng = np.random.default_rng(20)
    x = rng.random(g.n_cols)
    y = rng.standard_normal(geo.n_rows)
    lam = 1e-3

    def loss(v):
        res = oracle.forward(geo, v) - y
        return 0.5 * float(res @ res) + 0.5 * lam * float(v @ v)

    grad = oracle.ridge_gradient(geo, x, y, lam)
    h = 1e-3
    for i in rng.choice(g.n_cols, 16, replace=False):
        e = np.zeros(g.n_cols)
        e[i] = h
        fd = (loss(x + e) - loss(x - e)) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-7, abs=1e-9)


def test_operational_rank_threshold():
    s = np.array([3.0, 1.0, 0.02, 0.01, 0.005])
    assert oracle.operational_rank(s, s_reference=1.0, snr0=100.0) == 4   # sigma >= 0.01
    assert oracle.operational_rank(s, s_reference=1.0, snr0=100.0, rho=3.0) == 2


def test_oracle_rejects_bad_grid():
    geo = tiny_geometry(**GEOMS["ratio1"])
    bad = synth.Geometry(grid=synth.Grid(**{**geo.grid.as_dict(), "n_r": 1}), maps=geo.maps)
    with pytest.raises(ValueError):
        oracle.forward(bad, np.zeros(bad.grid.n_cols))


# ------------------------------------------------------------------ order mixer, eq. (4)
def _golden_mixer():
    """The hand-worked fixture tests/golden/order_mixer_example.txt as a geometry-like object."""
    import os
    import types
    rows, unres, tf, vu, vt = [], {}, None, {}, None
    with open(os.path.join(os.path.dirname(__file__), "golden", "order_mixer_example.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "ray":
                rows.append(tuple(float(v) for v in t[1:]))
            elif t[0] == "unresolved":
                unres[int(t[1])] = [float(t[2]), float(t[3])]
            elif t[0] == "total_flux":
                tf = [float(t[1]), float(t[2])]
            elif t[0] == "var_unresolved":
                vu[int(t[1])] = float(t[2])
            elif t[0] == "var_total_flux":
                vt = float(t[1])
    maps = []
    for n in range(3):
        pix = np.array([int(r[2]) for r in rows if int(r[1]) == n])
        maps.append(types.SimpleNamespace(pixel=pix, n_rays=pix.size))
    geo = types.SimpleNamespace(maps=maps, n_rays=len(rows), grid=types.SimpleNamespace(n_frames=2))
    y = np.array([[r[3], r[4]] for r in rows]).ravel()
    var = np.array([[r[5], r[5]] for r in rows]).ravel()
    return geo, y, var, unres, tf, vu, vt


def test_order_mixer_hand_worked_example():
    """eq. (4) on a five-ray, three-order example summed by hand (golden fixture)."""
    geo, y, var, unres, tf, vu, vt = _golden_mixer()
    L, pix = oracle.mixer_matrix(geo, "unresolved")
    assert list(pix) == sorted(unres)
    d = oracle.mix(geo, y, "unresolved").reshape(-1, 2)
    for i, p in enumerate(pix):
        assert np.array_equal(d[i], unres[p])
    assert np.array_equal(oracle.mix(geo, y, "total_flux"), tf)
    C = oracle.mix_covariance(geo, var, "unresolved")
    assert np.array_equal(C, np.diag(np.repeat([vu[p] for p in pix], 2)))
    assert np.array_equal(oracle.mix_covariance(geo, var, "total_flux"), vt * np.eye(2))


def test_order_mixer_adjoint_and_total_flux_invariants():
    """<L y, d> = <y, L^T d>; the total flux is the sum of the unresolved image over pixels."""
    geo = tiny_geometry(seed=41, rays=(30, 20, 10), n_frames=7)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((2, geo.n_rows))
    for kind in oracle.MIX_KINDS:
        d = rng.standard_normal((2, oracle.mixer_matrix(geo, kind)[0].shape[0] * geo.grid.n_frames))
        lhs = np.sum(oracle.mix(geo, y, kind) * d)
        rhs = np.sum(y * oracle.mix_adjoint(geo, d, kind))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs) + 1)
    du = oracle.mix(geo, y, "unresolved").reshape(2, -1, geo.grid.n_frames)
    assert np.allclose(du.sum(axis=1), oracle.mix(geo, y, "total_flux"), rtol=1e-13, atol=1e-12)


def test_order_mixer_covariance_matches_monte_carlo():
    """C_L of eq. (4) against the sample covariance of L applied to independent Gaussian noise
    with the per-datum variances of the fixture (a check that does not use the formula)."""
    geo, _, var, *_ = _golden_mixer()
    rng = np.random.default_rng(11)
    N = 40000
    Z = rng.standard_normal((N, var.size)) * np.sqrt(var)
    for kind in oracle.MIX_KINDS:
        D = oracle.mix(geo, Z, kind)
        emp = D.T @ D / N
        C = oracle.mix_covariance(geo, var, kind)
        scale = np.sqrt(np.outer(np.diag(C), np.diag(C)))
        # sample (co)variances have relative standard deviation about sqrt(2 / N) = 0.7%
        assert np.max(np.abs(emp - C) / scale) < 0.04, kind


def test_unresolved_echo_train_inverts_with_the_echo_recursion():
    """Sec. 4, the scalar echo train: when every pixel sees the same source point in orders
    n = 0, 1, 2 with delays Delta + n tau and weights a^n, the unresolved series is
    d(t) = sum_n a^n y0(t - n tau), so d(t) - a d(t - tau) = y0(t) - a^3 y0(t - 3 tau) for the
    three retained orders (tau a whole number of frames and hats, y0 the direct series)."""
    m, a = 3, 0.45
    grid = synth.Grid(n_orders=3, n_frames=40, t0=0.0, dt_obs=4.0, n_r=5, n_phi=7, r_in=6.0, r_out=20.0,
                      n_hat=80, s0=-150.0, dt_src=4.0)
    tau = m * grid.dt_obs
    rng = np.random.default_rng(5)
    npix = 25
    r = rng.uniform(grid.r_in, grid.r_out, npix)
    phi = rng.uniform(0.0, 2 * np.pi, npix)
    dl = rng.uniform(0.3, 9.7, npix)
    maps = [synth.RayMap(r=r, phi=phi, delay=dl + n * tau, weight=np.full(npix, a ** n),
                         pixel=np.arange(npix, dtype=np.int32)) for n in range(3)]
    geo = synth.Geometry(grid=grid, maps=maps)
    x = rng.random(grid.n_cols)
    y = oracle.forward(geo, x)
    F = grid.n_frames
    y0 = y[: npix * F].reshape(npix, F)
    d = oracle.mix(geo, y, "unresolved").reshape(npix, F)
    f = np.arange(3 * m, F)
    lhs = d[:, f] - a * d[:, f - m]
    rhs = y0[:, f] - a ** 3 * y0[:, f - 3 * m]
    assert np.max(np.abs(lhs - rhs)) <= 1e-11 * np.max(np.abs(y0))
    assert np.max(np.abs(rhs)) > 0.1 * np.max(np.abs(y0))


# ----------------------------------------------------------------------------- age probes (Sec. 3.3, 4.4)
def test_age_probe_has_unit_norm_over_the_annulus():
    """eq. (10)-(11): the continuum probe has unit L2 norm under the area measure r dr dphi dt,
    checked by numerical quadrature of the separable integrand (not by the closed form)."""
    from scipy.integrate import quad
    g = tiny_geometry(seed=1).grid
    for h in (3.0, 1.7):
        n2 = oracle.probe_norm(g, h) ** 2
        radial = quad(lambda r: r, g.r_in, g.r_out)[0] * 2.0 * math.pi
        for a in (0.0, 37.0):
            temporal = quad(lambda t: math.exp(-((t + a) ** 2) / (h * h)), -a - 40 * h, -a + 40 * h)[0]
            assert abs(radial * temporal / n2 - 1.0) < 1e-10


def test_age_probe_response_is_the_linear_interpolant_of_the_gaussian():
    """A flat probe on the nodes: the bilinear weights of a ray add to 1, so the datum is w times the
    piecewise-linear interpolant (numpy.interp) of the probe's values at the hat centres."""
    geo = tiny_geometry(seed=5, rays=(9, 4))
    g = geo.grid
    ages = np.array([0.0, 8.0, 20.0])
    h = 3.0
    Y = oracle.forward(geo, oracle.age_probes(g, ages, h))
    s_k = g.s0 + g.dt_src * np.arange(g.n_hat)
    t_f = g.t0 + g.dt_obs * np.arange(g.n_frames)
    nh = oracle.probe_norm(g, h)
    row = 0
    for m in geo.maps:
        for p in range(m.n_rays):
            for i, a in enumerate(ages):
                node = np.exp(-((s_k + a) ** 2) / (2 * h * h)) / nh
                want = m.weight[p] * np.interp(t_f - m.delay[p], s_k, node, left=0.0, right=0.0)
                assert np.allclose(Y[i, row * g.n_frames:(row + 1) * g.n_frames], want, rtol=1e-12, atol=1e-15)
            row += 1


def test_age_energy_orders_the_arms_and_a_one_ray_per_pixel_collapse_loses_nothing():
    """Collapsing whitened data never adds information: total flux <= unresolved <= resolved and
    direct <= resolved; a mixer that sends every ray to its own pixel is a permutation and keeps all."""
    geo = tiny_geometry(seed=9, rays=(14, 8, 5), n_frames=5)
    ages = np.arange(0.0, 40.0, 8.0)
    res = oracle.age_energy(geo, ages, arm="resolved")
    dire = oracle.age_energy(geo, ages, arm="direct")
    unr = oracle.age_energy(geo, ages, arm="unresolved")
    tot = oracle.age_energy(geo, ages, arm="total_flux")
    assert np.all(res > 0)
    assert np.all(dire <= res * (1 + 1e-12)) and np.all(unr <= res * (1 + 1e-12))
    assert np.all(tot <= unr * (1 + 1e-12))
    base = 0
    pix = []
    for m in geo.maps:
        pix.append(np.arange(base, base + m.n_rays))
        base += m.n_rays
    own = synth.Geometry(grid=geo.grid, maps=[dataclasses.replace(m, pixel=p) for m, p in zip(geo.maps, pix)])
    assert np.allclose(oracle.age_energy(own, ages, arm="unresolved"), res, rtol=1e-12)
    # per-datum variances scale the information down: var = 4 everywhere quarters it
    var = np.full(geo.n_rows, 4.0)
    assert np.allclose(oracle.age_energy(geo, ages, arm="unresolved", var=var), unr / 4.0, rtol=1e-12)


def test_supported_ages_match_the_footprint_of_eq_13():
    """Brute force over every datum agrees with the footprint [t_min - Delta_max, t_max - Delta_min]."""
    geo = tiny_geometry(seed=13, rays=(7, 5, 4), n_frames=20, delay_hi=30.0)
    g = geo.grid
    ages = np.arange(0.0, 120.0, 4.0)
    t_lo, t_hi = g.t0, g.t0 + g.dt_obs * (g.n_frames - 1)
    for mask in (1, 7):
        d = np.concatenate([m.delay for n, m in enumerate(geo.maps) if (mask >> n) & 1])
        lo, hi = t_lo - d.max(), t_hi - d.min()
        want = (-ages - 9.0 >= lo) & (-ages + 9.0 <= hi)
        assert np.array_equal(oracle.supported_ages(geo, ages, 3.0, order_mask=mask), want)
        assert want.any() and not want.all()


def test_throughput_age_boundary_hand_example():
    """Two direct rays (weights 1 and -3, delays 10 and 20) seen at t = 0 and 4: ages 10, 6, 20, 16
    with weights 1, 1, 3, 3; cumulative 1, 2, 5, 8 in age order."""
    grid = synth.Grid(n_orders=1, n_frames=2, t0=0.0, dt_obs=4.0, n_r=2, n_phi=2, r_in=6.0, r_out=20.0,
                      n_hat=4, s0=-30.0, dt_src=4.0)
    m = synth.RayMap(r=np.array([8.0, 9.0]), phi=np.array([0.1, 0.2]), delay=np.array([10.0, 20.0]),
                     weight=np.array([1.0, -3.0]))
    geo = synth.Geometry(grid=grid, maps=[m])
    assert oracle.throughput_age_boundary(geo, 0.999) == 20.0
    assert oracle.throughput_age_boundary(geo, 0.5) == 16.0
    assert oracle.throughput_age_boundary(geo, 0.2) == 10.0
    assert oracle.throughput_age_boundary(geo, 0.1) == 6.0


def test_reach_statistics_hand_example():
    rows, expect = [], None
    with open(os.path.join(os.path.dirname(__file__), "golden", "age_reach_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "expect":
                expect = [float(v) for v in line[1:]]
            else:
                rows.append([float(v) for v in line])
    ages, info, sup = zip(*rows)
    rho, boundary, t_reach, anchor, l_anchor, longest, j_old = expect
    r = oracle.reach(ages, info, rho=rho, supported=[bool(s) for s in sup], boundary=boundary)
    assert r["t_reach"] == t_reach and r["anchor"] == int(anchor)
    assert r["l_anchor"] == l_anchor and r["longest"] == longest
    assert abs(r["j_old"] - j_old) < 1e-12
    # no supported centre passing: no anchor-connected span
    r2 = oracle.reach(ages, info, rho=rho, supported=[i == 3 for i in range(len(ages))], boundary=boundary)
    assert r2["anchor"] == 3 and r2["l_anchor"] is None


# ----------------------------------------------------------------------------- estimator derivatives, noise
def _tiny_dense_geo():
    return tiny_geometry(seed=61, rays=(7, 4), n_r=3, n_phi=3, n_frames=4)


def test_ridge_data_gradient_matches_central_differences_of_the_cg_solve():
    """d/dy <g, x_hat(y)> against central differences of the CG ridge solve (a different route
    from the dense normal-matrix solve the gradient uses)."""
    geo = _tiny_dense_geo()
    rng = np.random.default_rng(62)
    lam = 0.05
    y = rng.standard_normal(geo.n_rows)
    g = rng.standard_normal(geo.grid.n_cols)
    d = rng.standard_normal(geo.n_rows)
    grad = oracle.ridge_data_gradient(geo, g, lam)
    eps = 1e-4
    xp, _ = oracle.ridge_solve(geo, y + eps * d, lam)
    xm, _ = oracle.ridge_solve(geo, y - eps * d, lam)
    fd = float(g @ (xp - xm)) / (2 * eps)
    assert abs(fd - float(grad @ d)) <= 1e-7 * max(1.0, abs(fd))
    # the normal-equation solve with b = A^T y is the ridge estimate itself
    x_cg, _ = oracle.ridge_solve(geo, y, lam)
    b = oracle.adjoint(geo, y)
    assert np.allclose(oracle.ridge_normal_solve(geo, b, lam), x_cg, rtol=1e-8, atol=1e-10)


def test_tsvd_projection_of_a_full_rank_factorisation_is_the_pseudo_inverse():
    """With every nonzero singular triplet kept, V diag(sigma^-2) V^T A^T y = pinv(A) y."""
    geo = _tiny_dense_geo()
    A = oracle.dense(geo)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    r = int(np.sum(s > 1e-10 * s[0]))
    y = np.random.default_rng(63).standard_normal(geo.n_rows)
    got = oracle.tsvd_project(Vt, s, oracle.adjoint(geo, y), r)
    assert np.allclose(got, np.linalg.pinv(A, rcond=1e-10) @ y, rtol=1e-8, atol=1e-10)


def test_age_window_error_hand_example():
    grid = synth.Grid(n_orders=1, n_frames=1, t0=0.0, dt_obs=4.0, n_r=2, n_phi=1, r_in=6.0, r_out=20.0,
                      n_hat=4, s0=-12.0, dt_src=4.0)
    x = np.array([1, 2, 3, 4, 5, 6, 7, 8], dtype=np.float64)
    d = np.array([0, 1, 0, 0, 0, 0, 3, -4], dtype=np.float64)
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "age_window_error_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                rows.append([float(v) for v in line])
    ages, want = zip(*rows)
    got = oracle.age_window_error(grid, x + d, x, ages, half_width=2.0, eta=0.5)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-15)
    # eta takes over when the window holds nothing of x
    assert oracle.age_window_error(grid, 0 * x + 1.0, 0 * x, [0.0], 2.0, eta=0.5)[0] == math.sqrt(2.0) / 0.5


def test_philox_known_answers():
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")) as f:
        n = 0
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            w = [int(v, 16) for v in line]
            assert oracle.philox4x32_10(w[0:4], w[4:6]) == w[6:10]
            n += 1
    assert n == 3


def test_normal_draws_are_standard_normal():
    """Moments and a Kolmogorov-Smirnov test against scipy's normal CDF; different seeds give
    different streams."""
    from scipy import stats
    z = oracle.normal_draws(40000, seed=1234)
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert not np.allclose(oracle.normal_draws(16, seed=1235), z[:16])


# ----------------------------------------------------------------------------- representation synthesis (Sec. 3.2, 7)
def test_radial_bsplines_are_the_bernstein_basis_and_a_partition_of_unity():
    """Clamped cubic B-splines without interior knots are the cubic Bernstein polynomials in
    u = log(r / r_in) / log(r_out / r_in); with interior knots they still sum to one."""
    r = np.linspace(6.0, 20.0, 57)
    u = np.log(r / 6.0) / math.log(20.0 / 6.0)
    B = oracle._radial_bsplines(r, 6.0, 20.0, 4)
    bern = np.stack([math.comb(3, a) * u ** a * (1 - u) ** (3 - a) for a in range(4)], axis=1)
    assert np.allclose(B, bern, atol=1e-13)
    B7 = oracle._radial_bsplines(r, 6.0, 20.0, 7)
    assert np.allclose(B7.sum(axis=1), 1.0, atol=1e-13)
    assert B7[0, 0] == 1.0 and abs(B7[-1, -1] - 1.0) < 1e-13 and np.all(B7 >= 0)


def test_synthesis_temporal_and_azimuthal_factors():
    """On the default window the DCT columns at the hat nodes are scipy's DCT-II vectors; the
    azimuthal factors are orthogonal over the node grid."""
    from scipy.fft import dct
    g = tiny_geometry(seed=1, n_phi=9).grid
    Q = oracle.synthesis_matrix(g, n_radial=4, m_max=3, n_temporal=8, temporal="dct")
    T = Q.reshape(g.n_r, g.n_phi, g.n_hat, 4, 7, 8)[0, 0, :, 0, 0, :]      # R_0(r_0) Phi_0 = R_0(r_0)
    T = T / T[0, 0]
    x = np.random.default_rng(3).standard_normal(g.n_hat)
    assert np.allclose(T.T @ x, dct(x, type=2)[:8] / 2.0, atol=1e-12)
    P = Q.reshape(g.n_r, g.n_phi, g.n_hat, 4, 7, 8)[0, :, 0, 0, :, 0]
    PtP = P.T @ P
    assert np.allclose(PtP - np.diag(np.diag(PtP)), 0.0, atol=1e-12 * np.abs(PtP).max())


def test_compact_temporal_class_has_exact_zero_columns_where_the_direct_footprint_is_missed():
    """Sec. 7 / Thm 4.1: a temporal function whose node support is farther than one hat width from
    every direct retarded time t_f - Delta_p gives an exactly zero column of A_0 Q for each of the
    28 spatial functions; counted by brute force over the data."""
    geo = tiny_geometry(seed=41, rays=(15, 6, 4), n_frames=3, n_r=4, n_phi=8, delay_hi=6.0)
    g = geo.grid
    Q = oracle.synthesis_matrix(g, temporal="hats", n_temporal=8)
    audit = oracle.synthesis_audit(geo, Q, order_mask=1)
    sk = g.s0 + g.dt_src * np.arange(g.n_hat)
    T = Q.reshape(g.n_r, g.n_phi, g.n_hat, 4, 7, 8)[0, 0, :, 0, 0, :]
    t_ret = np.array([g.t0 + g.dt_obs * f - d for d in geo.maps[0].delay for f in range(g.n_frames)])
    blind = [c for c in range(8)
             if not any(T[k, c] != 0 and np.any(np.abs(sk[k] - t_ret) < g.dt_src) for k in range(g.n_hat))]
    assert 0 < len(blind) < 8
    assert len(audit["zero_columns"]) == 28 * len(blind)
    assert sorted({c % 8 for c in audit["zero_columns"]}) == blind
    # the resolved stack reaches further back: fewer zero columns
    assert len(oracle.synthesis_audit(geo, Q)["zero_columns"]) < len(audit["zero_columns"])


def test_localized_probes_have_unit_norm():
    """eq. (14): psi_l g_a / N_{h,l} has unit L2 norm, by a 2-D quadrature over the annulus (in
    Cartesian-free polar form r dr dphi) that does not separate the radial and azimuthal factors."""
    from scipy.integrate import dblquad
    g = tiny_geometry(seed=1).grid
    n = oracle.localized_probe_norms(g, 4, 3, h=3.0)
    for l in (0, 5, 13, 27):
        a, b = divmod(l, 7)
        m = (b + 1) // 2

        def psi2(phi, r):
            R = oracle._radial_bsplines(np.array([r]), g.r_in, g.r_out, 4)[0, a]
            P = 1.0 if b == 0 else (math.cos(m * phi) if b % 2 == 1 else math.sin(m * phi))
            return (R * P) ** 2 * r
        sp = dblquad(psi2, g.r_in, g.r_out, 0.0, 2.0 * math.pi, epsabs=0.0, epsrel=1e-10)[0]
        assert abs(sp * 3.0 * math.sqrt(math.pi) / n[l] ** 2 - 1.0) < 1e-8


def test_fisher_reproduces_the_flat_probe_information():
    """The radial B-splines sum to one on the nodes, so the flat probe of eq. (10) is the combination
    sum_a (N_{h,(a,0)} / N_h) q_{a,(a,0)} of localised probes and its information (computed by the
    separate flat-probe routine) is the matching quadratic form of M(a)."""
    geo = tiny_geometry(seed=9, rays=(14, 8, 5), n_frames=5)
    ages = np.array([0.0, 7.0, 20.0])
    M = oracle.age_fisher(geo, ages, h=3.0)
    assert np.allclose(M, np.transpose(M, (0, 2, 1)), rtol=1e-12, atol=1e-15)
    assert np.all(np.linalg.eigvalsh(M) > -1e-12 * np.abs(M).max())
    nl = oracle.localized_probe_norms(geo.grid, 4, 3, 3.0)
    w = np.zeros(28)
    for a in range(4):
        w[a * 7] = nl[a * 7] / oracle.probe_norm(geo.grid, 3.0)
    flat = oracle.age_energy(geo, ages, h=3.0, arm="resolved")
    assert np.allclose(np.einsum("l,alm,m->a", w, M, w), flat, rtol=1e-10)


def test_compact_temporal_functions_are_tents_on_uniform_knots():
    """The compact temporal class of Sec. 7 (degree-one B-splines on n uniform knots spanning the
    window): isolated as the ratio of a "hats" column to the constant DCT column of the same
    spatial function (pinned to scipy's DCT-II above), each function is numpy.interp of its unit
    knot vector; with a window whose knots land on hat nodes it is 1 at its own knot and 0 at
    every other knot; the functions sum to one over the window."""
    g = tiny_geometry(seed=1, n_frames=20).grid
    K = g.n_hat
    sk = g.s0 + g.dt_src * np.arange(K)

    def temporal(n, window):
        Qh = oracle.synthesis_matrix(g, temporal="hats", n_temporal=n, window=window)
        Qd = oracle.synthesis_matrix(g, temporal="dct", n_temporal=n, window=window)
        Qh = Qh.reshape(g.n_r, g.n_phi, K, 4, 7, n)
        Qd = Qd.reshape(g.n_r, g.n_phi, K, 4, 7, n)
        i, j, a, b = 1, 2, 1, 0                  # R_1(r_1) Phi_0(phi_2) != 0
        assert abs(Qd[i, j, 0, a, b, 0]) > 1e-3
        return Qh[i, j, :, a, b, :] / Qd[i, j, :, a, b, 0][:, None]     # [K][n]

    # default window [s0 - dt/2, s0 + (K - 1/2) dt]
    lo, hi = g.s0 - 0.5 * g.dt_src, g.s0 + (K - 0.5) * g.dt_src
    for n in (2, 5, 8):
        T = temporal(n, None)
        knots = lo + (hi - lo) * np.arange(n) / (n - 1)
        for c in range(n):
            assert np.allclose(T[:, c], np.interp(sk, knots, np.eye(n)[c]), atol=1e-13), (n, c)
        assert np.allclose(T.sum(axis=1), 1.0, atol=1e-13)
    # knots on every fourth hat node: the Kronecker property at the knots
    n = (K - 1) // 4 + 1
    window = (sk[0], sk[4 * (n - 1)])
    T = temporal(n, window)
    for c in range(n):
        assert np.allclose(T[4 * np.arange(n), c], np.eye(n)[c], atol=1e-13), c
        support = np.nonzero(T[:, c])[0]
        assert support.min() >= 4 * c - 3 and support.max() <= 4 * c + 3, c
