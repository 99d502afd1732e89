"""Batched row: several geometries and histories per call, graph capture, batched autograd.

Every geometry of a block-diagonal handle is an independent problem; each is
checked against the FP64 oracle run on that geometry alone.  Tolerances as in
the other GPU tests: 1e-5 relative for outputs the oracle computes with the
same arithmetic, 1e-4 relative on singular values >= 1e-3 sigma_1.
"""
import sys

import numpy as np
import pytest

import oracle
from tinygeo import tiny_geometry

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def batch_geometries(n=3, seed=70):
    """Geometries of uneven size and frame count (shared source grid shape per geometry)."""
    return [tiny_geometry(seed=seed + i, rays=(40 + 13 * i, 12, 6), n_r=4 + (i % 2), n_phi=6 + 2 * i,
                          n_frames=8 + 4 * i) for i in range(n)]


def blocks(G, g):
    m = G.members[g]
    return (slice(m["col_offset"], m["col_offset"] + m["n_cols"]),
            slice(m["row_offset"], m["row_offset"] + m["n_rows"]))


def test_rsvd_of_every_geometry_in_one_call_matches_oracle(gpu_lib):
    rtt = gpu_lib
    geos = batch_geometries()
    G = rtt.Geometry(geos)
    say("case batched rsvd", [g.grid.n_cols for g in geos])
    k, p = 24, 8
    om = np.random.default_rng(7).standard_normal((k + p, G.n_cols)).astype(np.float32)
    sv = rtt.rsvd(G, k=k, p=p, q=2, omega=to_dev(om), geometry=rtt.RTT_EACH_GEOMETRY, keep_u=True)
    assert sv.sigma.shape == (3, k)
    V = sv.V().double().cpu().numpy()
    U = sv.U().double().cpu().numpy()
    for g, geo in enumerate(geos):
        cs, _ = blocks(G, g)
        s_o, V_o, _ = oracle.rsvd(geo, om[:, cs].astype(np.float64), q=2)
        ok = s_o[:k] >= 1e-3 * s_o[0]
        assert np.max(np.abs(sv.sigma[g][ok] - s_o[:k][ok]) / s_o[:k][ok]) <= 1e-4, g
        # leading right vectors agree up to sign where the spectrum has a gap
        Vg = V[:, cs]
        for i in range(4):
            gap = min(abs(s_o[i] - s_o[i + 1]), abs(s_o[i] - s_o[i - 1]) if i else np.inf) / s_o[0]
            if gap > 1e-2:
                c = abs(float(Vg[i] @ V_o[i])) / (np.linalg.norm(Vg[i]) * np.linalg.norm(V_o[i]))
                assert c >= 1 - 1e-4, (g, i)
        # the reported residuals ||A v_i - sigma_i u_i|| of this geometry, recomputed in FP64
        _, rs = blocks(G, g)
        Ug = U[:, rs]
        r64 = np.linalg.norm(oracle.forward(geo, Vg) - sv.sigma[g][:, None] * Ug, axis=1)
        assert np.max(np.abs(sv.residual[g] - r64)) <= 1e-5 * sv.sigma[g][0], g


def test_rsvd_segments_with_and_without_the_shifted_pass(gpu_lib):
    """One rSVD call over four geometries whose sketch of 340 vectors exceeds the rank of two of
    them (their first Cholesky QR pass is shifted and takes one more pass, decided per segment on
    the device) and not of the other two.  Every set against the oracle's rSVD on the same test
    block (1e-4 on sigma >= 1e-3 sigma_1), and bitwise against the same member factored alone."""
    rtt = gpu_lib
    geos = [tiny_geometry(seed=90, rays=(40, 12, 6), n_r=4, n_phi=6, n_frames=8),
            tiny_geometry(seed=95, rays=(80, 20, 10), n_r=4, n_phi=8, n_frames=16),
            tiny_geometry(seed=94, rays=(30, 10, 5), n_r=4, n_phi=6, n_frames=8, delay_hi=2.0),
            tiny_geometry(seed=92, rays=(60, 20, 10), n_r=4, n_phi=6, n_frames=12)]
    G = rtt.Geometry(geos)
    k, p = 300, 40
    say("case rsvd shifted segments", [(g.n_rows, g.grid.n_cols) for g in geos])
    om = np.random.default_rng(9).standard_normal((k + p, G.n_cols)).astype(np.float32)
    sv = rtt.rsvd(G, k=k, p=p, q=1, omega=to_dev(om), geometry=rtt.RTT_EACH_GEOMETRY)
    ranks = []
    for g, geo in enumerate(geos):
        cs, _ = blocks(G, g)
        D = oracle.dense(geo)
        s_true = np.linalg.svd(D, compute_uv=False)
        rank = int(np.sum(s_true > 1e-6 * s_true[0]))
        ranks.append(rank)
        s_o, _, _ = oracle.rsvd(geo, om[:, cs].astype(np.float64), q=1)
        ok = s_o[:k] >= 1e-3 * s_o[0]
        err = np.max(np.abs(sv.sigma[g][ok] - s_o[:k][ok]) / s_o[:k][ok])
        say("geometry", g, "rank", rank, "of sketch", k + p, "sigma err", err)
        assert err <= 1e-4, (g, err)
        one = rtt.rsvd(G, k=k, p=p, q=1, omega=to_dev(om[:, cs]), geometry=g)
        assert np.array_equal(one.sigma.ravel(), sv.sigma[g]), g
    # both kinds of segment are present: rank below the sketch (shifted) and above it
    assert min(ranks) < k + p <= max(ranks), ranks


def test_tsvd_of_every_geometry_matches_oracle(gpu_lib):
    rtt = gpu_lib
    geos = batch_geometries(seed=80)
    G = rtt.Geometry(geos)
    sv = rtt.rsvd(G, k=20, p=10, q=2, seed=5, geometry=rtt.RTT_EACH_GEOMETRY)
    V = sv.V().double().cpu().numpy()
    y = np.random.default_rng(8).standard_normal((2, G.n_rows)).astype(np.float32)
    for t, smin in ((9, 0.0), (0, None)):
        if smin is None:
            smin = float(np.median(sv.sigma[:, 5]))
        x = rtt.tsvd_solve(G, sv, to_dev(y), t=t, sigma_min=smin).cpu().numpy()
        for g, geo in enumerate(geos):
            cs, rs = blocks(G, g)
            tg = t if t > 0 else int(np.sum(sv.sigma[g] >= smin))
            xo = oracle.tsvd_solve(geo, V[:, cs], sv.sigma[g], y[:, rs].astype(np.float64), tg)
            assert rel(x[:, cs], xo) <= TOL, (t, g)


def test_ridge_solves_every_geometry_and_history_independently(gpu_lib):
    rtt = gpu_lib
    geos = batch_geometries(seed=90)
    G = rtt.Geometry(geos)
    lam = 1e-1
    y = np.random.default_rng(9).standard_normal((3, G.n_rows)).astype(np.float32)
    x, info = rtt.ridge_solve(G, to_dev(y), lam, tol=1e-6, maxit=2000)
    assert info["converged"] == 3 * len(geos)
    x = x.cpu().numpy()
    for g, geo in enumerate(geos):
        cs, rs = blocks(G, g)
        D = oracle.dense(geo)
        xe = np.linalg.solve(D.T @ D + lam * np.eye(D.shape[1]), D.T @ y[:, rs].T.astype(np.float64)).T
        assert rel(x[:, cs], xe) <= 1e-4, g
    # the same solve, geometry by geometry on handles of their own
    for g, geo in enumerate(geos):
        cs, rs = blocks(G, g)
        xg, _ = rtt.ridge_solve(rtt.Geometry(geo), to_dev(y[:, rs]), lam, tol=1e-6, maxit=2000)
        assert rel(x[:, cs], xg.cpu().numpy()) <= 1e-5, g


def test_async_ridge_equals_blocking(gpu_lib):
    import torch
    rtt = gpu_lib
    geos = batch_geometries(seed=100)
    G = rtt.Geometry(geos)
    y = to_dev(np.random.default_rng(10).standard_normal((2, G.n_rows)))
    xb, info = rtt.ridge_solve(G, y, 1e-1, tol=1e-6, maxit=2000)
    resid = torch.empty(2 * len(geos), dtype=torch.float32, device="cuda")
    xa, info_a = rtt.ridge_solve(G, y, 1e-1, tol=1e-6, maxit=info["iterations"] + 5, async_mode=True, resid=resid)
    torch.cuda.synchronize()
    assert info_a["converged"] == -1
    assert torch.equal(xa, xb)
    assert float(resid.max()) <= 1e-6 * (1 + 1e-3)


def test_graph_replay_of_batched_step_matches_eager(gpu_lib):
    """A, A^T, TSVD and a fixed-count ridge solve of every geometry captured once and replayed."""
    import torch
    rtt = gpu_lib
    geos = batch_geometries(seed=110)
    G = rtt.Geometry(geos)
    sv = rtt.rsvd(G, k=16, p=8, q=1, seed=3, geometry=rtt.RTT_EACH_GEOMETRY)
    nh = 4
    rng = np.random.default_rng(11)
    x_in = to_dev(rng.random((nh, G.n_cols)))
    y_in = to_dev(rng.standard_normal((nh, G.n_rows)))
    y_out = torch.empty((nh, G.n_rows), device="cuda")
    x_adj = torch.empty((nh, G.n_cols), device="cuda")
    x_ts = torch.empty((nh, G.n_cols), device="cuda")
    x_rg = torch.empty((nh, G.n_cols), device="cuda")
    resid = torch.empty(nh * len(geos), device="cuda")

    def step():
        rtt.op_apply(G, x_in, y=y_out)
        rtt.op_apply_adjoint(G, y_in, x=x_adj)
        rtt.tsvd_solve(G, sv, y_in, t=10, x=x_ts)
        rtt.ridge_solve(G, y_in, 1e-1, maxit=30, x=x_rg, async_mode=True, resid=resid)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                       # sizes the scratch of the solvers before capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        x_in.copy_(to_dev(rng.random((nh, G.n_cols))))
        y_in.copy_(to_dev(rng.standard_normal((nh, G.n_rows))))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in (y_out, x_adj, x_ts, x_rg, resid)]
        step()                       # eager on the same inputs, between replays
        torch.cuda.synchronize()
        ref = (y_out, x_adj, x_ts, x_rg, resid)
        for i, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a, b), (rep, i)
    # and the eager results are the oracle's
    xi = x_in.double().cpu().numpy()
    for g, geo in enumerate(geos):
        cs, rs = blocks(G, g)
        assert rel(y_out[:, rs].cpu().numpy(), oracle.forward(geo, xi[:, cs])) <= TOL


def test_batched_autograd_matches_per_geometry_oracle(gpu_lib):
    rtt = gpu_lib
    from paper_2609_05528_amd.autograd import ridge_loss
    geos = batch_geometries(seed=120)
    G = rtt.Geometry(geos)
    rng = np.random.default_rng(12)
    nh, lam = 3, 1e-3
    x0 = rng.random((nh, G.n_cols)).astype(np.float32)
    y = rng.standard_normal((nh, G.n_rows)).astype(np.float32)
    xd = to_dev(x0).requires_grad_(True)
    ridge_loss(xd, to_dev(y), G, lam).backward()
    grad = xd.grad.double().cpu().numpy()
    for g, geo in enumerate(geos):
        cs, rs = blocks(G, g)
        go = oracle.ridge_gradient(geo, x0[:, cs].astype(np.float64), y[:, rs].astype(np.float64), lam)
        assert rel(grad[:, cs], go) <= TOL, g
