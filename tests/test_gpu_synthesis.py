"""Representation synthesis Q_d (Sec. 3.2, Sec. 7) and the rank audit of A Q_d on the GPU against the
FP64 oracle: the rows of Q, the synthesis and its transpose, exactly zero columns and singular
values on a small geometry (DCT-II and compact temporal classes; singular values >= 1e-3 sigma_1 to
1e-4), and the S_224 audit of the 128^2 x 128-frame Kerr workload (zero columns exactly, singular
values >= 1e-3 sigma_1 to 1e-4).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tinygeo import tiny_geometry

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("temporal,n_radial,n_temporal", [("dct", 4, 8), ("hats", 6, 8), ("dct", 5, 3)])
def test_synthesis_rows_expand_and_project_match_oracle(gpu_lib, temporal, n_radial, n_temporal):
    import torch
    rtt = gpu_lib
    geo = tiny_geometry(seed=41, rays=(15, 6, 4), n_frames=3, n_r=4, n_phi=8, delay_hi=6.0)
    G = rtt.Geometry(geo)
    say("case synthesis", temporal, n_radial, n_temporal)
    S = rtt.Synthesis(G, 0, n_radial=n_radial, m_max=3, n_temporal=n_temporal, temporal=temporal)
    Q = oracle.synthesis_matrix(geo.grid, n_radial=n_radial, m_max=3, n_temporal=n_temporal, temporal=temporal)
    assert S.d == Q.shape[1] and S.n_cols == geo.grid.n_cols
    rows = S.expand(torch.eye(S.d, device="cuda")).cpu().numpy()
    assert rel(rows, Q.T) < 1e-6
    rng = np.random.default_rng(42)
    c = rng.standard_normal((5, S.d))
    x = rng.standard_normal((5, S.n_cols))
    assert rel(S.expand(to_dev(c)).cpu().numpy(), c.astype(np.float32) @ Q.T) < 1e-5
    assert rel(S.project(to_dev(x)).cpu().numpy(), x.astype(np.float32) @ Q) < 1e-5
    for mask in (1, 0):
        got = S.audit(G, order_mask=mask)
        want = oracle.synthesis_audit(geo, Q, order_mask=None if mask == 0 else mask)
        assert got["zero_columns"] == want["zero_columns"], (mask, len(got["zero_columns"]), len(want["zero_columns"]))
        s_w = want["sigma"]
        keep = s_w >= 1e-3 * s_w[0]          # FP32 responses: sigma_i good to ~1e-7 sigma_1 / sigma_i
        err = np.max(np.abs(got["sigma"][:keep.sum()] - s_w[keep]) / s_w[keep])
        assert err < 1e-4, (mask, int(keep.sum()), err)
    if temporal == "hats":
        assert len(S.audit(G, order_mask=1)["zero_columns"]) > 0


def test_s224_audit_on_the_kerr_128_workload(gpu_lib):
    """S_224 on the 128^2 workload: direct and resolved arms.  Zero columns against the oracle's
    responses to every column of Q; the singular values >= 1e-3 sigma_1 against the FP64 Gram of those
    responses."""
    rtt = gpu_lib
    geo = synth.geometry_for("cfg2")
    G = rtt.Geometry(geo)
    say("case S224 cfg2")
    for temporal in ("dct", "hats"):
        S = rtt.Synthesis(G, 0, temporal=temporal)
        Q = oracle.synthesis_matrix(geo.grid, temporal=temporal)
        m0 = geo.maps[0].n_rays * geo.grid.n_frames
        Ys = [oracle.forward(geo, Q[:, b:b + 32].T) for b in range(0, S.d, 32)]
        Y = np.concatenate(Ys, axis=0)                       # [d][rows], FP64
        for mask, rows in ((1, slice(0, m0)), (0, slice(0, Y.shape[1]))):
            got = S.audit(G, order_mask=mask)
            Ym = Y[:, rows]
            zero = [int(c) for c in range(S.d) if not np.any(Ym[c])]
            assert got["zero_columns"] == zero, (temporal, mask)
            Gm = Ym @ Ym.T
            s_w = np.sqrt(np.maximum(np.linalg.eigvalsh(Gm)[::-1], 0.0))
            say(temporal, mask, "zero", len(zero), "rank", got["rank"], "sigma1", got["sigma"][0])
            keep = int(np.sum(s_w >= 1e-3 * s_w[0]))
            err = np.max(np.abs(got["sigma"][:keep] - s_w[:keep]) / s_w[:keep])
            say(temporal, mask, "sigma >= 1e-3 sigma1:", keep, "max rel err", err)
            assert err < 1e-4, (temporal, mask, keep, err)


def test_age_fisher_matches_oracle(gpu_lib):
    """M(a) of eq. (14) against the oracle on a small geometry (direct and resolved rows), and the
    flat-probe information as its quadratic form (the radial B-splines sum to one on the nodes)."""
    rtt = gpu_lib
    geo = tiny_geometry(seed=9, rays=(14, 8, 5), n_frames=5)
    G = rtt.Geometry(geo)
    S = rtt.Synthesis(G, 0)
    ages = np.array([0.0, 7.0, 20.0, 33.5])
    say("case age fisher")
    for mask in (1, 0):
        M = S.age_fisher(G, ages, h=3.0, order_mask=mask)
        W = oracle.age_fisher(geo, ages, h=3.0, order_mask=None if mask == 0 else mask)
        for i in range(ages.size):
            assert rel(M[i], W[i]) < 1e-5, (mask, i, rel(M[i], W[i]))
    nl = oracle.localized_probe_norms(geo.grid, 4, 3, 3.0)
    w = np.zeros(28)
    for a in range(4):
        w[a * 7] = nl[a * 7] / oracle.probe_norm(geo.grid, 3.0)
    E = rtt.age_information(G, ages, h=3.0)[:, 0, :3].sum(axis=1)
    assert rel(np.einsum("l,alm,m->a", w, S.age_fisher(G, ages), w), E) < 1e-5


def test_age_fisher_on_the_kerr_128_workload(gpu_lib):
    rtt = gpu_lib
    geo = synth.geometry_for("cfg2")
    G = rtt.Geometry(geo)
    S = rtt.Synthesis(G, 0)
    ages = np.array([0.0, 40.0])
    say("case age fisher cfg2")
    M = S.age_fisher(G, np.arange(0.0, 256.0, 4.0), h=3.0, order_mask=0)
    W = oracle.age_fisher(geo, ages, h=3.0)
    for i, a in enumerate(ages):
        assert rel(M[int(a) // 4], W[i]) < 1e-5
