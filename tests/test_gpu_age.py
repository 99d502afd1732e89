"""Age-localised probe information (Sec. 3.3, 4.4) on the GPU against the FP64 oracle.

age_information per (age, geometry, order) and through the two order mixers, s_ref (eq. (17)),
the supported-age window (eq. (13)) and the direct throughput boundary, on a ragged batch of
small geometries and on the 128^2 x 128-frame Kerr workload.  FP32 responses reduced in FP64:
1e-5 relative is the bar.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tinygeo import tiny_geometry

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def batch():
    return [tiny_geometry(seed=91, rays=(40, 12, 7), n_frames=6, delay_hi=30.0),
            tiny_geometry(seed=92, rays=(25, 0, 9), n_frames=9, n_phi=8, delay_hi=20.0),
            tiny_geometry(seed=93, rays=(60, 30), n_frames=8, n_r=5, delay_hi=40.0)]


def test_age_information_per_order_and_arm_matches_oracle(gpu_lib):
    rtt = gpu_lib
    geos = batch()
    G = rtt.Geometry(geos)
    ages = np.arange(-8.0, 80.0, 4.0) + 0.37
    say("case age information per order", len(ages))
    E = rtt.age_information(G, ages, h=3.0)
    assert E.shape == (ages.size, 3, 8)
    for g, geo in enumerate(geos):
        no = geo.grid.n_orders
        assert np.all(E[:, g, no:] == 0.0)
        d = oracle.age_energy(geo, ages, arm="direct")
        r = oracle.age_energy(geo, ages, arm="resolved")
        assert relerr(E[:, g, 0], d) < TOL, (g, relerr(E[:, g, 0], d))
        assert relerr(E[:, g, :no].sum(axis=1), r) < TOL, (g, relerr(E[:, g, :no].sum(axis=1), r))
    # through the mixers, with non-uniform per-datum variances
    var = np.random.default_rng(94).uniform(0.5, 2.0, G.n_rows)
    pix = [np.asarray(m.pixel, dtype=np.int64) for geo in geos for m in geo.maps]
    for kind in ("unresolved", "total_flux"):
        say("case age information mixer", kind)
        M = rtt.Mixer(G, kind, pix if kind == "unresolved" else None)
        Em = rtt.age_information(G, ages, h=3.0, mixer=M, var=to_dev(var))
        E1 = rtt.age_information(G, ages, h=3.0, mixer=M)
        assert Em.shape == (ages.size, 3)
        for g, geo in enumerate(geos):
            m = G.members[g]
            vg = var[m["row_offset"]:m["row_offset"] + m["n_rows"]]
            want = oracle.age_energy(geo, ages, arm=kind, var=vg)
            assert relerr(Em[:, g], want) < TOL, (kind, g, relerr(Em[:, g], want))
            want1 = oracle.age_energy(geo, ages, arm=kind)
            assert relerr(E1[:, g], want1) < TOL, (kind, g)


def test_reference_response_window_and_boundary_match_oracle(gpu_lib):
    rtt = gpu_lib
    geos = batch()
    G = rtt.Geometry(geos)
    say("case s_ref and windows")
    sref = rtt.reference_response(G)
    ages = np.arange(-40.0, 120.0, 4.0) + 0.5
    for g, geo in enumerate(geos):
        want = oracle.s_ref(geo)
        assert abs(sref[g] - want) <= 1e-6 * want, (g, sref[g], want)
        for mask in (1, 0):
            a0, a1, b = rtt.age_window(G, g, order_mask=mask, h=3.0, q=0.999)
            sup = (ages >= a0) & (ages <= a1)
            want_sup = oracle.supported_ages(geo, ages, 3.0, order_mask=None if mask == 0 else mask)
            assert np.array_equal(sup, want_sup), (g, mask)
        for q in (0.999, 0.5, 0.1):
            b = rtt.age_window(G, g, h=3.0, q=q)[2]
            assert abs(b - oracle.throughput_age_boundary(geo, q)) < 1e-9, (g, q)


def test_age_statistics_on_the_kerr_128_workload(gpu_lib):
    """Every age of the 0-252M grid for the direct and resolved arms, and the total flux; reach
    statistics at SNR0 = 100 through the library against the oracle's loops on the same numbers."""
    rtt = gpu_lib
    geo = synth.geometry_for("cfg2")
    G = rtt.Geometry(geo)
    ages = np.arange(0.0, 256.0, 4.0)
    say("case age cfg2")
    E = rtt.age_information(G, ages, h=3.0)
    # 300 centres on a 0.85M grid take three passes of the library's age chunks: same values
    fine = np.arange(300) * 0.85
    Ef = rtt.age_information(G, fine, h=3.0)
    Xf = oracle.age_probes(geo.grid, fine[[0, 150, 299]], 3.0)
    Yf = oracle.forward(geo, Xf)
    assert relerr(Ef[[0, 150, 299], 0, :3].sum(axis=1), np.einsum("ar,ar->a", Yf, Yf)) < TOL
    sample = [0, 9, 21, 40, 63]
    X = oracle.age_probes(geo.grid, ages[sample], 3.0)
    Y = oracle.forward(geo, X)
    m0 = geo.maps[0].n_rays * geo.grid.n_frames
    want_d = np.einsum("ar,ar->a", Y[:, :m0], Y[:, :m0])
    want_r = np.einsum("ar,ar->a", Y, Y)
    assert relerr(E[sample, 0, 0], want_d) < TOL
    assert relerr(E[sample, 0, :3].sum(axis=1), want_r) < TOL
    Mt = rtt.Mixer(G, "total_flux")
    Et = rtt.age_information(G, ages[sample], h=3.0, mixer=Mt)
    tf = oracle.mix(geo, Y, "total_flux")
    want_t = np.sum(tf * tf, axis=1) / geo.n_rays     # C_L = n_rays I for unit variances
    assert relerr(Et[:, 0], want_t) < TOL
    sref = rtt.reference_response(G)[0]
    assert abs(sref - oracle.s_ref(geo)) <= 1e-6 * sref
    a0, a1, bnd = rtt.age_window(G, 0, order_mask=1, h=3.0, q=0.999)
    for arm, e in (("direct", E[:, 0, 0]), ("resolved", E[:, 0, :3].sum(axis=1))):
        info = 100.0 ** 2 * e / sref ** 2
        got = rtt.age_reach(ages, info, 1.0, a0, a1, bnd)
        want = oracle.reach(ages, info, 1.0, supported=list((ages >= a0) & (ages <= a1)), boundary=bnd)
        say(arm, got["t_reach"], got["l_anchor"], got["j_old"])
        assert got["t_reach"] == want["t_reach"] and got["l_anchor"] == want["l_anchor"]
        assert abs(got["j_old"] - want["j_old"]) <= 1e-12 * max(1.0, want["j_old"])


@pytest.mark.parametrize("arm", ["pairing_destroyed", "spatial_only", "delay_only"])
def test_age_information_of_the_mechanism_arms(gpu_lib, arm):
    """The mechanism arms of Sec. 6.4 as input transforms through the same path: every order's
    energy against the oracle run on the same transformed maps."""
    rtt = gpu_lib
    base = tiny_geometry(seed=95, rays=(50, 20, 10), n_frames=7, delay_hi=30.0)
    geo = {"pairing_destroyed": lambda: synth.pairing_destroyed(base, seed=3),
           "spatial_only": lambda: synth.spatial_only(base),
           "delay_only": lambda: synth.delay_only(base, seed=4)}[arm]()
    G = rtt.Geometry(geo)
    ages = np.arange(0.0, 64.0, 4.0) + 0.21
    say("case mechanism arm", arm)
    E = rtt.age_information(G, ages, h=3.0)
    assert relerr(E[:, 0, :3].sum(axis=1), oracle.age_energy(geo, ages, arm="resolved")) < TOL
    assert relerr(E[:, 0, 0], oracle.age_energy(geo, ages, arm="direct")) < TOL
