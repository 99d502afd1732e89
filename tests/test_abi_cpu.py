"""Host-side checks of the C ABI that need no GPU: exports and input validation."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2609_05528_amd as rtt
import synth
from tinygeo import tiny_geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "rtt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = rtt.require_native()
    names = declared_functions()
    assert {"geometry_load", "op_apply", "op_apply_adjoint", "rsvd", "tsvd_solve", "ridge_solve"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(rtt.EXPORTED) == set(names)


def _load_err(geo, **kw):
    with pytest.raises(rtt.RttError) as ei:
        rtt.Geometry(geo, **kw)
    return ei.value


def test_validation_rejects_bad_inputs_before_device_work():
    geo = tiny_geometry(seed=3, rays=(6, 3))
    g = geo.grid

    def with_grid(**kw):
        return synth.Geometry(grid=synth.Grid(**{**g.as_dict(), **kw}), maps=geo.maps)

    for kw, frag in [(dict(n_r=1), "n_r"), (dict(n_hat=1), "n_hat"), (dict(n_frames=0), "n_frames"),
                     (dict(r_out=5.0), "r_in < r_out"), (dict(dt_src=0.0), "dt_src"),
                     (dict(dt_obs=4.0 * math.pi), "rational")]:
        e = _load_err(with_grid(**kw))
        assert e.code == rtt.RTT_EINVAL and frag in str(e), (kw, str(e))
    bad = [synth.RayMap(r=m.r.copy(), phi=m.phi, delay=m.delay, weight=m.weight) for m in geo.maps]
    bad[1].r[2] = 25.0
    e = _load_err(synth.Geometry(grid=g, maps=bad))
    assert e.code == rtt.RTT_EINVAL and "outside" in str(e) and "order 1 ray 2" in str(e)
    bad[1].r[2] = np.nan
    e = _load_err(synth.Geometry(grid=g, maps=bad))
    assert e.code == rtt.RTT_EINVAL and "non-finite" in str(e)


def test_drop_invalid_passes_validation():
    geo = tiny_geometry(seed=3, rays=(6, 3))
    bad = [synth.RayMap(r=m.r.copy(), phi=m.phi, delay=m.delay, weight=m.weight) for m in geo.maps]
    bad[0].r[0] = 30.0
    try:
        rtt.Geometry(synth.Geometry(grid=geo.grid, maps=bad), drop_invalid=True)
    except rtt.RttError as e:           # without a GPU the upload is what fails
        assert e.code in (rtt.RTT_EDEVICE, rtt.RTT_ENOMEM)


def test_null_arguments_are_errors():
    lib = rtt.require_native()
    assert lib.geometry_load(None, None, 1, None, None) == rtt.RTT_EINVAL
    assert lib.op_apply(None, None, None, 1, 0, None) == rtt.RTT_EINVAL
    assert lib.op_apply_adjoint(None, None, None, 1, 0, None) == rtt.RTT_EINVAL
    assert b"invalid geometry handle" in lib.last_error()
    assert lib.geometry_free(None) == rtt.RTT_OK
    info = rtt.rtt_solve_info()
    assert lib.ridge_solve(None, None, 1, 1e-3, None, None, ctypes.byref(info), None) == rtt.RTT_EINVAL
    h = ctypes.c_void_p()
    assert lib.mixer_create(None, 0, None, ctypes.byref(h)) == rtt.RTT_EINVAL and not h.value
    assert b"invalid geometry handle" in lib.last_error()
    assert lib.mixer_create(None, 0, None, None) == rtt.RTT_EINVAL
    assert lib.mix_apply(None, None, None, 1, None) == rtt.RTT_EINVAL
    assert lib.mix_adjoint(None, None, None, 1, None) == rtt.RTT_EINVAL
    assert lib.mix_covariance(None, None, None, None) == rtt.RTT_EINVAL
    assert b"invalid mixer handle" in lib.last_error()
    assert lib.mixer_free(None) == rtt.RTT_OK
    d = ctypes.c_double()
    dp = ctypes.byref(d)
    assert lib.reference_response(None, dp, None) == rtt.RTT_EINVAL
    assert lib.age_information(None, dp, 1, 3.0, None, None, dp, None) == rtt.RTT_EINVAL
    assert lib.age_window(None, 0, 0, 3.0, 0.999, dp, dp, dp) == rtt.RTT_EINVAL
    assert lib.age_window_error(None, None, None, 1, dp, 1, 2.0, 0.0, dp, None) == rtt.RTT_EINVAL
    assert b"invalid geometry handle" in lib.last_error()
    assert lib.tsvd_project(None, None, None, 1, 1, 0.0, None, None) == rtt.RTT_EINVAL
    assert lib.noise_add(None, 5, 1, 1.0, None) == rtt.RTT_EINVAL
    assert lib.noise_add(None, 0, 1, 1.0, None) == rtt.RTT_OK
    h = ctypes.c_void_p()
    assert lib.synthesis_create(None, 0, None, ctypes.byref(h)) == rtt.RTT_EINVAL and not h.value
    assert lib.synth_expand(None, None, None, 1, None) == rtt.RTT_EINVAL
    assert lib.synth_project(None, None, None, 1, None) == rtt.RTT_EINVAL
    assert lib.synthesis_audit(None, None, 0, None, None, None) == rtt.RTT_EINVAL
    assert lib.age_fisher(None, None, dp, 1, 3.0, 0, dp, None) == rtt.RTT_EINVAL
    assert lib.synthesis_free(None) == rtt.RTT_OK


def test_synthetic_workload_shapes():
    """The synthetic geometries have the ray counts stated for the workloads."""
    assert synth.geometry_for("cfg1").rays_per_order == [2944]
    assert synth.geometry_for("cfg2").rays_per_order == [11732, 184, 164]
    assert synth.geometry_for("cfg3").rays_per_order == [46840]
    g5 = synth.geometry_for("cfg5")
    assert g5.rays_per_order == [187348, 2720, 2696] and g5.n_rows == 98695168
    gs = synth.batch_geometries()
    assert len(gs) == 12 and sum(g.n_rays for g in gs) == 295508
    assert [g.grid.s0 for g in (synth.geometry_for(c) for c in ("cfg1", "cfg2", "cfg5"))] == [-32.0, -72.0, -76.0]


def test_bench_script_parses_and_refuses_several_gpus():
    """bench.py is a driver contract: it must at least compile, and a request for more than one
    GPU ends with a message (before any device work)."""
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, "bench.py")).read()
    compile(src, "bench.py", "exec")
    r = subprocess.run([_sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_age_reach_matches_the_oracle_on_random_masks():
    """The host-only threshold statistics of the library against the oracle's plain loops."""
    import oracle
    rng = np.random.default_rng(17)
    ages = np.arange(0.0, 256.0, 4.0)
    for trial in range(200):
        info = rng.exponential(1.0, ages.size) * rng.choice([0.3, 1.0, 3.0])
        lo, hi = sorted(rng.uniform(-20, 270, 2))
        boundary = rng.uniform(-10, 260) if trial % 7 else math.nan
        got = rtt.age_reach(ages, info, rho=1.0, a_min=lo, a_max=hi, boundary=boundary)
        sup = [(lo <= a <= hi) for a in ages]
        want = oracle.reach(ages, info, rho=1.0, supported=sup, boundary=None if math.isnan(boundary) else boundary)
        assert list(got["mask"]) == want["mask"]
        assert got["t_reach"] == want["t_reach"] and got["anchor"] == want["anchor"]
        assert got["l_anchor"] == want["l_anchor"] and got["longest"] == want["longest"]
        if want["j_old"] is None:
            assert got["j_old"] is None
        else:
            assert abs(got["j_old"] - want["j_old"]) <= 1e-12 * max(1.0, want["j_old"])
    with pytest.raises(rtt.RttError, match="equally spaced"):
        rtt.age_reach([0.0, 4.0, 9.0], [1.0, 1.0, 1.0])


def test_pairing_destroyed_control_keeps_delay_marginals():
    geo = tiny_geometry(seed=5, rays=(30, 12, 9))
    ctl = synth.pairing_destroyed(geo, seed=1)
    for m, c in zip(geo.maps, ctl.maps):
        assert np.array_equal(np.sort(m.delay), np.sort(c.delay))
        assert np.array_equal(m.r, c.r) and np.array_equal(m.weight, c.weight) and np.array_equal(m.pixel, c.pixel)
    assert not np.array_equal(geo.maps[0].delay, ctl.maps[0].delay)
    assert np.array_equal(synth.pairing_destroyed(geo, seed=1).maps[1].delay, ctl.maps[1].delay)


def test_spatial_only_and_delay_only_arms():
    geo = tiny_geometry(seed=6, rays=(30, 12, 9))
    sp = synth.spatial_only(geo)
    for n, (m, s) in enumerate(zip(geo.maps, sp.maps)):
        assert np.array_equal(m.r, s.r) and np.array_equal(m.phi, s.phi) and np.array_equal(m.weight, s.weight)
        assert abs(np.median(s.delay) - np.median(geo.maps[0].delay)) < 1e-9
        assert np.allclose(np.diff(np.sort(s.delay)), np.diff(np.sort(m.delay)))
    do = synth.delay_only(geo, seed=2)
    r0 = set(geo.maps[0].r.tolist())
    for m, d in zip(geo.maps[1:], do.maps[1:]):
        assert np.array_equal(m.delay, d.delay) and np.array_equal(m.weight, d.weight)
        assert set(d.r.tolist()) <= r0
    assert np.array_equal(do.maps[0].r, geo.maps[0].r)
