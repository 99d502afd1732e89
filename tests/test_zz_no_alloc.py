"""mix_apply_noalloc: the order mixer of eq. (4) through the entry point that allocates no device
memory (partial rows in the library's fixed per-GPU scratch array).  It must give the bits of
mix_apply, the entry point whose kernels it shares, on consecutive calls whose sizes shrink (the
scratch keeps the previous call's contents), and reject a call that needs more scratch than the
array holds before launching anything."""
import re
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


def rand_block(nvec, n, seed):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    y = torch.empty((nvec, n), device="cuda")
    y.normal_(generator=gen)
    return y


def test_noalloc_mixer_equals_mix_apply_on_shrinking_calls(gpu_lib):
    import torch
    rtt = gpu_lib
    geo = synth.geometry_for("cfg2")
    G = rtt.Geometry(geo)
    pix = [np.asarray(m.pixel, dtype=np.int64) for m in geo.maps]
    tf = rtt.Mixer(G, "total_flux")
    un = rtt.Mixer(G, "unresolved", pix)
    small = tiny_geometry(seed=71, rays=(150, 40, 30), n_frames=13)
    Gs = rtt.Geometry(small)
    tfs = rtt.Mixer(Gs, "total_flux")
    # (mixer, vectors, seed): the first call fills most of the scratch, the later ones use less of it
    calls = [(tf, 120, 1), (tf, 5, 2), (tfs, 3, 3), (un, 9, 4), (tf, 1, 5)]
    for i, (M, nvec, seed) in enumerate(calls):
        say("call", i, "rows", M.n_src_rows, "->", M.n_rows, "vectors", nvec)
        Y = rand_block(nvec, M.n_src_rows, seed)
        want = rtt.mix_apply(M, Y)
        got = torch.full_like(want, float("nan"))
        rtt.mix_apply_noalloc(M, Y, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), i
    # and against the oracle's dense L on one vector of the total flux
    Y = rand_block(2, tf.n_src_rows, 6)
    got = torch.empty((2, tf.n_rows), device="cuda")
    rtt.mix_apply_noalloc(tf, Y, got)
    ref = oracle.mix(geo, Y[1].double().cpu().numpy(), "total_flux")
    err = float(np.linalg.norm(got[1].double().cpu().numpy() - ref) / np.linalg.norm(ref))
    assert err <= 1e-5, err


def test_noalloc_mixer_rejects_calls_beyond_its_scratch(gpu_lib):
    import torch
    rtt = gpu_lib
    geo = synth.geometry_for("cfg2")
    G = rtt.Geometry(geo)
    tf = rtt.Mixer(G, "total_flux")
    # one vector's partial rows: chunks of 64 rays, frame rows padded to a multiple of 4 floats
    per_vec = -(-geo.n_rays // 64) * (-(-geo.grid.n_frames // 4) * 4) * 4
    est = (16 << 20) // per_vec
    Y = torch.zeros((400, tf.n_src_rows), device="cuda")
    D = torch.zeros((400, tf.n_rows), device="cuda")
    with pytest.raises(rtt.RttError) as ei:
        rtt.mix_apply_noalloc(tf, Y, D)
    msg = str(ei.value)
    assert ei.value.code == rtt.RTT_EINVAL and "scratch" in msg
    limit = int(re.search(r"at most (\d+) vectors", msg).group(1))
    say("vector limit", limit, "estimated", est)
    assert abs(limit - est) <= 2
    with pytest.raises(rtt.RttError):
        rtt.mix_apply_noalloc(tf, Y[:limit + 1], D[:limit + 1])
    # at the limit it runs and matches mix_apply
    rtt.mix_apply_noalloc(tf, Y[:limit], D[:limit])
    assert torch.equal(D[:limit], rtt.mix_apply(tf, Y[:limit]))
