#!/usr/bin/env python3
"""Benchmark of the retarded-time operator pair A / A^T on one MI355X.

Workload (default): the Kerr a=0.5, i=50 deg geometry with orders n=0,1,2 on a
128^2 screen, 128 frames at 4M cadence, 64x64 polar cells x 96 hats, and a
block of l = k + p = 256 + 8 = 264 coefficient vectors (the randomized-SVD
block).  One step = one block application of A (264 vectors) followed by one
block application of A^T (264 vectors): 528 applies.  Inputs are synthetic,
seeded, and resident in HBM before the timed region starts.

Printed: one JSON line with the throughput (applies/s), the roofline of the
dominant kernel (algorithmic bytes / measured kernel time vs the 8 TB/s HBM
peak), the plain per-vector throughput beside the batched one, parity against
the FP64 oracle on sampled vectors, and the oracle's own CPU throughput on
one full step of the same work.  Extra sections: the 512^2 x 512-frame
geometry one vector at a time, the rSVD wall time, and the batch of 12
geometries x 60 histories (batched vs per-instance A/A^T and autograd, the
rSVD of every geometry in one call, and one captured graph of A, A^T, TSVD
and a fixed-count ridge solve of every (geometry, history) pair).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A+A^T applies/sec and HBM GB/s; batched vs plain at 1e-5 rel err"
HBM_PEAK_GBPS = 8000.0
RAY_RECORD_BYTES = 32
KERNEL_SOURCE = os.path.join(ROOT, "paper_2609_05528_amd", "csrc", "operator.hip")
# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE on this workload
# (FETCH_SIZE scaled by 2.0, the factor a 2 GiB plain copy reads; WRITE_SIZE by 1.0), valid only
# for the kernel source digest and variant they were taken on (see profiles/).
MEASURED_TRAFFIC = {
    "op_apply_adjoint": [{"bytes": 2050789488, "digest": "2475b31d9f92872d", "nvec": 264, "variant": "visitp2v"}],
    "op_apply": [{"bytes": 2105012096, "digest": "2475b31d9f92872d", "nvec": 264, "variant": "abs4"},
                 {"bytes": 2099961088, "digest": "2475b31d9f92872d", "nvec": 264, "variant": "abs8"}],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n_rows, n_cols, n_rays, n_cells, n_orders, nvec, adjoint):
    """Bytes the method must move per launch: y (write or read) + x + ray tables (+ CSR)."""
    b = 4 * nvec * (n_rows + n_cols) + RAY_RECORD_BYTES * n_rays
    if adjoint:
        b += 4 * (n_cells + 1)
    return b


def source_digest():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def time_pair(torch, rtt, G, X, Y, XT, reps=10):
    """Average kernel time (ms) of op_apply and of op_apply_adjoint, each over `reps`
    back-to-back launches bracketed by HIP events on the current stream."""
    rtt.op_apply(G, X, Y)
    rtt.op_apply_adjoint(G, Y, XT)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        rtt.op_apply(G, X, Y)
    e[1].record()
    for _ in range(reps):
        rtt.op_apply_adjoint(G, Y, XT)
    e[2].record()
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps


def mixer_section(torch, rtt, oracle, geo, G, Y, reps=10):
    """Order mixers of eq. (4) on the benchmark block Y = A X: the unresolved image (screen pixels)
    and the total flux, forward and transpose, each timed over `reps` launches with HIP events.
    Algorithmic bytes per launch: read the source rows and write the mixed rows (or the reverse),
    4 * nvec * (n_src_rows + n_rows); the gather tables (8-32 B per ray) are left out."""
    nvec = Y.shape[0]
    pix = [np.asarray(m.pixel, dtype=np.int64) for m in geo.maps]
    out = {}
    for kind in ("unresolved", "total_flux"):
        M = rtt.Mixer(G, kind, pix if kind == "unresolved" else None)
        D = rtt.mix_apply(M, Y)
        YT = rtt.mix_adjoint(M, D)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            rtt.mix_apply(M, Y, D)
        e[1].record()
        for _ in range(reps):
            rtt.mix_adjoint(M, D, YT)
        e[2].record()
        torch.cuda.synchronize()
        ms_f, ms_t = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
        b = 4 * nvec * (M.n_src_rows + M.n_rows)
        out[kind] = {"mixed_rows": M.n_rows, "mix_apply": {"ms": ms_f, "GBps": b / (ms_f * 1e-3) / 1e9,
                                                             "frac": b / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBPS},
                     "mix_adjoint": {"ms": ms_t, "GBps": b / (ms_t * 1e-3) / 1e9,
                                     "frac": b / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBPS}, "bytes": b}
        if kind == "total_flux":
            ref = oracle.mix(geo, Y[0].double().cpu().numpy(), kind)
            got = D[0].double().cpu().numpy()
            out[kind]["parity_rel_err_vector0"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        log("mixer %s: apply %.3f ms (%.0f GB/s), adjoint %.3f ms (%.0f GB/s)" % (
            kind, ms_f, out[kind]["mix_apply"]["GBps"], ms_t, out[kind]["mix_adjoint"]["GBps"]))
        del D, YT, M
        torch.cuda.empty_cache()
    return out


def age_section(torch, rtt, geos, G, snr0=100.0, rho=1.0, h=3.0):
    """Age-probe information over the 0-252M grid (4M steps) for every geometry of G: the direct,
    resolved, unresolved and total-flux arms (Sec. 3.3, 4.4, 6.4), each arm one library call timed
    end to end, then the reach statistics at SNR0 with s_ref of each geometry (eq. (17)-(18))."""
    ages = np.arange(0.0, 256.0, 4.0)
    pix = [np.asarray(m.pixel, dtype=np.int64) for geo in geos for m in geo.maps]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sref = rtt.reference_response(G)
    t_sref = time.perf_counter() - t0
    t0 = time.perf_counter()
    E = rtt.age_information(G, ages, h=h)
    t_orders = time.perf_counter() - t0
    arms = {"direct": E[:, :, 0], "resolved": E.sum(axis=2)}
    t_mix = {}
    for kind in ("unresolved", "total_flux"):
        M = rtt.Mixer(G, kind, pix if kind == "unresolved" else None)
        t0 = time.perf_counter()
        arms[kind] = rtt.age_information(G, ages, h=h, mixer=M)
        t_mix[kind] = time.perf_counter() - t0
        del M
    # mechanism arms of Sec. 6.4 as input transforms, with the noise density of the original geometry:
    # pairing destroyed (delays permuted within each order), spatial only (higher orders shifted to the
    # direct order's median delay), delay only (higher orders at direct-order source positions)
    import synth
    for arm, tf in (("pairing_destroyed", lambda i, geo: synth.pairing_destroyed(geo, seed=600 + i)),
                    ("spatial_only", lambda i, geo: synth.spatial_only(geo)),
                    ("delay_only", lambda i, geo: synth.delay_only(geo, seed=700 + i))):
        Gc = rtt.Geometry([tf(i, geo) for i, geo in enumerate(geos)])
        t0 = time.perf_counter()
        arms[arm] = rtt.age_information(Gc, ages, h=h).sum(axis=2)
        t_mix[arm] = time.perf_counter() - t0
        del Gc
    stats = {}
    for arm, e in arms.items():
        per = []
        for g in range(G.n_geometries):
            a0, a1, bnd = rtt.age_window(G, g, order_mask=1 if arm == "direct" else 0, h=h, q=0.999)
            r = rtt.age_reach(ages, snr0 ** 2 * e[:, g] / sref[g] ** 2, rho, a0, a1, bnd)
            per.append(r)

        def med(key):
            v = [r[key] for r in per if r[key] is not None]
            return float(np.median(v)) if v else None

        stats[arm] = {"median_t_reach": med("t_reach"), "median_l_anchor": med("l_anchor"),
                      "median_j_old": med("j_old")}
        if G.n_geometries == 1:
            stats[arm].update({"t_reach": per[0]["t_reach"], "l_anchor": per[0]["l_anchor"],
                               "j_old": per[0]["j_old"], "anchor_age": None if per[0]["anchor"] is None
                               else float(ages[per[0]["anchor"]])})
    out = {"ages": "0-252M step 4M (64 centres), h = %gM, SNR0 = %g, rho = %g" % (h, snr0, rho),
           "seconds": {"s_ref": t_sref, "orders": t_orders, **t_mix},
           "probe_applies_per_s": ages.size * G.n_geometries / t_orders, "arms": stats}
    log("age information: orders %.3f s, unresolved %.3f s, total flux %.3f s; %s" % (
        t_orders, t_mix["unresolved"], t_mix["total_flux"],
        {a: (v["median_l_anchor"], v["median_j_old"]) for a, v in stats.items()}))
    return out


def estimator_section(torch, rtt, synth, geo, G, snr0=100.0, nh=16, lam=1e-3):
    """Held-out-style recovery on the benchmark geometry: nh Gaussian-blob histories, data
    y = A x + seeded noise at sigma_Omega = s_ref / SNR0 (eq. (18)); the ridge estimate and its
    derivative with respect to the data (forward CG + one more CG), the TSVD estimate and its
    derivative from the rSVD factors, and the age-window error E(a) of eq. (32) over 0-252M."""
    from paper_2609_05528_amd.autograd import ridge_estimate, tsvd_estimate
    dev = torch.device("cuda:0")
    X = torch.from_numpy(synth.blob_histories(geo.grid, nh, dtype=np.float32)).to(dev)
    sref = float(rtt.reference_response(G)[0])
    Y = rtt.op_apply(G, X)
    rtt.noise_add(Y, seed=4242, sigma=sref / snr0)
    ages = np.arange(0.0, 256.0, 4.0)
    out = {"histories": nh, "lambda": lam, "sigma_omega": sref / snr0}
    y = Y.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xr = ridge_estimate(y, G, lam, tol=1e-4, maxit=400)
    loss = 0.5 * ((xr - X) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    out["ridge_forward_backward_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    E = rtt.age_window_error(G, xr.detach(), X, ages, half_width=2.0, eta=1e-6)
    out["age_window_error_s"] = time.perf_counter() - t0
    out["ridge_median_E"] = {str(int(a)): float(np.median(E[:, 0, i])) for i, a in enumerate(ages) if a in (0, 20, 40, 60)}
    sv = rtt.rsvd(G, k=256, p=8, q=2, seed=2001)
    y2 = Y.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xt = tsvd_estimate(y2, G, sv, t=0, sigma_min=sref / snr0)
    (0.5 * ((xt - X) ** 2).sum()).backward()
    torch.cuda.synchronize()
    out["tsvd_forward_backward_s"] = time.perf_counter() - t0
    Et = rtt.age_window_error(G, xt.detach(), X, ages, half_width=2.0, eta=1e-6)
    out["tsvd_median_E"] = {str(int(a)): float(np.median(Et[:, 0, i])) for i, a in enumerate(ages) if a in (0, 20, 40, 60)}
    log("estimators: ridge fwd+bwd %.3f s, tsvd fwd+bwd %.3f s, E(a) %.4f s" % (
        out["ridge_forward_backward_s"], out["tsvd_forward_backward_s"], out["age_window_error_s"]))
    del sv, y, y2, xr, xt, Y, X
    torch.cuda.empty_cache()
    return out


def synthesis_section(torch, rtt, G, snr0=100.0):
    """Table-4-style audit of the benchmark geometry (Sec. 3.2, Sec. 7): A Q_d for S_224 with global
    DCT-II and with compact temporal functions, direct and resolved arms: exactly zero columns,
    numerical rank (1e-6 sigma_1) and operational rank at SNR0 (sigma >= s_ref / SNR0, eq. (31));
    and the throughput of A^(d) = A Q_d on a block of 264 coefficient vectors."""
    sref = float(rtt.reference_response(G)[0])
    out = {"snr0": snr0}
    for temporal in ("dct", "hats"):
        S = rtt.Synthesis(G, 0, temporal=temporal)
        for arm, mask in (("direct", 1), ("resolved", 0)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a = S.audit(G, order_mask=mask)
            dt = time.perf_counter() - t0
            out["%s_%s" % (temporal, arm)] = {
                "d": S.d, "zero_columns": len(a["zero_columns"]), "rank": a["rank"],
                "operational_rank": int(np.sum(a["sigma"] >= sref / snr0)), "sigma_1": float(a["sigma"][0]),
                "audit_s": dt}
        if temporal == "dct":
            C = torch.randn(264, S.d, device="cuda")
            X = torch.empty(264, S.n_cols, device="cuda")
            Y = torch.empty(264, G.n_rows, device="cuda")
            S.expand(C, X)
            rtt.op_apply(G, X, Y)
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            for _ in range(5):
                S.expand(C, X)
            e[1].record()
            for _ in range(5):
                rtt.op_apply(G, X, Y)
            e[2].record()
            torch.cuda.synchronize()
            ms_q, ms_a = e[0].elapsed_time(e[1]) / 5, e[1].elapsed_time(e[2]) / 5
            out["expand_ms"] = ms_q
            out["a_of_q_applies_per_s"] = 264 / ((ms_q + ms_a) * 1e-3)
            del C, X, Y
        del S
        torch.cuda.empty_cache()
    # localised probe class of eq. (14): M(a) over the 64-centre grid; localised directional reach =
    # deepest age at which some normalised direction clears threshold (SNR0^2 M_ll / s_ref^2 >= 1)
    S = rtt.Synthesis(G, 0)
    ages = np.arange(0.0, 256.0, 4.0)
    for arm, mask in (("direct", 1), ("resolved", 0)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = S.age_fisher(G, ages, h=3.0, order_mask=mask)
        dt = time.perf_counter() - t0
        diag = snr0 ** 2 * np.einsum("all->al", M) / sref ** 2
        passing = ages[np.any(diag >= 1.0, axis=1)]
        out["fisher_%s" % arm] = {"seconds": dt, "localized_reach": float(passing.max()) if passing.size else None}
    del S
    log("synthesis audit: %s" % {k: (v["zero_columns"], v["rank"], v["operational_rank"])
                                  for k, v in out.items() if isinstance(v, dict) and "rank" in v})
    return out


def calibrate(torch, dev, gib=2):
    """Streaming bandwidth of torch's plain copy and fill kernels on 2 GiB (HBM reference)."""
    n = gib * (1 << 30) // 4
    a = torch.empty(n, dtype=torch.float32, device=dev)
    b = torch.empty(n, dtype=torch.float32, device=dev)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 5
    e[0].record()
    for _ in range(reps):
        b.copy_(a)
    e[1].record()
    for _ in range(reps):
        a.fill_(2.0)
    e[2].record()
    torch.cuda.synchronize()
    t_copy = e[0].elapsed_time(e[1]) / reps * 1e-3
    t_fill = e[1].elapsed_time(e[2]) / reps * 1e-3
    out = {"copy_gbps": 2 * 4 * n / t_copy / 1e9, "fill_gbps": 4 * n / t_fill / 1e9, "bytes": 4 * n}
    del a, b
    torch.cuda.empty_cache()
    return out


def batch_section(torch, rtt, synth, oracle, dev, ridge_iters=20, k=256, p=8, q=2):
    """The 12-geometry x 60-history batch: batched vs per-instance A/A^T and autograd, and one
    captured graph of A, A^T, TSVD and a fixed-count ridge solve of every (geometry, history)."""
    from paper_2609_05528_amd.autograd import ridge_loss
    geos = synth.batch_geometries()
    ng, nh = len(geos), synth.BATCH_HISTORIES
    G = rtt.Geometry(geos)
    lam = 1e-3
    t0 = time.perf_counter()
    G.tune(nvec=nh, reps=3)
    t_tune = time.perf_counter() - t0
    H = torch.from_numpy(synth.blob_histories(geos[0].grid, nh, dtype=np.float32)).to(dev)   # [60][S*K]
    X = H.repeat(1, ng).contiguous()          # history h in every geometry's column block
    Y = torch.empty((nh, G.n_rows), dtype=torch.float32, device=dev)
    XT = torch.empty_like(X)
    pairs = ng * nh
    log("batch: %d geometries, %d histories, rows %d, cols %d, launch modes %s" % (
        ng, nh, G.n_rows, G.n_cols, G.batch_mode))

    # batched A + A^T over every (geometry, history) pair
    rtt.op_apply(G, X, Y)
    rtt.op_apply_adjoint(G, Y, XT)
    torch.cuda.synchronize()
    reps = 5
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        rtt.op_apply(G, X, Y)
    ev[1].record()
    for _ in range(reps):
        rtt.op_apply_adjoint(G, Y, XT)
    ev[2].record()
    torch.cuda.synchronize()
    ms_a, ms_at = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
    ncell = sum(g.grid.n_cells for g in geos)
    b_a = algorithmic_bytes(G.n_rows, G.n_cols, G.n_rays, ncell, 3, nh, False)
    b_at = algorithmic_bytes(G.n_rows, G.n_cols, G.n_rays, ncell, 3, nh, True)
    batched = 2 * pairs / ((ms_a + ms_at) * 1e-3)

    # parity of sampled (geometry, history) pairs against the FP64 oracle
    par = []
    for gi, hi in ((0, 0), (ng - 1, nh - 1), (5, 31)):
        m = G.members[gi]
        yr = oracle.forward(geos[gi], H[hi].double().cpu().numpy())
        ya = Y[hi, m["row_offset"]:m["row_offset"] + m["n_rows"]].double().cpu().numpy()
        par.append(float(np.linalg.norm(ya - yr) / np.linalg.norm(yr)))
        xr = oracle.adjoint(geos[gi], Y[hi, m["row_offset"]:m["row_offset"] + m["n_rows"]].double().cpu().numpy())
        xa = XT[hi, m["col_offset"]:m["col_offset"] + m["n_cols"]].double().cpu().numpy()
        par.append(float(np.linalg.norm(xa - xr) / np.linalg.norm(xr)))

    # the same work as a plain loop: one handle per geometry, one history per call
    singles = [rtt.Geometry(g) for g in geos]
    for Gs in singles:
        Gs.tune(nvec=1, reps=3)
    yb = [torch.empty(Gs.n_rows, dtype=torch.float32, device=dev) for Gs in singles]
    xb = [torch.empty(Gs.n_cols, dtype=torch.float32, device=dev) for Gs in singles]
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for h in range(nh):
        for gi, Gs in enumerate(singles):
            rtt.op_apply(Gs, H[h], yb[gi])
            rtt.op_apply_adjoint(Gs, yb[gi], xb[gi])
    torch.cuda.synchronize()
    plain = 2 * pairs / (time.perf_counter() - tp0)

    # autograd: ridge loss of every pair and its gradient in one call, vs one pair per call
    Yobs = Y.clone()
    Yobs.add_(0.01)
    Xg = X.clone().requires_grad_(True)

    def grad_step():
        Xg.grad = None
        ridge_loss(Xg, Yobs, G, lam).backward()

    grad_step()
    torch.cuda.synchronize()
    ta0 = time.perf_counter()
    for _ in range(3):
        grad_step()
    torch.cuda.synchronize()
    ag_batched = 3 * pairs / (time.perf_counter() - ta0)
    xs = [H[h].clone().requires_grad_(True) for h in range(nh)]
    ys = [[Yobs[h, m["row_offset"]:m["row_offset"] + m["n_rows"]].contiguous() for m in G.members] for h in range(nh)]
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    for h in range(nh):
        for gi, Gs in enumerate(singles):
            xs[h].grad = None
            ridge_loss(xs[h], ys[h][gi], Gs, lam).backward()
    torch.cuda.synchronize()
    ag_plain = pairs / (time.perf_counter() - tb0)
    g_rel = float((xs[nh - 1].grad - Xg.grad[nh - 1, G.members[ng - 1]["col_offset"]:
                                               G.members[ng - 1]["col_offset"] + G.members[ng - 1]["n_cols"]]).norm()
                  / xs[nh - 1].grad.norm())
    del xs, ys, singles, yb, xb, Xg
    torch.cuda.empty_cache()

    # rSVD of every geometry in one call, then the captured step
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    sv = rtt.rsvd(G, k=k, p=p, q=q, seed=4001, geometry=rtt.RTT_EACH_GEOMETRY)
    torch.cuda.synchronize()
    t_rsvd = time.perf_counter() - tr0
    Xts = torch.empty_like(X)
    Xrg = torch.empty_like(X)
    resid = torch.empty(pairs, dtype=torch.float32, device=dev)

    def step():
        rtt.op_apply(G, X, Y)
        rtt.op_apply_adjoint(G, Yobs, XT)
        rtt.tsvd_solve(G, sv, Yobs, t=k, x=Xts)
        rtt.ridge_solve(G, Yobs, lam, maxit=ridge_iters, x=Xrg, async_mode=True, resid=resid)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    te0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - te0
    ref = [t.clone() for t in (Y, XT, Xts, Xrg)]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    same = all(bool(torch.equal(a, b)) for a, b in zip(ref, (Y, XT, Xts, Xrg)))
    gev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    greps = 3
    gev[0].record()
    for _ in range(greps):
        graph.replay()
    gev[1].record()
    torch.cuda.synchronize()
    ms_graph = gev[0].elapsed_time(gev[1]) / greps
    del graph, sv
    torch.cuda.empty_cache()
    ages = age_section(torch, rtt, geos, G)
    out = {
        "workload": "12 geometries (spins 0/0.3/0.6/0.94 x incl 20/50/75, 96^2-256^2, 64-160 frames, "
                    "orders 0-2) x 60 Gaussian-blob histories on a shared 64x64x96 basis",
        "pairs": pairs, "rows": G.n_rows, "cols": G.n_cols, "rays": G.n_rays,
        "launch_modes": list(G.batch_mode), "tune_seconds": t_tune,
        "op_apply": {"ms": ms_a, "GBps": b_a / (ms_a * 1e-3) / 1e9},
        "op_apply_adjoint": {"ms": ms_at, "GBps": b_at / (ms_at * 1e-3) / 1e9},
        "batched_applies_per_s": batched, "plain_applies_per_s": plain,
        "autograd_pairs_per_s": {"batched": ag_batched, "plain": ag_plain, "grad_rel_diff": g_rel},
        "parity_max_rel_err": max(par),
        "rsvd_each_geometry": {"seconds": t_rsvd, "k": k, "p": p, "q": q},
        "graph_step": {"ms_replay": ms_graph, "s_eager": t_eager, "replay_equals_eager": same,
                       "ridge_iterations": ridge_iters, "tsvd_t": k,
                       "contents": "A + A^T + TSVD + ridge CG on every (geometry, history) pair"},
        "age_information": ages,
    }
    log("batch: A %.2f ms A^T %.2f ms (%.0f / %.0f GB/s); batched %.0f vs plain %.0f applies/s; "
        "autograd %.0f vs %.0f pairs/s; graph %.1f ms" % (ms_a, ms_at, out["op_apply"]["GBps"],
                                                          out["op_apply_adjoint"]["GBps"], batched, plain,
                                                          ag_batched, ag_plain, ms_graph))
    del X, Y, XT, Xts, Xrg, Yobs, H, G
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--nvec", type=int, default=264)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-rsvd", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-mixer", action="store_true")
    ap.add_argument("--no-age", action="store_true")
    ap.add_argument("--no-estimators", action="store_true")
    ap.add_argument("--no-synthesis", action="store_true")
    ap.add_argument("--apply-variant", default="", help="pin the forward kernel variant (name) after tuning")
    ap.add_argument("--adjoint-variant", default="", help="pin the adjoint kernel variant (name) after tuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_05528_amd as rtt
    import synth

    rtt.require_native()
    dev = torch.device("cuda:0")
    calib = calibrate(torch, dev)
    log("calibration: %s" % calib)
    p = synth.config(args.workload)
    geo = synth.geometry_for(p)
    g = geo.grid
    G = rtt.Geometry(geo)
    nvec = args.nvec
    log("workload %s: rays %s, rows %d, cols %d, nvec %d" % (args.workload, geo.rays_per_order, G.n_rows,
                                                             G.n_cols, nvec))
    if not args.no_tune:
        choice = G.tune(nvec=nvec, reps=5)
        log("autotuner choice (apply, adjoint): %s = %s" % (choice, [
            (rtt.variant_names(False)[a], rtt.variant_names(True)[b]) for a, b in choice]))
    if args.apply_variant or args.adjoint_variant:
        G.set_variant(apply=rtt.variant_names(False).index(args.apply_variant) if args.apply_variant else -1,
                      adjoint=rtt.variant_names(True).index(args.adjoint_variant) if args.adjoint_variant else -1)
        log("variants pinned: %s / %s" % (args.apply_variant, args.adjoint_variant))
    om = synth.gaussian_block(G.n_cols, nvec, seed=p["seed"] + 1)
    X = torch.from_numpy(om).to(dev)
    del om
    Y = torch.empty((nvec, G.n_rows), dtype=torch.float32, device=dev)
    XT = torch.empty((nvec, G.n_cols), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def step(evs=None):
        if evs is not None:
            evs[0].record()
        rtt.op_apply(G, X, Y)
        if evs is not None:
            evs[1].record()
        rtt.op_apply_adjoint(G, Y, XT)
        if evs is not None:
            evs[2].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    t_a = [e[0].elapsed_time(e[1]) for e in events]
    t_at = [e[1].elapsed_time(e[2]) for e in events]
    ms_a, ms_at = float(np.mean(t_a)), float(np.mean(t_at))
    applies = 2 * nvec * args.steps
    value = applies / wall
    log("A %.3f ms, A^T %.3f ms per block launch; step %.3f ms" % (ms_a, ms_at, 1e3 * wall / args.steps))

    nc = g.n_cells
    b_a = algorithmic_bytes(G.n_rows, G.n_cols, G.n_rays, nc, g.n_orders, nvec, False)
    b_at = algorithmic_bytes(G.n_rows, G.n_cols, G.n_rays, nc, g.n_orders, nvec, True)
    gbps_a = b_a / (ms_a * 1e-3) / 1e9
    gbps_at = b_at / (ms_at * 1e-3) / 1e9
    dom = "op_apply_adjoint" if ms_at >= ms_a else "op_apply"
    dom_gbps = gbps_at if ms_at >= ms_a else gbps_a
    dom_bytes = b_at if ms_at >= ms_a else b_a

    variants = {"op_apply": rtt.variant_names(False)[G.members[0]["apply_variant"]],
                "op_apply_adjoint": rtt.variant_names(True)[G.members[0]["adjoint_variant"]]}

    # parity of two vectors of the block against the FP64 oracle
    import oracle
    par = {}
    for b in (0, nvec - 1):
        xb = X[b].double().cpu().numpy()
        yr = oracle.forward(geo, xb)
        ya = Y[b].double().cpu().numpy()
        par.setdefault("A", []).append(float(np.linalg.norm(ya - yr) / np.linalg.norm(yr)))
        xr = oracle.adjoint(geo, Y[b].double().cpu().numpy())
        xa = XT[b].double().cpu().numpy()
        par.setdefault("AT", []).append(float(np.linalg.norm(xa - xr) / np.linalg.norm(xr)))
    parity = {"A_max_rel_err": max(par["A"]), "AT_max_rel_err": max(par["AT"]), "vectors": [0, nvec - 1],
              "tol": 1e-5}

    mixers = None if args.no_mixer else mixer_section(torch, rtt, oracle, geo, G, Y)
    ages = None if args.no_age else age_section(torch, rtt, [geo], G)
    estimators = None if args.no_estimators else estimator_section(torch, rtt, synth, geo, G)
    synthesis = None if args.no_synthesis else synthesis_section(torch, rtt, G)

    # plain per-instance loop on the same GPU (one vector per call)
    plain = None
    if not args.no_plain:
        xs = [X[b] for b in range(nvec)]
        ys = [Y[b] for b in range(nvec)]
        xts = [XT[b] for b in range(nvec)]
        for b in range(min(nvec, 8)):
            rtt.op_apply(G, xs[b], ys[b])
            rtt.op_apply_adjoint(G, ys[b], xts[b])
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for b in range(nvec):
            rtt.op_apply(G, xs[b], ys[b])
            rtt.op_apply_adjoint(G, ys[b], xts[b])
        torch.cuda.synchronize()
        plain = 2 * nvec / (time.perf_counter() - tp0)

    cpu = None
    if not args.no_cpu_baseline:
        n_s = nvec
        xs = X[:n_s].double().cpu().numpy()
        tc0 = time.perf_counter()
        yo = oracle.forward(geo, xs)
        oracle.adjoint(geo, yo)
        tc = time.perf_counter() - tc0
        cpu = {"value": 2 * n_s / tc, "unit": "applies/s", "cores": 1, "kind": "oracle",
               "sample": "one full step: %d A + %d A^T FP64 applies (plain C, single thread), %.1f s"
                         % (n_s, n_s, tc)}

    # the large single geometry (512^2 x 512 frames, orders 0-2): one vector per launch
    large = None
    if not args.no_large:
        del X, Y, XT
        torch.cuda.empty_cache()
        geo5 = synth.geometry_for("cfg5")
        G5 = rtt.Geometry(geo5)
        G5.tune(nvec=1, reps=3)
        x5 = torch.from_numpy(synth.uniform_emissivity(geo5.grid, seed=5000).astype(np.float32)).to(dev)
        y5 = torch.empty(G5.n_rows, dtype=torch.float32, device=dev)
        xt5 = torch.empty_like(x5)
        ta5, tat5 = time_pair(torch, rtt, G5, x5, y5, xt5, reps=20)
        g5 = geo5.grid
        b5 = algorithmic_bytes(G5.n_rows, G5.n_cols, G5.n_rays, g5.n_cells, g5.n_orders, 1, False)
        b5t = algorithmic_bytes(G5.n_rows, G5.n_cols, G5.n_rays, g5.n_cells, g5.n_orders, 1, True)
        v1 = (rtt.variant_names(False)[G5.members[0]["apply_variant"]],
              rtt.variant_names(True)[G5.members[0]["adjoint_variant"]])
        # block Lanczos on the large geometry (512 right vectors: 16 steps of 32), wall time, with
        # the kernel variants tuned for its 32-vector blocks
        G5.tune(nvec=32, reps=3)
        torch.cuda.synchronize()
        t0l = time.perf_counter()
        svl = rtt.rsvd(G5, method="lanczos", k=64, block=32, steps=16, seed=5001)
        torch.cuda.synchronize()
        t_lz = time.perf_counter() - t0l
        lz = {"seconds": t_lz, "block": 32, "steps": 16, "theta_1": float(svl.sigma[0]),
              "residual_1": float(svl.residual[0]),
              "variants": [rtt.variant_names(False)[G5.members[0]["apply_variant"]],
                           rtt.variant_names(True)[G5.members[0]["adjoint_variant"]]]}
        del svl
        log("lanczos (512 vectors, large geometry): %.2f s" % t_lz)
        large = {"workload": "cfg5: " + synth.config("cfg5")["label"] + ", one vector per launch",
                 "block_lanczos_512": lz,
                 "op_apply": {"ms": ta5, "GBps": b5 / (ta5 * 1e-3) / 1e9,
                              "frac": b5 / (ta5 * 1e-3) / 1e9 / HBM_PEAK_GBPS, "variant": v1[0]},
                 "op_apply_adjoint": {"ms": tat5, "GBps": b5t / (tat5 * 1e-3) / 1e9,
                                      "frac": b5t / (tat5 * 1e-3) / 1e9 / HBM_PEAK_GBPS, "variant": v1[1]},
                 "applies_per_s": 2.0 / ((ta5 + tat5) * 1e-3)}
        log("large geometry: A %.3f ms (%.0f GB/s), A^T %.3f ms (%.0f GB/s)" % (
            ta5, large["op_apply"]["GBps"], tat5, large["op_apply_adjoint"]["GBps"]))
        del G5, x5, y5, xt5
        torch.cuda.empty_cache()

    # randomized SVD of the benchmark geometry (k = 256, p = 8, q = 2), wall time
    rs = None
    if not args.no_rsvd:
        torch.cuda.synchronize()
        t0r = time.perf_counter()
        sv = rtt.rsvd(G, k=p.get("rsvd_k", 256), p=p.get("rsvd_p", 8), q=p.get("rsvd_q", 2), seed=2001)
        torch.cuda.synchronize()
        t_rs = time.perf_counter() - t0r
        # (q + 1) block applies of A and of A^T on l = k + p vectors; the rest is the dense part
        # (MFMA Gram / combine, FP64 small factorisations on the host)
        t_app = (p.get("rsvd_q", 2) + 1) * (ms_a + ms_at) * 1e-3
        rs = {"seconds": t_rs, "k": sv.k, "sigma_1": float(sv.sigma[0]),
              "sigma_k": float(sv.sigma[-1]), "block_applies": 6 * (p.get("rsvd_k", 256) + p.get("rsvd_p", 8)),
              "apply_seconds_est": t_app, "dense_seconds_est": t_rs - t_app}
        log("rsvd: %.2f s, sigma_1 %.4g sigma_k %.4g" % (rs["seconds"], rs["sigma_1"], rs["sigma_k"]))
        del sv

    n_rows, n_cols = G.n_rows, G.n_cols
    batch = None
    if not args.no_batch:
        del G
        torch.cuda.empty_cache()
        batch = batch_section(torch, rtt, synth, oracle, dev)

    digest = source_digest()
    traffic = None
    for meas in MEASURED_TRAFFIC.get(dom, []):
        if meas["digest"] == digest and meas["nvec"] == nvec and meas["variant"] == variants[dom]:
            traffic = meas["bytes"]

    out = {
        "metric": METRIC, "value": value, "unit": "applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: %s; block of %d vectors (rSVD l=k+p); step = A + A^T on the block"
                               % (args.workload, p["label"], nvec),
                   "rays_per_order": geo.rays_per_order, "rows": n_rows, "cols": n_cols, "nvec": nvec},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dom_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": dom_gbps / HBM_PEAK_GBPS, "traffic": traffic, "bytes_per_launch": dom_bytes,
                     "kernel_source_digest": digest},
        "kernels": {"op_apply": {"ms": ms_a, "GBps": gbps_a, "bytes": b_a,
                                 "ms_p10_median_p90": [float(np.percentile(t_a, q)) for q in (10, 50, 90)],
                                 "frac_of_copy": gbps_a / calib["copy_gbps"]},
                    "op_apply_adjoint": {"ms": ms_at, "GBps": gbps_at, "bytes": b_at,
                                         "ms_p10_median_p90": [float(np.percentile(t_at, q)) for q in (10, 50, 90)],
                                         "frac_of_copy": gbps_at / calib["copy_gbps"]}},
        "hbm_gbps": (b_a + b_at) / ((ms_a + ms_at) * 1e-3) / 1e9,
        "variants": variants,
        "plain_value": plain,
        "calibration": calib,
        "large_single_vector": large,
        "rsvd": rs,
        "batch": batch,
        "mixers": mixers,
        "age_information": ages,
        "estimators": estimators,
        "synthesis": synthesis,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
