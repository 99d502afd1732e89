"""The five synthetic workloads: sizes, cadences and the readings they fix.

Every choice that the paper leaves open is written down here once:

* frames at t_f = f * dt_obs (t0 = 0); dt_obs = 4M except the large geometry
  (2M); hats at dt_src = 4M everywhere (the paper's 4M age grid, Sec. 3.3);
* the hat window is old-anchored: s0 = dt_src * floor((t0 - tau_max)/dt_src)
  - dt_src with tau_max the largest delay over all orders, so the oldest hat
  is blind to every order and the hats between the direct and the resolved
  old edges are blind to the direct image (the structure of Thm 4.1);
* source cells are uniform in r over [6M, 20M] and periodic in phi.
"""
from __future__ import annotations

import math

from .geometry import Geometry, Grid, screen_raymaps

R_IN, R_OUT = 6.0, 20.0
ORDER_DELAY = 16.3


def old_anchor(t0: float, tau_max: float, dt_src: float) -> float:
    return dt_src * math.floor((t0 - tau_max) / dt_src) - dt_src


def _tau_max(incl_deg: float, n_orders: int) -> float:
    return R_OUT * (1.0 + math.sin(math.radians(incl_deg))) + ORDER_DELAY * (n_orders - 1)


# name -> parameters; "incl" in degrees; "spin" is a label only
CONFIGS = {
    "cfg1": dict(label="Schwarzschild i=20 n=0, 64^2 x 40 frames", spin=0.0, incl=20.0,
                 side=64, n_orders=1, n_frames=40, dt_obs=4.0, n_r=32, n_phi=32,
                 n_hat=40, dt_src=4.0, seed=1000),
    "cfg2": dict(label="Kerr a=0.5 i=50 n=0-2, 128^2 x 128 frames", spin=0.5, incl=50.0,
                 side=128, n_orders=3, n_frames=128, dt_obs=4.0, n_r=64, n_phi=64,
                 n_hat=96, dt_src=4.0, seed=2000, rsvd_k=256, rsvd_p=8, rsvd_q=2),
    "cfg3": dict(label="Schwarzschild i=20 n=0, 256^2 x 192 frames (ridge)", spin=0.0,
                 incl=20.0, side=256, n_orders=1, n_frames=192, dt_obs=4.0, n_r=32,
                 n_phi=32, n_hat=200, dt_src=4.0, seed=3000, ridge_lambda=1e-3),
    "cfg5": dict(label="Kerr a=0.94 i=75 n=0-2, 512^2 x 512 frames", spin=0.94, incl=75.0,
                 side=512, n_orders=3, n_frames=512, dt_obs=2.0, n_r=128, n_phi=128,
                 n_hat=256, dt_src=4.0, seed=5000, lanczos_vectors=512),
}

BATCH_SPINS = (0.0, 0.3, 0.6, 0.94)
BATCH_INCLS = (20.0, 50.0, 75.0)


def batch_members():
    """The 12 spin x inclination geometries of the batched workload.

    Geometry g = 3 * spin_index + incl_index has an image side
    96 + round(160 g / 11) and 64 + round(96 ((7 g) mod 12) / 11) frames (a
    permutation that decouples image size from frame count); all share one
    64 x 64 x 96 source basis with s0 = -76.
    """
    out = []
    for si, a in enumerate(BATCH_SPINS):
        for ii, inc in enumerate(BATCH_INCLS):
            g = 3 * si + ii
            side = 96 + int(round(160.0 * g / 11.0))
            frames = 64 + int(round(96.0 * ((7 * g) % 12) / 11.0))
            out.append(dict(label=f"a={a} i={inc:g}", spin=a, incl=inc, side=side,
                            n_orders=3, n_frames=frames, dt_obs=4.0, n_r=64, n_phi=64,
                            n_hat=96, dt_src=4.0))
    return out


BATCH_S0 = -76.0
BATCH_HISTORIES = 60


def config(name: str) -> dict:
    return dict(CONFIGS[name])


def grid_for(p: dict, s0: float = None) -> Grid:
    if s0 is None:
        s0 = old_anchor(0.0, _tau_max(p["incl"], p["n_orders"]), p["dt_src"])
    return Grid(n_orders=p["n_orders"], n_frames=p["n_frames"], t0=0.0, dt_obs=p["dt_obs"],
                n_r=p["n_r"], n_phi=p["n_phi"], r_in=R_IN, r_out=R_OUT,
                n_hat=p["n_hat"], s0=float(s0), dt_src=p["dt_src"])


def geometry_for(p, s0: float = None) -> Geometry:
    """Build the synthetic geometry of a config name or parameter dict."""
    if isinstance(p, str):
        p = config(p)
    g = grid_for(p, s0)
    maps = screen_raymaps(p["side"], p["incl"], p["n_orders"], R_IN, R_OUT,
                          order_delay=ORDER_DELAY)
    return Geometry(grid=g, maps=maps, label=p["label"], image_side=p["side"])


def batch_geometries():
    return [geometry_for(m, s0=BATCH_S0) for m in batch_members()]
