"""Small seeded test geometries whose hat window covers every retarded time."""
import math

import synth


def tiny_grid(n_orders=3, n_frames=6, dt_obs=4.0, n_r=4, n_phi=6, dt_src=4.0,
              delay_hi=10.0, order_delay=16.3, extra_hats=1):
    tau_max = delay_hi + order_delay * (n_orders - 1)
    s0 = synth.configs.old_anchor(0.0, tau_max, dt_src)
    t_last = (n_frames - 1) * dt_obs
    n_hat = int(math.ceil((t_last - s0) / dt_src)) + 1 + extra_hats
    return synth.Grid(n_orders=n_orders, n_frames=n_frames, t0=0.0, dt_obs=dt_obs, n_r=n_r,
                      n_phi=n_phi, r_in=6.0, r_out=20.0, n_hat=n_hat, s0=s0, dt_src=dt_src)


def tiny_geometry(seed=1, rays=(12, 6, 5), **kw):
    g = tiny_grid(n_orders=len(rays), **kw)
    return synth.random_geometry(g, list(rays), seed=seed, delay_range=(0.0, kw.get("delay_hi", 10.0)))
