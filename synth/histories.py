"""Seeded emissivity coefficient vectors and random blocks.

* ``uniform_emissivity``: coefficients uniform on [0, 1) (the direct draws of
  numpy's default generator with the given seed).
* ``blob_histories``: smooth histories made of Gaussian blobs, sampled at the
  cell centres and hat nodes (both bases interpolate their nodal values).  Per
  blob: amplitude exp(0.5 N(0,1)) (lognormal, sigma 0.5), lifetime L ~ U[8M,
  40M] used as the temporal Gaussian width, spatial width U[1M, 3M], centre
  area-uniform in the annulus, peak time uniform over the hat window; three
  blobs per history; history h uses ``default_rng(40000 + h)``.
* ``gaussian_block``: N(0,1) test matrices (e.g. the range-finder block).
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Grid


def uniform_emissivity(grid: Grid, seed: int, nvec: int = 1, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.random((nvec, grid.n_cells * grid.n_hat))
    return x.astype(dtype) if nvec > 1 else x[0].astype(dtype)


def gaussian_block(n: int, ncol: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Column block of shape (ncol, n) (one row per vector), N(0,1) entries."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ncol, n), dtype=np.float64).astype(dtype)


def cell_centres(grid: Grid):
    dr = (grid.r_out - grid.r_in) / grid.n_r
    dphi = 2.0 * math.pi / grid.n_phi
    rc = grid.r_in + (np.arange(grid.n_r) + 0.5) * dr
    pc = (np.arange(grid.n_phi) + 0.5) * dphi
    return rc, pc


def blob_histories(grid: Grid, n_hist: int, base_seed: int = 40000, n_blobs: int = 3,
                   dtype=np.float64) -> np.ndarray:
    rc, pc = cell_centres(grid)
    R, P = np.meshgrid(rc, pc, indexing="ij")            # [n_r][n_phi]
    X, Y = R * np.cos(P), R * np.sin(P)
    tk = grid.s0 + grid.dt_src * np.arange(grid.n_hat)
    out = np.zeros((n_hist, grid.n_cells, grid.n_hat))
    for h in range(n_hist):
        rng = np.random.default_rng(base_seed + h)
        for _ in range(n_blobs):
            amp = math.exp(0.5 * rng.standard_normal())
            life = rng.uniform(8.0, 40.0)
            width = rng.uniform(1.0, 3.0)
            rb = math.sqrt(rng.uniform(grid.r_in ** 2, grid.r_out ** 2))
            pb = rng.uniform(0.0, 2.0 * math.pi)
            tb = rng.uniform(tk[0], tk[-1])
            sp = np.exp(-((X - rb * math.cos(pb)) ** 2 + (Y - rb * math.sin(pb)) ** 2)
                        / (2.0 * width ** 2)).reshape(-1)
            tp = np.exp(-((tk - tb) ** 2) / (2.0 * life ** 2))
            out[h] += amp * np.outer(sp, tp)
    return out.reshape(n_hist, -1).astype(dtype)
