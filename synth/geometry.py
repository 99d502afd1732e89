"""Grid descriptors and synthetic per-order ray maps (inputs of the operator).

A ray map lists, for every retained screen ray of one image order n, the
source-plane point the ray lands on (r, phi), its coordinate-time delay and its
transfer weight: the quantities chi, w, (r_n, phi_n) and Delta_n of the
transfer map of Sec. 3.1, eq. (2).  Rays with chi = 0 are simply not listed
(only retained rays P_n enter eq. (23) and eq. (47)).

The synthetic maps stand in for the paper's ray-traced Kerr maps, which are
not available.  Their recipe:

* screen: a W x W pixel grid over the square field of view [-R, R]^2 with
  R = r_out; pixel centres at (i + 1/2) * 2R/W - R; impact radius b and screen
  angle theta = atan2(beta, alpha) mod 2 pi;
* order 0: every pixel with r_in <= b <= r_out; r_src = b (a monotone map),
  phi_src = theta, delay = r_src (1 - sin i cos phi_src), weight 1;
* order n >= 1: pixels in a thin ring |b - rho_n| <= width/2 with
  rho_n = 5.2 (1 + 0.02 (2 - n)); across the ring r_src runs linearly from
  r_in to r_out; phi_src = theta + n pi; delay = r_src (1 - sin i cos phi_src)
  + 16.3 n; weight exp(-pi n).

Spin enters none of these formulas: it is a label of the geometry only.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass(frozen=True)
class Grid:
    """Observer frames, polar source cells and source-time hats.

    Frames sit at t_f = t0 + f * dt_obs (f = 0..n_frames-1).  Source cells are
    n_r x n_phi polar cells over r in [r_in, r_out] and phi in [0, 2 pi); the
    spatial coefficient of cell (i, j) lives at index s = i * n_phi + j.  Hats
    are centred at s_k = s0 + k * dt_src (k = 0..n_hat-1) with half-width
    dt_src.  Coefficient vectors are laid out [s][k] with k fastest.
    """

    n_orders: int
    n_frames: int
    t0: float
    dt_obs: float
    n_r: int
    n_phi: int
    r_in: float
    r_out: float
    n_hat: int
    s0: float
    dt_src: float

    @property
    def n_cells(self) -> int:
        return self.n_r * self.n_phi

    @property
    def n_cols(self) -> int:
        return self.n_r * self.n_phi * self.n_hat

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


@dataclasses.dataclass
class RayMap:
    """Retained rays of one image order (all arrays FP64 except ``pixel``)."""

    r: np.ndarray
    phi: np.ndarray
    delay: np.ndarray
    weight: np.ndarray
    pixel: Optional[np.ndarray] = None

    def __post_init__(self):
        self.r = np.ascontiguousarray(self.r, dtype=np.float64)
        self.phi = np.ascontiguousarray(self.phi, dtype=np.float64)
        self.delay = np.ascontiguousarray(self.delay, dtype=np.float64)
        self.weight = np.ascontiguousarray(self.weight, dtype=np.float64)
        if self.pixel is not None:
            self.pixel = np.ascontiguousarray(self.pixel, dtype=np.int32)
        n = self.r.shape[0]
        for a in (self.phi, self.delay, self.weight):
            if a.shape != (n,):
                raise ValueError("ray map arrays must share one length")

    @property
    def n_rays(self) -> int:
        return int(self.r.shape[0])


@dataclasses.dataclass
class Geometry:
    """One imaging geometry: a grid plus one ray map per order."""

    grid: Grid
    maps: List[RayMap]
    label: str = ""
    image_side: int = 0

    def __post_init__(self):
        if len(self.maps) != self.grid.n_orders:
            raise ValueError("need one ray map per order")

    @property
    def rays_per_order(self) -> List[int]:
        return [m.n_rays for m in self.maps]

    @property
    def n_rays(self) -> int:
        return sum(self.rays_per_order)

    @property
    def n_rows(self) -> int:
        return self.n_rays * self.grid.n_frames

    def digest(self) -> str:
        """SHA-256 of the grid and the raw ray maps (a content hash)."""
        h = hashlib.sha256()
        h.update(repr(sorted(self.grid.as_dict().items())).encode())
        for m in self.maps:
            for a in (m.r, m.phi, m.delay, m.weight):
                h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def ring_radius(n: int) -> float:
    """Screen radius of the order-n ring, 5.2 (1 + 0.02 (2 - n))."""
    return 5.2 * (1.0 + 0.02 * (2 - n))


def screen_raymaps(side: int, incl_deg: float, n_orders: int, r_in: float,
                   r_out: float, ring_width: float = 0.5,
                   order_delay: float = 16.3) -> List[RayMap]:
    """Synthetic per-order ray maps on a side x side screen (module recipe)."""
    half = r_out
    c = (np.arange(side, dtype=np.float64) + 0.5) * (2.0 * half / side) - half
    alpha, beta = np.meshgrid(c, c, indexing="xy")       # beta varies over rows
    alpha = alpha.ravel()
    beta = beta.ravel()
    pix = np.arange(side * side, dtype=np.int64)
    b = np.hypot(alpha, beta)
    theta = np.mod(np.arctan2(beta, alpha), TWO_PI)
    sin_i = math.sin(math.radians(incl_deg))
    maps = []
    for n in range(n_orders):
        if n == 0:
            sel = (b >= r_in) & (b <= r_out)
            r_src = b[sel]
            phi_src = theta[sel]
            extra = 0.0
            wn = 1.0
        else:
            rho = ring_radius(n)
            lo = rho - 0.5 * ring_width
            sel = np.abs(b - rho) <= 0.5 * ring_width
            r_src = r_in + (b[sel] - lo) / ring_width * (r_out - r_in)
            r_src = np.clip(r_src, r_in, r_out)
            phi_src = np.mod(theta[sel] + n * math.pi, TWO_PI)
            extra = order_delay * n
            wn = math.exp(-math.pi * n)
        delay = r_src * (1.0 - sin_i * np.cos(phi_src)) + extra
        maps.append(RayMap(r=r_src, phi=phi_src, delay=delay,
                           weight=np.full(r_src.shape, wn),
                           pixel=pix[sel].astype(np.int32)))
    return maps


def random_geometry(grid: Grid, rays_per_order, seed: int,
                    delay_range=(0.0, 30.0), order_delay: float = 16.3,
                    edge_guard: float = 1e-6) -> Geometry:
    """Small random geometry for tests: rays spread over the whole annulus.

    Radii are uniform on [r_in, r_out] (including the clamped half-cells next
    to both edges), azimuths uniform on [0, 2 pi) (so the periodic seam is
    crossed), delays uniform on ``delay_range`` shifted by ``order_delay * n``
    and weights uniform on [0.5, 1.5) times exp(-pi n).  Retarded times are
    nudged off the hat nodes by at least ``edge_guard * dt_src`` so that the
    set of touched hats does not hinge on rounding.
    """
    rng = np.random.default_rng(seed)
    maps = []
    for n, cnt in enumerate(rays_per_order):
        r = rng.uniform(grid.r_in, grid.r_out, cnt)
        phi = rng.uniform(0.0, TWO_PI, cnt)
        delay = rng.uniform(delay_range[0], delay_range[1], cnt) + order_delay * n
        # keep (t0 - delay - s0)/dt_src away from integers
        u = (grid.t0 - delay - grid.s0) / grid.dt_src
        ratio = grid.dt_obs / grid.dt_src
        frac_steps = np.mod(np.arange(max(grid.n_frames, 1)) * ratio, 1.0)
        for _ in range(8):
            bad = np.zeros(cnt, dtype=bool)
            for fs in np.unique(np.round(frac_steps, 12)):
                v = u + fs
                d = np.abs(v - np.round(v))
                bad |= d < edge_guard
            if not bad.any():
                break
            delay[bad] += 3.7 * edge_guard * grid.dt_src
            u = (grid.t0 - delay - grid.s0) / grid.dt_src
        w = rng.uniform(0.5, 1.5, cnt) * math.exp(-math.pi * n)
        maps.append(RayMap(r=r, phi=phi, delay=delay, weight=w,
                           pixel=np.arange(cnt, dtype=np.int32)))
    return Geometry(grid=grid, maps=maps, label=f"random-{seed}")


def pairing_destroyed(geom: Geometry, seed: int) -> Geometry:
    """The pairing-destroyed control of Sec. 6.4 as an input transform: within every order the
    delays are permuted among the rays by a seeded permutation, so each order keeps its delay
    marginal while the association of delay with source position and transfer weight is lost.
    Radii, azimuths, weights and pixels stay with their rays."""
    rng = np.random.default_rng(seed)
    maps = []
    for m in geom.maps:
        perm = rng.permutation(m.n_rays)
        maps.append(dataclasses.replace(m, delay=np.ascontiguousarray(m.delay[perm])))
    return Geometry(grid=geom.grid, maps=maps, label=(geom.label or "") + "-pairing-destroyed",
                    image_side=geom.image_side)


def spatial_only(geom: Geometry) -> Geometry:
    """Spatial-only mechanism arm (Sec. 6.4) as an input transform: every order n >= 1 keeps its rays'
    source positions and weights, but its delays are shifted by the difference of the order's median
    delay and the direct order's, so the higher orders add new source positions at the direct
    image's epochs."""
    d0 = float(np.median(geom.maps[0].delay)) if geom.maps[0].n_rays else 0.0
    maps = [geom.maps[0]]
    for m in geom.maps[1:]:
        shift = float(np.median(m.delay)) - d0 if m.n_rays else 0.0
        maps.append(dataclasses.replace(m, delay=np.ascontiguousarray(m.delay - shift)))
    return Geometry(grid=geom.grid, maps=maps, label=(geom.label or "") + "-spatial-only", image_side=geom.image_side)


def delay_only(geom: Geometry, seed: int) -> Geometry:
    """Delay-only mechanism arm (Sec. 6.4) as an input transform: every order n >= 1 keeps its rays'
    delays and weights, but each ray's source position is replaced by that of a direct-order ray
    drawn uniformly (seeded), so the higher orders sample the direct image's spatial distribution
    and can add only retarded-time information."""
    rng = np.random.default_rng(seed)
    m0 = geom.maps[0]
    maps = [m0]
    for m in geom.maps[1:]:
        pick = rng.integers(0, m0.n_rays, m.n_rays) if m0.n_rays else np.zeros(m.n_rays, dtype=np.int64)
        maps.append(dataclasses.replace(m, r=np.ascontiguousarray(m0.r[pick]), phi=np.ascontiguousarray(m0.phi[pick])))
    return Geometry(grid=geom.grid, maps=maps, label=(geom.label or "") + "-delay-only", image_side=geom.image_side)
