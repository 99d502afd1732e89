"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package produces inputs only: observer/source grid descriptors, per-order
ray maps (source radius, azimuth, delay, transfer weight), emissivity
coefficient vectors and random test blocks.  It contains none of the
operator's arithmetic (no stencil, no hat evaluation, no gather or scatter),
so both the CPU oracle and the GPU path can consume the same arrays without
sharing any code of the method itself.
"""
from .configs import (CONFIGS, config, grid_for, geometry_for, batch_members,  # noqa: F401
                      batch_geometries, BATCH_S0, BATCH_HISTORIES)
from .geometry import (Grid, RayMap, Geometry, screen_raymaps, random_geometry, pairing_destroyed,  # noqa: F401
                       spatial_only, delay_only)
from .histories import uniform_emissivity, blob_histories, gaussian_block  # noqa: F401
