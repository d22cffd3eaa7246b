"""Seeded synthetic inputs for the FCC-film Ising workloads.

This package produces *inputs only*: surface height maps, field ramps,
temperature schedules, batched-film and serving-request descriptions.  It
holds none of the Monte Carlo arithmetic (no neighbour sums, no acceptance
rule, no random-number generator of the dynamics), so both the CPU oracle
and the GPU library may consume what it produces.

The paper builds its spin lattice from STM/AFM raster images (Sections 2-3);
those images are not available, so seeded Gaussian-blurred noise height maps
stand in for them.
"""

from .heightmap import height_map, occupancy_count
from .configs import (
    PlainConfig,
    config_plain_hysteresis_small,
    config_plain_tscan,
    config_plain_hysteresis_large,
    batched_films,
    BatchedReplica,
    serving_requests,
    ServeRequest,
    ramp_hnum,
    tscan_temperatures,
)

__all__ = [
    "height_map",
    "occupancy_count",
    "PlainConfig",
    "config_plain_hysteresis_small",
    "config_plain_tscan",
    "config_plain_hysteresis_large",
    "batched_films",
    "BatchedReplica",
    "serving_requests",
    "ServeRequest",
    "ramp_hnum",
    "tscan_temperatures",
]
