"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only *generates* inputs (positions, velocities, parameters,
topologies). It holds none of the method's arithmetic: no neighbour search,
no energies or forces, no Ewald parameters, no integration.
"""
from .systems import (  # noqa: F401
    System,
    lj_fluid,
    water_box,
    random_box,
    lj_fluid_n,
    batch_replicas,
    smooth_grid_size,
    config_system,
    CONFIGS,
)
