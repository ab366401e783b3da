"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only *draws* inputs: mesh vertex positions and connectivity,
land masks and random fields. It holds none of the filter's arithmetic
(no areas, no Laplacian weights, no solves), so the oracle and the HIP
library can both consume its output without sharing any of the method.
"""
from .mesh import (
    Mesh,
    GEOM_PLANAR,
    GEOM_PERIODIC,
    GEOM_SPHERE,
    split_square,
    icosphere,
    land_mask,
    edge_length_scale,
)
from .fields import (
    planar_k3_field,
    planar_mode_field,
    planar_k3_velocity,
    sphere_k3_field,
    sphere_k3_velocity,
    log_scales,
)

__all__ = [
    "Mesh",
    "GEOM_PLANAR",
    "GEOM_PERIODIC",
    "GEOM_SPHERE",
    "split_square",
    "icosphere",
    "land_mask",
    "edge_length_scale",
    "planar_k3_field",
    "planar_mode_field",
    "planar_k3_velocity",
    "sphere_k3_field",
    "sphere_k3_velocity",
    "log_scales",
]
