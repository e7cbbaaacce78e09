"""Seeded synthetic inputs shared by the oracle and the GPU path.

Nothing here computes any part of the decomposition method: these modules
only produce point clouds, kernel bandwidths and streams of uniform random
numbers, which are then handed to both implementations as plain arrays.
"""
from .philox import philox4x32_10, uniform_stream
from .torus import torus_points
from .ks import ks_trajectory, delay_embed, ks_points
from .bandwidth import median_sq_distance
from .batch import batch_specs, batch_points, BANDWIDTH_MULTIPLIERS
from .vsa import vsa_points, vsa_initial_field

__all__ = [
    "philox4x32_10",
    "uniform_stream",
    "torus_points",
    "ks_trajectory",
    "delay_embed",
    "ks_points",
    "median_sq_distance",
    "batch_specs",
    "batch_points",
    "BANDWIDTH_MULTIPLIERS",
    "vsa_points",
    "vsa_initial_field",
]
