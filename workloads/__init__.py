"""Seeded synthetic point clouds shared by the tests, the bench and the oracle runs.

This package only draws random numbers and lays them out as float64 arrays.  It holds
none of the clustering arithmetic, so both the CPU oracle and the GPU path can be fed
from it without sharing any part of the method.
"""

from .generators import (  # noqa: F401
    SEED_BASE,
    Instance,
    blobs_2d,
    config_workload,
    gaussian_mixture,
    gaussian_mixture_hd,
    multi_cloud_batch,
    seed_spreader_3d,
)
