"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module draws random numbers and lays them out in memory. It holds none of
the solver's or the constitutive law's arithmetic: the only arithmetic here is
input construction (b = A @ x_true) and the spectral-condition filter that
decides which random matrices are kept.
"""
from .gen import (  # noqa: F401
    CHUNK,
    aos_to_soa,
    device_systems,
    mixed_systems,
    newton_points,
    serving_requests,
    special_matrices,
    systems,
)
