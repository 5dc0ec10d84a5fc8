"""Seeded synthetic event sets shaped like the paper's county-level case data.

This module only draws inputs (times, locations, county ids, county rectangles,
per-event bandwidth scales).  It holds none of the likelihood arithmetic, so the
CPU oracle and the GPU path can both read its output without sharing any of the
method's code.
"""

from .events import N1M, N2K, N100K, WORKLOADS, EventSet, WorkloadConfig, generate, generate_clustered, theta_default

__all__ = ["N1M", "N2K", "N100K", "WORKLOADS", "EventSet", "WorkloadConfig", "generate", "generate_clustered",
           "theta_default"]
