"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the propagation method: it only draws
bit patterns, builds Gaussian pulse trains on a periodic time grid and
describes the dispersion-managed maps and grid sizes of the workloads.
"""
from .wdm import (DMMap, Grid, MPASettings, Workload, dm_map, wdm_field,
                  workload, WORKLOADS)

__all__ = ["DMMap", "Grid", "MPASettings", "Workload", "dm_map", "wdm_field",
           "workload", "WORKLOADS"]
