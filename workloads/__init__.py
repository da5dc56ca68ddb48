"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds no arithmetic of the method: it only draws orbital
energies, RI coefficients and frequency grids.  Both `oracle/` (the CPU
reference) and the GPU binding consume what it produces; neither imports
the other.
"""
from .configs import CONFIGS, EV_PER_HA, WorkloadConfig, serving_request_config
from .generate import System, make_system, make_vv, mgl_grid, system_from_config, vv_block

__all__ = [
    "CONFIGS",
    "EV_PER_HA",
    "WorkloadConfig",
    "System",
    "make_system",
    "make_vv",
    "mgl_grid",
    "serving_request_config",
    "system_from_config",
    "vv_block",
]
