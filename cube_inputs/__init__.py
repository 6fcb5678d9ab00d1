"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This package holds workload parameters and seeded generators only.  It
contains none of the particle-mesh step's arithmetic (no codec, no deposit,
no FFT solve, no integrator): both the HIP library and the CPU oracle receive
the float arrays produced here and apply their own, independent encoders to
them.  The one exception to float inputs is lattice_run_state, which lays out
a compressed state byte by byte (a fixed lattice plus random runs) for tests
at sizes where the oracle cannot encode a billion particles in seconds.
"""

from .configs import BoxSpec, CONFIGS, config, served_box
from .lattice import lattice_run_state
from .zeldovich import zeldovich_ics, zeldovich_ics_device, plane_wave_ics

__all__ = ["BoxSpec", "CONFIGS", "config", "served_box", "zeldovich_ics", "zeldovich_ics_device", "plane_wave_ics", "lattice_run_state"]
