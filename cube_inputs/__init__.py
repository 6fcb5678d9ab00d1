"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This package holds workload parameters and the seeded initial-condition
generator only.  It contains none of the particle-mesh step's arithmetic
(no codec, no deposit, no FFT solve, no integrator): both the HIP library and
the CPU oracle receive the float arrays produced here and apply their own,
independent encoders to them.
"""

from .configs import BoxSpec, CONFIGS, config
from .zeldovich import zeldovich_ics, plane_wave_ics

__all__ = ["BoxSpec", "CONFIGS", "config", "zeldovich_ics", "plane_wave_ics"]
