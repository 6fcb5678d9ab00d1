"""FP64 CPU oracle of the CUBE two-level particle-mesh (PMPM) step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or runs
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and imports nothing from it.

It is a plain, slow, step-by-step implementation of the method of
Cheng et al., "CUBE -- Towards an Optimal Scaling of Cosmological N-body
Simulations" (arXiv:2003.03931):

* Sec. II: force split F_G = F_s + F_l, PM convolution Eq. (1), a global coarse
  mesh for the long-range force and per-tile fine meshes (tile plus buffer) for
  the short-range force; optionally the extended PP force between close pairs
  with the fine kernel corrected to match (pp.py).
* Sec. III-A: fixed-point compression -- positions as a 1-byte offset inside the
  parent coarse cell (Eq. (2)), cell-ordered storage with a per-cell count;
  optionally velocities as cell means plus companded bytes (Eq. (3)) with the
  fast arctangent of Eq. (4).

Where the paper is silent the oracle follows numbered readings R1-R22 (units,
codec details, CIC, Green's functions, integrator, drift, compaction order);
each module's header states the ones it takes.  Every floating-point step runs in float64.

Parity status of each function is stated in its module header; the pins live
in ``tests/test_oracle_*.py``.
"""

from .geometry import Box
from . import codec, cic, green, pm, pp, step, diag, ewald, float_mode, vcodec, cosmo

__all__ = ["Box", "codec", "cic", "green", "pm", "pp", "step", "diag", "ewald",
           "float_mode", "vcodec", "cosmo"]
