"""MI355X-native CUBE two-level particle-mesh step (arXiv:2003.03931).

The compute path is the HIP library ``libcube.so`` (C ABI in include/cube.h);
this package only marshals arguments to it.
"""

from ._lib import CubeError, load, LIB_PATH, SIGNATURES
from .box import CubeBox, fft3d, desc_from

__all__ = ["CubeBox", "CubeError", "fft3d", "load", "desc_from", "LIB_PATH", "SIGNATURES"]
