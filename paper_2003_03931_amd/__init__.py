"""MI355X-native CUBE two-level particle-mesh step (arXiv:2003.03931).

The compute path is the HIP library ``libcube.so`` (C ABI in include/cube.h);
this package only marshals arguments to it.
"""

from ._lib import CubeError, load, LIB_PATH, SIGNATURES
from .box import (CubeBox, fft3d, desc_from, footprint, CUBE_FP32, CUBE_MIXED_BF16, CUBE_MIXED_FP16,
                  CUBE_VEL_LINEAR, CUBE_VEL_CELL_MEAN)
from .server import CubeServer
from .ensemble import CubeEnsemble

__all__ = ["CubeBox", "CubeServer", "CubeEnsemble", "CubeError", "fft3d", "footprint", "load", "desc_from", "LIB_PATH",
           "SIGNATURES", "CUBE_FP32", "CUBE_MIXED_BF16", "CUBE_MIXED_FP16", "CUBE_VEL_LINEAR",
           "CUBE_VEL_CELL_MEAN"]
