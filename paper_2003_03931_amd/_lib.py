"""ctypes binding of libcube.so (the C ABI declared in include/cube.h).

Argument marshalling only: every stage of the particle-mesh step runs in the
library's HIP kernels.  Importing this module fails loudly if the shared
library has not been built; there is no fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcube.so")

CUBE_OK = 0
STATUS = {0: "OK", 1: "INVALID", 2: "OOM", 3: "DEVICE", 4: "NOT_READY", 5: "OVERFLOW", 6: "UNSUPPORTED"}


class CubeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cube status {STATUS.get(status, status)}: {msg}")
        self.status = status


class BoxDesc(ctypes.Structure):
    _fields_ = [
        ("n_side", ctypes.c_int32),
        ("tiles_per_dim", ctypes.c_int32),
        ("fine_per_spacing", ctypes.c_int32),
        ("coarse_ratio", ctypes.c_int32),
        ("buffer_fine", ctypes.c_int32),
        ("r_cut_fine", ctypes.c_int32),
        ("dt", ctypes.c_float),
        ("v_headroom", ctypes.c_float),
        ("precision", ctypes.c_int32),
        ("with_ids", ctypes.c_int32),
        ("tiles_per_batch", ctypes.c_int32),
        ("fd_order", ctypes.c_int32),
        ("vel_codec", ctypes.c_int32),
        ("comoving", ctypes.c_int32),
        ("omega_m", ctypes.c_float),
        ("omega_l", ctypes.c_float),
        ("a_start", ctypes.c_float),
        ("pp_range", ctypes.c_int32),
    ]


class StateView(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int64),
        ("n_cells", ctypes.c_int64),
        ("m", ctypes.c_void_p * 3),
        ("u", ctypes.c_void_p * 3),
        ("counts", ctypes.c_void_p),
        ("ids", ctypes.c_void_p),
        ("s_v", ctypes.c_double),
        ("max_u", ctypes.c_int32),
        ("on_device", ctypes.c_int32),
        ("step", ctypes.c_int64),
        ("vc", ctypes.c_void_p * 3),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_int64),
        ("momentum", ctypes.c_double * 3),
        ("kinetic", ctypes.c_double),
        ("potential", ctypes.c_double),
        ("saturations", ctypes.c_int64),
        ("max_carry", ctypes.c_int32),
        ("max_u", ctypes.c_int32),
        ("s_v", ctypes.c_double),
        ("step", ctypes.c_int64),
        ("last_step_ms", ctypes.c_double),
    ]


class StageStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class ServerDesc(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("desc", BoxDesc),
        ("n_steps", ctypes.c_int32),
        ("want_diag", ctypes.c_int32),
        ("pos", ctypes.c_void_p),
        ("vel", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("out_state", ctypes.POINTER(StateView)),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("steps_done", ctypes.c_int64),
        ("footprint_bytes", ctypes.c_int64),
        ("submit_ms", ctypes.c_double),
        ("start_ms", ctypes.c_double),
        ("done_ms", ctypes.c_double),
        ("diag", Diag),
        ("message", ctypes.c_char * 160),
    ]


class EnsembleDesc(ctypes.Structure):
    _fields_ = [
        ("streams", ctypes.c_int32),
        ("tiles_in_flight", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("device", ctypes.c_int32),
    ]


# exported symbol -> (restype, argtypes); mirrors include/cube.h
SIGNATURES = {
    "cube_last_error": (ctypes.c_char_p, []),
    "cube_init": (ctypes.c_int, [ctypes.POINTER(BoxDesc), ctypes.POINTER(Allocator), ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "cube_footprint": (ctypes.c_int, [ctypes.POINTER(BoxDesc), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "cube_destroy": (None, [ctypes.c_void_p]),
    "cube_compress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int32]),
    "cube_decompress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_int32]),
    "cube_pm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cube_pm_step_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cube_forces": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "cube_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StateView)]),
    "cube_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StateView)]),
    "cube_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Diag)]),
    "cube_power_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "cube_debug_mesh": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "cube_debug_force": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "cube_fft3d": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cube_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cube_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StageStat), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "cube_server_create": (ctypes.c_int, [ctypes.POINTER(ServerDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "cube_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "cube_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "cube_server_destroy": (None, [ctypes.c_void_p]),
    "cube_ensemble_create": (ctypes.c_int, [ctypes.POINTER(BoxDesc), ctypes.c_int32, ctypes.POINTER(EnsembleDesc),
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "cube_ensemble_box": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "cube_ensemble_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cube_ensemble_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(EnsembleDesc)]),
    "cube_ensemble_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(EnsembleDesc)]),
    "cube_ensemble_destroy": (None, [ctypes.c_void_p]),
}

_lib = None


def load():
    """Load libcube.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != CUBE_OK:
        msg = load().cube_last_error()
        raise CubeError(status, msg.decode() if msg else "")
