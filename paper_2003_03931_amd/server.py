"""Python handle on the library's box server (cube_server_* in include/cube.h).

Requests are independent boxes given as float positions and velocities; the
server admits them first-in first-out against an HBM budget and runs up to
max_slots of them at once, each on its own stream and context.  Argument
marshalling only: admission, scheduling and every step run in libcube.so.
"""

import ctypes
import time

import numpy as np

from ._lib import Request, Result, ServerDesc, StateView, check, load
from .box import desc_from

CUBE_NOT_READY = 4


class CubeServer:
    def __init__(self, hbm_budget_bytes, max_slots=2, precision=-1, device=0):
        self.lib = load()
        d = ServerDesc(int(hbm_budget_bytes), int(max_slots), int(precision), int(device), 0)
        ptr = ctypes.c_void_p()
        check(self.lib.cube_server_create(ctypes.byref(d), ctypes.byref(ptr)))
        self.ptr = ptr
        self._held = {}          # ticket -> what the request points at

    def submit(self, spec, pos, vel, n_steps, precision=0, tiles_per_batch=0, want_diag=False, want_state=False):
        """Queue one box; returns its ticket.  pos/vel: (n, 3) float arrays."""
        pos = np.ascontiguousarray(pos, dtype=np.float32)
        vel = np.ascontiguousarray(vel, dtype=np.float32)
        n = spec.n_side ** 3
        held = {"pos": pos, "vel": vel}
        view = None
        if want_state:
            nc = (spec.n_side * spec.fine_per_spacing // spec.coarse_ratio) ** 3
            m = [np.empty(n, np.uint8) for _ in range(3)]
            u = [np.empty(n, np.int8) for _ in range(3)]
            counts = np.empty(nc, np.int32)
            view = StateView()
            view.n_particles, view.n_cells = n, nc
            for k in range(3):
                view.m[k] = m[k].ctypes.data
                view.u[k] = u[k].ctypes.data
            view.counts = counts.ctypes.data
            view.ids = None
            view.on_device = 0
            held.update(m=m, u=u, counts=counts, view=view)
        req = Request(desc_from(spec, False, tiles_per_batch, precision), int(n_steps), 1 if want_diag else 0,
                      pos.ctypes.data, vel.ctypes.data, n, ctypes.pointer(view) if view is not None else None)
        held["req"] = req
        t = ctypes.c_uint64()
        check(self.lib.cube_submit(self.ptr, ctypes.byref(req), ctypes.byref(t)))
        self._held[t.value] = held
        return t.value

    def poll(self, ticket):
        """None while queued or running; else a dict with the result (and the
        final state when it was asked for)."""
        r = Result()
        st = self.lib.cube_poll(self.ptr, ctypes.c_uint64(ticket), ctypes.byref(r))
        if st == CUBE_NOT_READY:
            return None
        check(st)
        held = self._held.pop(ticket)
        out = {
            "status": r.status, "steps_done": r.steps_done, "footprint_bytes": r.footprint_bytes,
            "submit_ms": r.submit_ms, "start_ms": r.start_ms, "done_ms": r.done_ms,
            "message": r.message.decode(errors="replace"),
            "diag": {"mass": r.diag.mass, "momentum": tuple(r.diag.momentum), "kinetic": r.diag.kinetic,
                     "potential": r.diag.potential, "max_u": r.diag.max_u, "s_v": r.diag.s_v},
        }
        if "view" in held:
            v = held["view"]
            out["state"] = {"m": held["m"], "u": held["u"], "counts": held["counts"], "s_v": v.s_v,
                            "max_u": v.max_u, "step": v.step}
        return out

    def wait(self, ticket, poll_s=0.002):
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            time.sleep(poll_s)

    def close(self):
        if self.ptr is not None and self.ptr.value:
            self.lib.cube_server_destroy(self.ptr)
        self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
