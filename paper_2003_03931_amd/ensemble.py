"""Python handle on a batched ensemble of boxes (cube_ensemble_* of libcube.so).

Argument marshalling only: the library's kernels do the work.  Each box is
reachable as a CubeBox handle (compress, set_state, get_state, diagnostics)
on a context the ensemble owns.
"""

import ctypes

from ._lib import BoxDesc, EnsembleDesc, check, load
from .box import CubeBox, desc_from


class CubeEnsemble:
    def __init__(self, specs, streams=0, tiles_in_flight=0, use_graph=True, with_ids=False, precision=0,
                 device=0):
        """specs: box specs (the fields of cube_box_desc).  streams and
        tiles_in_flight 0: chosen by the library's autotuner."""
        import torch
        torch.cuda.set_device(device)
        self.lib = load()
        self.specs = list(specs)
        arr = (BoxDesc * len(self.specs))(*[desc_from(s, with_ids, 0, precision) for s in self.specs])
        opts = EnsembleDesc(int(streams), int(tiles_in_flight), 0 if use_graph else -1, int(device))
        h = ctypes.c_void_p()
        check(self.lib.cube_ensemble_create(arr, len(self.specs), ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h
        self.boxes = []
        for i, s in enumerate(self.specs):
            c = ctypes.c_void_p()
            check(self.lib.cube_ensemble_box(h, i, ctypes.byref(c)))
            self.boxes.append(CubeBox.borrowed(c, s, with_ids=with_ids, device=device))

    def step(self, nsteps=1):
        check(self.lib.cube_ensemble_step(self.handle, int(nsteps)))

    def tune(self):
        d = EnsembleDesc()
        check(self.lib.cube_ensemble_tune(self.handle, ctypes.byref(d)))
        return {"streams": d.streams, "tiles_in_flight": d.tiles_in_flight}

    def schedule(self):
        d = EnsembleDesc()
        check(self.lib.cube_ensemble_schedule(self.handle, ctypes.byref(d)))
        return {"streams": d.streams, "tiles_in_flight": d.tiles_in_flight, "use_graph": d.use_graph == 0}

    def close(self):
        if self.handle is not None and self.handle.value:
            for b in self.boxes:
                b.ctx = None
            self.lib.cube_ensemble_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
