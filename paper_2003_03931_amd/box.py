"""Python handle on one simulation box of libcube.so.

PyTorch supplies device memory and the stream; the library's HIP kernels do
all of the work.  Host inputs may be numpy arrays; device results come back as
torch tensors on the box's device.
"""

import ctypes

import numpy as np

from ._lib import ALLOC_FN, FREE_FN, Allocator, BoxDesc, Diag, StageStat, StateView, check, load

CUBE_FP32 = 0
CUBE_MIXED_BF16 = 1
CUBE_MIXED_FP16 = 2
PRECISIONS = {"fp32": CUBE_FP32, "bf16": CUBE_MIXED_BF16, "fp16": CUBE_MIXED_FP16}
CUBE_VEL_LINEAR = 0
CUBE_VEL_CELL_MEAN = 1


def desc_from(spec, with_ids=False, tiles_per_batch=0, precision=CUBE_FP32):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    return BoxDesc(int(spec.n_side), int(spec.tiles_per_dim), int(spec.fine_per_spacing),
                   int(spec.coarse_ratio), int(spec.buffer_fine), int(spec.r_cut_fine),
                   float(spec.dt), float(spec.v_headroom), int(precision), 1 if with_ids else 0,
                   int(tiles_per_batch), int(getattr(spec, "fd_order", 2)), int(getattr(spec, "vel_codec", 0)),
                   int(getattr(spec, "comoving", 0)), float(getattr(spec, "omega_m", 1.0)),
                   float(getattr(spec, "omega_l", 0.0)), float(getattr(spec, "a_start", 1.0)),
                   int(getattr(spec, "pp_range", 0)))


def footprint(spec, tiles_per_batch=0, precision=CUBE_FP32, with_ids=False):
    """(persistent, transient) device bytes of a box, from cube_footprint."""
    lib = load()
    d = desc_from(spec, with_ids, tiles_per_batch, precision)
    p, t = ctypes.c_int64(), ctypes.c_int64()
    check(lib.cube_footprint(ctypes.byref(d), ctypes.byref(p), ctypes.byref(t)))
    return p.value, t.value


class TorchAllocator:
    """cube_allocator callbacks backed by torch's caching allocator on one
    device; counts live bytes so that callers can check the library's
    footprint."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.peak = 0
        self.calls = 0

        def _alloc(user, nbytes, stream):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:
                return None
            self.live[ptr] = int(nbytes)
            self.calls += 1
            self.peak = max(self.peak, self.live_bytes())
            return ptr

        def _free(user, ptr, nbytes, stream):
            try:
                self.live.pop(int(ptr), None)
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = Allocator(self._alloc, self._free, None)

    def live_bytes(self):
        return sum(self.live.values())


class CubeBox:
    """One box: owns a cube_ctx.  `spec` carries the geometry fields of
    cube_box_desc (n_side, tiles_per_dim, fine_per_spacing, coarse_ratio,
    buffer_fine, r_cut_fine, dt, v_headroom, and optionally fd_order,
    vel_codec, the comoving fields comoving, omega_m, omega_l, a_start, and
    pp_range)."""

    def __init__(self, spec, with_ids=False, tiles_per_batch=0, device=0, precision=CUBE_FP32,
                 allocator="torch"):
        """allocator: "torch" (device memory from torch's caching allocator,
        the default) or "hip" (the library's own hipMalloc)."""
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.desc = desc_from(spec, with_ids, tiles_per_batch, precision)
        self.with_ids = with_ids
        self.allocator = TorchAllocator(self.device.index) if allocator == "torch" else None
        ctx = ctypes.c_void_p()
        al = ctypes.byref(self.allocator.struct) if self.allocator else None
        check(self.lib.cube_init(ctypes.byref(self.desc), al, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(ctx)))
        self.ctx = ctx
        self._owned = True
        self._set_sizes(spec)

    @classmethod
    def borrowed(cls, ctx, spec, with_ids=False, device=0):
        """A handle on a context owned elsewhere (an ensemble's box): the same
        calls, and close() leaves the context alone."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        self.stream = None
        self.desc = desc_from(spec, with_ids)
        self.with_ids = with_ids
        self.allocator = None
        self.ctx = ctx
        self._owned = False
        self._set_sizes(spec)
        return self

    def _set_sizes(self, spec):
        n = spec.n_side
        self.n = n ** 3
        nc = n * spec.fine_per_spacing // spec.coarse_ratio
        self.n_coarse = nc
        self.n_cells = nc ** 3
        T = n * spec.fine_per_spacing // spec.tiles_per_dim
        self.F = T if spec.tiles_per_dim == 1 else T + 2 * spec.buffer_fine
        self.vel_codec = int(getattr(spec, "vel_codec", 0))

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_owned", True) and self.ctx is not None and self.ctx.value:
            self.lib.cube_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --------------------------------------------------------------- codec
    def compress(self, pos, vel):
        t = self.torch
        if isinstance(pos, t.Tensor):
            p = pos.to(self.device, t.float32).contiguous()
            v = vel.to(self.device, t.float32).contiguous()
            check(self.lib.cube_compress(self.ctx, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                         self.n, 1))
        else:
            p = np.ascontiguousarray(pos, dtype=np.float32)
            v = np.ascontiguousarray(vel, dtype=np.float32)
            check(self.lib.cube_compress(self.ctx, p.ctypes.data_as(ctypes.c_void_p),
                                         v.ctypes.data_as(ctypes.c_void_p), self.n, 0))

    def decompress(self):
        t = self.torch
        pos = t.empty((self.n, 3), dtype=t.float32, device=self.device)
        vel = t.empty((self.n, 3), dtype=t.float32, device=self.device)
        check(self.lib.cube_decompress(self.ctx, ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()),
                                       self.n, 1))
        return pos, vel

    # ---------------------------------------------------------------- step
    def step(self, nsteps=1):
        check(self.lib.cube_pm_step(self.ctx, int(nsteps)))

    def forces(self):
        t = self.torch
        acc = t.empty((self.n, 3), dtype=t.float32, device=self.device)
        check(self.lib.cube_forces(self.ctx, ctypes.c_void_p(acc.data_ptr()), 1))
        return acc

    # --------------------------------------------------------------- state
    def get_state(self):
        """Host copy: dict(counts int32[N_c^3], m uint8[3,N], u int8[3,N], ids, s, M, step,
        vc float32[3, N_c^3] with the cell-mean velocity codec, else None)."""
        m = np.empty((3, self.n), dtype=np.uint8)
        u = np.empty((3, self.n), dtype=np.int8)
        counts = np.empty(self.n_cells, dtype=np.int32)
        ids = np.empty(self.n, dtype=np.uint32) if self.with_ids else None
        vc = np.empty((3, self.n_cells), dtype=np.float32) if self.vel_codec else None
        v = StateView()
        v.n_particles = self.n
        v.n_cells = self.n_cells
        for k in range(3):
            v.m[k] = m[k].ctypes.data
            v.u[k] = u[k].ctypes.data
            v.vc[k] = vc[k].ctypes.data if vc is not None else None
        v.counts = counts.ctypes.data
        v.ids = ids.ctypes.data if ids is not None else None
        v.on_device = 0
        check(self.lib.cube_get_state(self.ctx, ctypes.byref(v)))
        return {"counts": counts, "m": m, "u": u, "ids": ids, "s": v.s_v, "M": v.max_u, "step": v.step,
                "vc": vc}

    def set_state(self, counts, m, u, s, M, ids=None, step=0, vc=None):
        """vc: float32 (3, N_c^3) cell means, required with the cell-mean codec."""
        counts = np.ascontiguousarray(counts, dtype=np.int32)
        m = np.ascontiguousarray(m, dtype=np.uint8)
        u = np.ascontiguousarray(u, dtype=np.int8)
        v = StateView()
        v.n_particles = self.n
        v.n_cells = self.n_cells
        for k in range(3):
            v.m[k] = m[k].ctypes.data
            v.u[k] = u[k].ctypes.data
        v.counts = counts.ctypes.data
        keep = [counts, m, u]
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.uint32)
            keep.append(ids)
            v.ids = ids.ctypes.data
        else:
            v.ids = None
        if vc is not None:
            vc = np.ascontiguousarray(vc, dtype=np.float32)
            keep.append(vc)
            for k in range(3):
                v.vc[k] = vc[k].ctypes.data
        v.s_v = float(s)
        v.max_u = int(M)
        v.on_device = 0
        v.step = int(step)
        check(self.lib.cube_set_state(self.ctx, ctypes.byref(v)))

    # ----------------------------------------------------------- diagnostics
    def diagnostics(self):
        d = Diag()
        check(self.lib.cube_diagnostics(self.ctx, ctypes.byref(d)))
        return {"mass": d.mass, "momentum": np.array(d.momentum[:]), "kinetic": d.kinetic,
                "potential": d.potential, "saturations": d.saturations, "max_carry": d.max_carry,
                "max_u": d.max_u, "s": d.s_v, "step": d.step, "last_step_ms": d.last_step_ms}

    def power_spectrum(self):
        nb = int(round(self.n ** (1.0 / 3.0))) // 4 - 1
        k = np.zeros(nb)
        pk = np.zeros(nb)
        nm = np.zeros(nb, dtype=np.int64)
        check(self.lib.cube_power_spectrum(self.ctx, nb, k.ctypes.data_as(ctypes.c_void_p),
                                           pk.ctypes.data_as(ctypes.c_void_p), nm.ctypes.data_as(ctypes.c_void_p)))
        return k, pk, nm

    def profile(self, enable=True):
        check(self.lib.cube_profile_enable(self.ctx, 1 if enable else 0))

    def profile_read(self):
        """[{name, launches, total_ms, bytes}] per stage of cube_pm_step."""
        buf = (StageStat * 32)()
        n = ctypes.c_int32()
        check(self.lib.cube_profile_read(self.ctx, buf, 32, ctypes.byref(n)))
        return [{"name": buf[i].name.decode(), "launches": buf[i].launches, "total_ms": buf[i].total_ms,
                 "bytes": buf[i].bytes} for i in range(n.value)]

    def debug_force(self, what, count=1):
        """Test hook: 1 FP16 range flag, 2 sorted compaction, 3 re-plan, for the next `count` steps."""
        check(self.lib.cube_debug_force(self.ctx, int(what), int(count)))

    def debug_mesh(self, what, tile=0):
        t = self.torch
        side = self.n_coarse if what in (0, 1) else self.F
        out = t.empty((side, side, side), dtype=t.float32, device=self.device)
        check(self.lib.cube_debug_mesh(self.ctx, int(what), int(tile), ctypes.c_void_p(out.data_ptr())))
        return out


def fft3d(data, inverse=False):
    """In-place 3-D complex FFT of a (n, n, n) complex64 cuda tensor ([z][y][x])."""
    import torch
    assert data.dtype == torch.complex64 and data.is_cuda and data.is_contiguous()
    n = data.shape[0]
    stream = torch.cuda.current_stream(data.device)
    check(load().cube_fft3d(int(n), ctypes.c_void_p(data.data_ptr()), 1 if inverse else 0,
                            ctypes.c_void_p(stream.cuda_stream)))
    return data
