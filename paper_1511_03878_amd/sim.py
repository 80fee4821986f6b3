"""Thin Python binding over the C ABI (include/pic.h): argument marshalling only.

Every step of the PIC path runs in the HIP kernels of libpic.so.  PyTorch is
used for plumbing: device memory comes from torch's caching allocator through
the library's allocator hook, and work is ordered on torch's current HIP
stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _capi
from ._capi import check

_D = C.POINTER(C.c_double)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# Handles still open at interpreter exit are closed by an exit hook: their
# device memory goes back through torch's allocator, which must still be
# there (module teardown would otherwise run the frees after torch is gone).
# The hook is registered after torch is loaded, so it runs before torch's own.
_LIVE_BATCHES: "weakref.WeakSet" = weakref.WeakSet()
_LIVE_SIMS: "weakref.WeakSet" = weakref.WeakSet()
_exit_hook = False


def _close_all():
    for b in list(_LIVE_BATCHES):
        b.close()
    for s in list(_LIVE_SIMS):
        s.close()


def _track(registry, obj):
    global _exit_hook
    if not _exit_hook:
        atexit.register(_close_all)
        _exit_hook = True
    registry.add(obj)


class _TorchAllocator:
    """Allocator hook that routes device allocations to torch's caching allocator."""

    def __init__(self, stream_handle: int):
        import torch
        self._torch = torch
        self._stream = stream_handle
        self._dev = torch.cuda.current_device()

        def _alloc(nbytes, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self._dev, self._stream))
            except Exception:  # out of memory: report NULL to the library
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._cb_alloc = _capi.ALLOC_FN(_alloc)
        self._cb_free = _capi.FREE_FN(_free)
        self.struct = _capi.Allocator(self._cb_alloc, self._cb_free, None)


def current_stream_handle() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def make_desc(grid: dict, precision: int, chunk: int = 0, block: int = 0,
              capacity_factor: float = 0.0, min_capacity: int = 0,
              field_tile: int = 0, lane_stride: int = 0, graph: int = 0,
              patch_order: int = 0, maxwell_order: int = 0, deterministic: int = 0) -> _capi.SimDesc:
    nd = int(grid["ndim"])
    n = list(grid["n"]) + [1] * (3 - len(grid["n"]))
    d = list(grid["d"]) + [1.0] * (3 - len(grid["d"]))
    patch = list(grid["patch"]) + [1] * (3 - len(grid["patch"]))
    per = list(grid.get("periodic", [1, 1, 1])) + [1] * 3
    return _capi.SimDesc(nd, int(precision), (C.c_int32 * 3)(*n), (C.c_double * 3)(*d),
                         float(grid["dt"]), (C.c_int32 * 3)(*patch),
                         (C.c_int32 * 3)(*[int(p) for p in per[:3]]),
                         float(grid.get("q", -1.0)), float(grid.get("m", 1.0)),
                         float(capacity_factor), int(min_capacity), int(chunk), int(block),
                         int(field_tile), int(lane_stride), int(graph), int(patch_order),
                         int(maxwell_order), int(deterministic))


def estimate_bytes(grid: dict, precision: int, nparticles: int, laser_steps: int = 0,
                   **tune) -> int:
    """Device bytes a simulation is expected to allocate (host-only query)."""
    out = C.c_int64()
    desc = make_desc(grid, precision, **tune)
    check(_capi.load().pic_estimate_bytes(C.byref(desc), int(nparticles), int(laser_steps),
                                          C.byref(out)))
    return out.value


def species_desc(sp: dict) -> _capi.SpeciesDesc:
    from .workloads import LOADINGS, PROFILES
    return _capi.SpeciesDesc(float(sp.get("q", -1.0)), float(sp.get("m", 1.0)),
                             PROFILES[sp["profile"]], LOADINGS[sp.get("loading", "weight")],
                             int(sp["ppc"]), 0, float(sp.get("n0", 1.0)),
                             (C.c_double * 6)(*(list(sp.get("param", [])) + [0.0] * 6)[:6]),
                             float(sp.get("temperature", 0.0)), int(sp.get("seed", 0)) & (2 ** 64 - 1))


def laser_desc(laser: dict) -> _capi.LaserDesc:
    return _capi.LaserDesc(float(laser["a0"]), float(laser.get("omega0", 1.0)), float(laser["w0"]),
                           float(laser["tau"]), float(laser["t0"]), float(laser["x_focus"]),
                           float(laser["y_center"]), float(laser.get("phase", 0.0)),
                           int(laser.get("polarisation", 1)), 0)


def _tune_dict(r) -> dict:
    return {k: (list(getattr(r, k)) if k == "patch" else getattr(r, k)) for k, _ in _capi.TuneResult._fields_}


def autotune_patch(wl: dict, precision: int, candidates=(16, 32), warm: int = 20, steps: int = 20,
                   cache: str | None = None, **tune):
    """Pick the patch edge (and particle-kernel workgroup size) for a workload
    described by a species (pic_autotune_patch): temporary simulations at each
    candidate are loaded on the device and timed.  Returns (grid with the
    chosen patch, tune settings to pass to Sim, the tuner's result)."""
    desc = make_desc(wl["grid"], precision, **tune)
    sp = species_desc(wl["species"])
    las = laser_desc(wl["laser"]) if wl.get("laser") and "a0" in wl["laser"] else None
    cand = (C.c_int32 * len(candidates))(*[int(c) for c in candidates])
    stream = current_stream_handle()
    alloc = _TorchAllocator(stream)
    r = _capi.TuneResult()
    check(_capi.load().pic_autotune_patch(C.byref(desc), C.byref(sp), C.byref(las) if las else None, cand,
                                          len(candidates), int(warm), int(steps), C.byref(alloc.struct),
                                          C.c_void_p(stream), cache.encode() if cache else None,
                                          C.byref(r)))
    grid = dict(wl["grid"])
    grid["patch"] = list(desc.patch)[:int(wl["grid"]["ndim"])]
    return grid, {"block": int(desc.block)}, _tune_dict(r)


def patch_order(np_) -> np.ndarray:
    """Patch ids in Hilbert-curve order for a grid of np_ patches per axis
    (pic_patch_order)."""
    nd = len(np_)
    p = (C.c_int32 * 3)(*(list(int(v) for v in np_) + [1] * (3 - nd)))
    n = int(np.prod(np_))
    out = np.empty(n, dtype=np.int32)
    check(_capi.load().pic_patch_order(nd, p, out.ctypes.data_as(C.POINTER(C.c_int32)), n))
    return out


def curve_segments(costs, k: int) -> np.ndarray:
    """Segment boundaries (k + 1 entries) of a cost sequence in curve order
    (pic_curve_segments)."""
    c = np.ascontiguousarray(costs, dtype=np.int64)
    out = np.empty(int(k) + 1, dtype=np.int64)
    check(_capi.load().pic_curve_segments(c.ctypes.data_as(C.POINTER(C.c_int64)), c.size, int(k),
                                          out.ctypes.data_as(C.POINTER(C.c_int64))))
    return out


class Sim:
    """One simulation on the GPU (a handle of the C library)."""

    def __init__(self, grid: dict, precision: int = 64, stream: int | None = None,
                 torch_alloc: bool = True, **tune):
        lib = _capi.load()
        self.grid = dict(grid)
        self.precision = int(precision)
        self.stream = current_stream_handle() if stream is None else int(stream)
        self._alloc = _TorchAllocator(self.stream) if torch_alloc else None
        desc = make_desc(grid, precision, **tune)
        h = C.c_void_p()
        check(lib.pic_sim_create(C.byref(desc), C.byref(self._alloc.struct) if self._alloc else None,
                                 C.c_void_p(self.stream), C.byref(h)))
        self._h = h
        _track(_LIVE_SIMS, self)
        self.ndim = int(grid["ndim"])
        n = list(grid["n"])
        per = list(grid.get("periodic", [1] * self.ndim))
        self.fn = [n[a] if per[a] else n[a] + 1 for a in range(self.ndim)] + [1] * (3 - self.ndim)
        self.npatch = int(np.prod([n[a] // grid["patch"][a] for a in range(self.ndim)]))

    @property
    def handle(self):
        return self._h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _capi.load().pic_sim_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state in ----------------------------------------------------------
    def set_particles(self, x, u, w):
        x = [_f64(a) for a in x]
        u = [_f64(a) for a in u]
        w = _f64(w)
        n = w.size
        check(_capi.load().pic_particles_set(self._h, n, _dp(x[0]), _dp(x[1]),
                                             _dp(x[2]) if self.ndim == 3 else None,
                                             _dp(u[0]), _dp(u[1]), _dp(u[2]), _dp(w)))

    def add_species(self, sp: dict) -> int:
        """Describe the species (pic_species_add); see workloads.species."""
        d = species_desc(sp)
        sid = C.c_int32()
        check(_capi.load().pic_species_add(self._h, C.byref(d), C.byref(sid)))
        return sid.value

    def particles_init(self, sid: int = 0):
        """Generate the species' particles on the device (pic_particles_init)."""
        check(_capi.load().pic_particles_init(self._h, int(sid)))

    def add_laser(self, laser: dict):
        """Gaussian laser through x = 0 (pic_laser_add); see workloads.gaussian_laser."""
        d = laser_desc(laser)
        check(_capi.load().pic_laser_add(self._h, C.byref(d)))

    def set_laser(self, ey=None, ez=None):
        ey, ez = _f64(ey), _f64(ez)
        nsteps = (ey if ey is not None else ez).shape[0]
        check(_capi.load().pic_laser_set(self._h, nsteps, _dp(ey), _dp(ez)))

    def set_step(self, step: int):
        """Completed-step counter of a state loaded from elsewhere (pic_step_set)."""
        check(_capi.load().pic_step_set(self._h, int(step)))

    def set_field(self, comp, values):
        c = _capi.COMPONENTS.index(comp) if isinstance(comp, str) else int(comp)
        v = _f64(np.asarray(values).reshape(-1))
        check(_capi.load().pic_fields_set(self._h, c, _dp(v), v.size))

    def set_merge(self, every: int, cell_max: int = 16, iterations: int = 8):
        """Merge crowded cells after every `every`-th step (0: never); pic_merge_set."""
        check(_capi.load().pic_merge_set(self._h, int(every), int(cell_max), int(iterations)))

    def merge(self, cell_max: int = 16, iterations: int = 8) -> int:
        """One merge pass now (pic_merge); returns the particles taken out."""
        t = C.c_int64()
        check(_capi.load().pic_merge(self._h, int(cell_max), int(iterations), C.byref(t)))
        return t.value

    def set_window(self, start: int, velocity: float, ppc, density):
        """Moving window along x (pic_window_set): jumps of one patch column,
        cold plasma of density[global column] injected at ppc = (ppc_x, ppc_y)."""
        d = _f64(np.atleast_1d(density))
        check(_capi.load().pic_window_set(self._h, int(start), float(velocity), int(ppc[0]),
                                          int(ppc[1]), _dp(d), d.size))

    @classmethod
    def from_workload(cls, wl: dict, precision: int = 64, **kw) -> "Sim":
        """A simulation of a workload: explicit particle arrays (x, u, w) when
        the workload holds them, else the species description loaded on the
        device; a laser description is added, an incident-field table set."""
        s = cls(wl["grid"], precision, **kw)
        if "x" in wl:
            s.set_particles(wl["x"], wl["u"], wl["w"])
        else:
            s.add_species(wl["species"])
            s.particles_init()
        laser = wl.get("laser")
        if laser:
            if "a0" in laser:
                s.add_laser(laser)
            else:
                s.set_laser(laser.get("ey"), laser.get("ez"))
        return s

    # -- stepping ------------------------------------------------------------
    def step(self, nsteps: int = 1):
        check(_capi.load().pic_step(self._h, int(nsteps)))

    def sync(self):
        check(_capi.load().pic_sync(self._h))

    # -- state out -------------------------------------------------------------
    def field(self, comp) -> np.ndarray:
        c = _capi.COMPONENTS.index(comp) if isinstance(comp, str) else int(comp)
        out = np.zeros(self.fn[0] * self.fn[1] * self.fn[2])
        check(_capi.load().pic_fields_get(self._h, c, _dp(out), out.size))
        if self.ndim == 3:
            return out.reshape(self.fn[2], self.fn[1], self.fn[0])
        return out.reshape(self.fn[1], self.fn[0])

    def num_particles(self) -> int:
        n = C.c_int64()
        check(_capi.load().pic_num_particles(self._h, C.byref(n)))
        return n.value

    def particles(self):
        """(x[ndim], u[3], w, id) in canonical (patch, slot) order, positions global."""
        n = self.num_particles()
        x = [np.zeros(n) for _ in range(self.ndim)]
        u = [np.zeros(n) for _ in range(3)]
        w = np.zeros(n)
        ids = np.zeros(n, dtype=np.int64)
        check(_capi.load().pic_particles_get(
            self._h, _dp(x[0]), _dp(x[1]), _dp(x[2]) if self.ndim == 3 else None,
            _dp(u[0]), _dp(u[1]), _dp(u[2]), _dp(w),
            ids.ctypes.data_as(C.POINTER(C.c_int64)), n))
        return x, u, w, ids

    def device_bytes(self) -> int:
        """Device memory the handle holds now (pic_device_bytes, no sync)."""
        b = C.c_int64()
        check(_capi.load().pic_device_bytes(self._h, C.byref(b)))
        return b.value

    def perm(self) -> np.ndarray:
        """Particle ids in canonical (patch, slot) order (pic_perm_get)."""
        n = self.num_particles()
        ids = np.zeros(n, dtype=np.int64)
        check(_capi.load().pic_perm_get(self._h, ids.ctypes.data_as(C.POINTER(C.c_int64)), n))
        return ids

    def counts(self) -> np.ndarray:
        c = np.zeros(self.npatch, dtype=np.int32)
        check(_capi.load().pic_patch_counts_get(self._h, c.ctypes.data_as(C.POINTER(C.c_int32)),
                                                c.size))
        return c

    def diag(self) -> dict:
        d = _capi.Diag()
        check(_capi.load().pic_diag_get(self._h, C.byref(d)))
        return {k: getattr(d, k) for k, _ in _capi.Diag._fields_}

    def residuals(self) -> dict:
        """Gauss and continuity residuals of the current state (pic_residuals);
        the continuity entry is NaN unless the previous call was one step earlier."""
        r = _capi.Residuals()
        check(_capi.load().pic_residuals(self._h, C.byref(r)))
        return {k: getattr(r, k) for k, _ in _capi.Residuals._fields_}

    def history(self, first: int, n: int):
        U = np.zeros(n)
        K = np.zeros(n)
        P = np.zeros(n, dtype=np.int64)
        check(_capi.load().pic_history_get(self._h, int(first), int(n), _dp(U), _dp(K),
                                           P.ctypes.data_as(C.POINTER(C.c_int64))))
        return U, K, P

    def autotune(self, steps: int = 10, cache: str | None = None) -> dict:
        """Pick the fastest launch settings for this simulation (its state is
        restored afterwards); with a cache file, reuse a stored choice."""
        r = _capi.TuneResult()
        check(_capi.load().pic_autotune(self._h, int(steps),
                                        cache.encode() if cache else None, C.byref(r)))
        return _tune_dict(r)

    def save_state(self) -> bytes:
        """Checkpoint of the whole simulation state (host bytes)."""
        lib = _capi.load()
        n = C.c_size_t()
        check(lib.pic_state_save(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(lib.pic_state_save(self._h, C.cast(buf, C.c_void_p), C.byref(n)))
        return buf.raw[:n.value]

    def load_state(self, blob: bytes):
        """Restore a checkpoint written by save_state of a simulation with the
        same grid, patches and precision."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        check(_capi.load().pic_state_load(self._h, C.cast(buf, C.c_void_p), len(blob)))

    def rebin_codes(self, codes):
        c = np.ascontiguousarray(codes, dtype=np.uint8)
        check(_capi.load().pic_rebin_codes(self._h, c.ctypes.data_as(C.POINTER(C.c_uint8)), c.size))

    def timing_enable(self, on=True):
        """True / 1: time every kernel group; 2 or "particles": the particle
        kernel only; 3 or "stamps": the particle kernel and per-item stamps
        (for imbalance()); False / 0: off."""
        mode = {"particles": 2, "stamps": 3}.get(on, on) if isinstance(on, str) else int(on)
        check(_capi.load().pic_timing_enable(self._h, mode))

    def imbalance(self) -> dict:
        """Load imbalance of the last stamped particle launch (pic_imbalance)."""
        r = _capi.Imbalance()
        check(_capi.load().pic_imbalance(self._h, C.byref(r)))
        return {k: getattr(r, k) for k, _ in _capi.Imbalance._fields_}

    def timing(self) -> dict:
        t = _capi.Timing()
        check(_capi.load().pic_timing_get(self._h, C.byref(t)))
        return {t.name[k].decode(): (t.total_ms[k], t.launches[k]) for k in range(t.nkernels)}


class Batch:
    """Simulations of one precision stepped together (one queue, one launch per kernel)."""

    def __init__(self, precision: int = 32, stream: int | None = None, ndim: int = 2):
        lib = _capi.load()
        self.stream = current_stream_handle() if stream is None else int(stream)
        h = C.c_void_p()
        check(lib.pic_batch_create(int(ndim), int(precision), C.c_void_p(self.stream), C.byref(h)))
        self._h = h
        _track(_LIVE_BATCHES, self)
        self.members = {}

    def add(self, sim: Sim, nsteps: int):
        check(_capi.load().pic_batch_add(self._h, sim.handle, int(nsteps)))
        self.members[sim.handle.value] = sim

    def remove(self, sim: Sim):
        check(_capi.load().pic_batch_remove(self._h, sim.handle))
        self.members.pop(sim.handle.value, None)

    def step(self, max_steps: int) -> int:
        done = C.c_int32()
        check(_capi.load().pic_batch_step(self._h, int(max_steps), C.byref(done)))
        return done.value

    def finished(self):
        n = C.c_int32()
        cap = max(1, len(self.members))
        arr = (C.c_void_p * cap)()
        check(_capi.load().pic_batch_finished(self._h, arr, cap, C.byref(n)))
        return [self.members[arr[i]] for i in range(min(n.value, cap))]

    def __len__(self):
        n = C.c_int32()
        check(_capi.load().pic_batch_size(self._h, C.byref(n)))
        return n.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _capi.load().pic_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
