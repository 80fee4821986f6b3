"""Oracle: plain FP64 CPU PIC step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
it shares no code with the HIP path; both sides take their inputs from the
seeded workload generator, which holds none of the method's arithmetic.

The C source ``orc.c`` is the oracle; this module is a ctypes wrapper around
it.  ``build()`` compiles it with gcc (plain ``-O2``, no fast-math).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

COMPONENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz")


_LIB_OMP = os.path.join(_HERE, "liborc_omp.so")


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so next to it and return the path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_timing(force: bool = True) -> str:
    """Compile the timing build of the same source (-O3 -march=native for this
    host, OpenMP over the particle loop with per-thread current arrays) into
    liborc_omp.so; only the CPU baseline of the benchmark loads it."""
    if force or not os.path.exists(_LIB_OMP):
        tmp = _LIB_OMP + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_OMP)
    return _LIB_OMP


def use_timing_build():
    """Load the timing build in place of the plain one (CPU baseline only)."""
    global _lib, _LIB
    build_timing(force=True)
    _LIB = _LIB_OMP
    _lib = None
    return _load()


def set_threads(n: int) -> int:
    """Host threads of the particle loop (timing build); returns the count in effect."""
    lib = _load()
    lib.orc_set_threads(int(n))
    return int(lib.orc_threads())


class _Desc(C.Structure):
    _fields_ = [
        ("ndim", C.c_int),
        ("n", C.c_int * 3),
        ("d", C.c_double * 3),
        ("dt", C.c_double),
        ("patch", C.c_int * 3),
        ("periodic", C.c_int * 3),
        ("q", C.c_double),
        ("m", C.c_double),
    ]


_lib = None
_D = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = C.CDLL(_LIB)
    vp = C.c_void_p
    sig = {
        "orc_create": (vp, [C.POINTER(_Desc)]),
        "orc_destroy": (None, [vp]),
        "orc_fsize": (C.c_int64, [vp]),
        "orc_npatch": (C.c_int, [vp]),
        "orc_npart": (C.c_int64, [vp]),
        "orc_step_index": (C.c_int64, [vp]),
        "orc_removed": (C.c_int64, [vp]),
        "orc_set_step": (None, [vp, C.c_int64]),
        "orc_set_particles": (C.c_int, [vp, C.c_int64, _D * 3, _D * 3, _D]),
        "orc_get_particles": (None, [vp, _D * 3, _D * 3, _D, C.POINTER(C.c_int64)]),
        "orc_get_counts": (None, [vp, C.POINTER(C.c_int32)]),
        "orc_get_field": (None, [vp, C.c_int, _D]),
        "orc_set_field": (None, [vp, C.c_int, _D]),
        "orc_set_laser": (None, [vp, C.c_int64, _D, _D]),
        "orc_add_laser": (C.c_int, [vp] + [C.c_double] * 8 + [C.c_int]),
        "orc_gauss_beam": (C.c_double, [C.c_double] * 10),
        "orc_splitmix64": (C.c_uint64, [C.c_uint64, C.c_uint64]),
        "orc_particles_init": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_double, _D, C.c_double,
                                         C.c_uint64]),
        "orc_round_storage": (None, [vp]),
        "orc_set_threads": (None, [C.c_int]),
        "orc_threads": (C.c_int, []),
        "orc_step": (None, [vp, C.c_int64]),
        "orc_energy": (None, [vp, _D, _D]),
        "orc_field_energy": (C.c_double, [vp]),
        "orc_rho": (None, [vp, _D]),
        "orc_maxwell": (None, [vp]),
        "orc_set_maxwell_order": (C.c_int, [vp, C.c_int]),
        "orc_set_window": (C.c_int, [vp, C.c_int64, C.c_double, C.c_int, C.c_int, _D, C.c_int64]),
        "orc_window_shift": (C.c_int64, [vp]),
        "orc_merge": (C.c_int64, [vp, C.c_int, C.c_int]),
        "orc_set_merge": (C.c_int, [vp, C.c_int, C.c_int, C.c_int]),
        "orc_merged": (C.c_int64, [vp]),
        "orc_next_id": (C.c_int64, [vp]),
        "orc_deposit": (None, [vp, _D, _D, C.c_double, C.c_double]),
        "orc_gather": (None, [vp, _D, _D]),
        "orc_boris": (None, [_D, _D, _D, C.c_double, C.c_double, C.c_double]),
        "orc_shape": (None, [C.c_double, C.c_int, C.POINTER(C.c_int64), _D]),
        "orc_s2": (C.c_double, [C.c_double]),
        "orc_patch_of": (C.c_int, [vp, _D]),
        "orc_rebin": (None, [C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# operator-level entry points (used by the pins)

def s2(delta: float) -> float:
    """Quadratic B-spline S2(delta) from its piecewise definition."""
    return _load().orc_s2(float(delta))


def shape(xi: float, stag: int):
    """(i0, [w-1, w0, w+1]) for a sample staggered by stag/2 cells."""
    i0 = C.c_int64()
    w = np.zeros(3)
    _load().orc_shape(float(xi), int(stag), C.byref(i0), _dp(w))
    return i0.value, w


def boris(u, E, B, q: float, m: float, dt: float) -> np.ndarray:
    """One relativistic Boris update of u = p/(mc) under fields E, B."""
    uu = _f64(np.array(u, dtype=np.float64).copy())
    EE = _f64(E)
    BB = _f64(B)
    _load().orc_boris(_dp(uu), _dp(EE), _dp(BB), float(q), float(m), float(dt))
    return uu


def splitmix64(seed: int, n: int) -> int:
    """Output n of the SplitMix64 generator seeded with `seed`."""
    return int(_load().orc_splitmix64(int(seed) & (2 ** 64 - 1), int(n)))


def gauss_beam(laser: dict, t: float, y: float) -> float:
    """Incident field of a Gaussian laser description at the x = 0 face."""
    L = laser
    return float(_load().orc_gauss_beam(L["a0"], L.get("omega0", 1.0), L["w0"], L["tau"], L["t0"],
                                        L["x_focus"], L["y_center"], L.get("phase", 0.0), float(t),
                                        float(y)))


PROFILES = {"uniform": 0, "ramp": 1, "cos_sphere": 2}
LOADINGS = {"weight": 0, "count": 1}


def rebin(counts, dest):
    """Canonical re-binning.  Returns (newcount, src) with src[k'] the old
    flat index of the particle placed at new flat index k'."""
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    dest = np.ascontiguousarray(dest, dtype=np.int32)
    npatch = counts.size
    newcount = np.zeros(npatch, dtype=np.int32)
    kept = int(np.count_nonzero(dest >= 0))
    src = np.full(max(kept, 1), -1, dtype=np.int64)
    _load().orc_rebin(npatch, counts.ctypes.data_as(C.POINTER(C.c_int32)),
                      dest.ctypes.data_as(C.POINTER(C.c_int32)),
                      newcount.ctypes.data_as(C.POINTER(C.c_int32)),
                      src.ctypes.data_as(C.POINTER(C.c_int64)))
    return newcount, src[:kept]


class Sim:
    """One oracle simulation (FP64, global arrays, patch-list particle view).

    Geometry keys of ``cfg``: ndim, n (cells per axis), d (cell sizes), dt,
    patch (cells per patch per axis), periodic (per axis; only x may be open),
    q, m.  Particle arrays are given in id order.
    """

    def __init__(self, cfg: dict):
        lib = _load()
        nd = int(cfg["ndim"])
        n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
        d = list(cfg["d"]) + [1.0] * (3 - len(cfg["d"]))
        patch = list(cfg["patch"]) + [1] * (3 - len(cfg["patch"]))
        per = list(cfg.get("periodic", [1, 1, 1])) + [1] * 3
        desc = _Desc(nd, (C.c_int * 3)(*n), (C.c_double * 3)(*d), float(cfg["dt"]),
                     (C.c_int * 3)(*patch), (C.c_int * 3)(*[int(p) for p in per[:3]]),
                     float(cfg.get("q", -1.0)), float(cfg.get("m", 1.0)))
        self._p = lib.orc_create(C.byref(desc))
        if not self._p:
            raise ValueError("oracle: invalid geometry")
        self.cfg = dict(cfg)
        self.ndim = nd
        self.n = n
        self.periodic = per[:3]
        self.fn = [n[a] if (a >= nd or per[a]) else n[a] + 1 for a in range(3)]
        if nd == 2:
            self.fn[2] = 1
        self.fsize = lib.orc_fsize(self._p)
        self.npatch = lib.orc_npatch(self._p)

    def __del__(self):
        p = getattr(self, "_p", None)
        if p and _lib is not None:
            _lib.orc_destroy(p)
            self._p = None

    # -- state ----------------------------------------------------------
    def set_particles(self, x, u, w):
        x = [_f64(a) for a in x] + [np.zeros(len(w))] * (3 - len(x))
        u = [_f64(a) for a in u]
        w = _f64(w)
        rc = _load().orc_set_particles(self._p, len(w), (_D * 3)(*[_dp(a) for a in x]),
                                       (_D * 3)(*[_dp(a) for a in u]), _dp(w))
        if rc != 0:
            raise ValueError("oracle: particle outside the domain")
        self._keep = (x, u, w)

    def particles(self):
        """(x[3], u[3], w, id) in canonical (patch, slot) order."""
        n = _load().orc_npart(self._p)
        x = [np.zeros(n) for _ in range(3)]
        u = [np.zeros(n) for _ in range(3)]
        w = np.zeros(n)
        ids = np.zeros(n, dtype=np.int64)
        _load().orc_get_particles(self._p, (_D * 3)(*[_dp(a) for a in x]),
                                  (_D * 3)(*[_dp(a) for a in u]), _dp(w),
                                  ids.ctypes.data_as(C.POINTER(C.c_int64)))
        return x, u, w, ids

    def counts(self) -> np.ndarray:
        c = np.zeros(self.npatch, dtype=np.int32)
        _load().orc_get_counts(self._p, c.ctypes.data_as(C.POINTER(C.c_int32)))
        return c

    def field(self, comp) -> np.ndarray:
        """Field component as an array shaped (fn_z, fn_y, fn_x) (x fastest)."""
        c = COMPONENTS.index(comp) if isinstance(comp, str) else int(comp)
        out = np.zeros(self.fsize)
        _load().orc_get_field(self._p, c, _dp(out))
        return out.reshape(self.fn[2], self.fn[1], self.fn[0])

    def set_field(self, comp, values):
        c = COMPONENTS.index(comp) if isinstance(comp, str) else int(comp)
        v = _f64(np.asarray(values).reshape(-1))
        assert v.size == self.fsize
        _load().orc_set_field(self._p, c, _dp(v))

    def set_laser(self, ey=None, ez=None):
        """Incident-field table, shape (steps, transverse nodes)."""
        arrs = [None if a is None else _f64(a) for a in (ey, ez)]
        nsteps = next(a.shape[0] for a in arrs if a is not None)
        ptrs = [None if a is None else _dp(a) for a in arrs]
        _load().orc_set_laser(self._p, nsteps, ptrs[0], ptrs[1])

    def particles_init(self, sp: dict):
        """Load a species description (profile, loading, ppc, n0, param,
        temperature, seed) with the oracle's own SplitMix64 loader."""
        p = _f64(list(sp.get("param", [])) + [0.0] * 6)[:6].copy()
        rc = _load().orc_particles_init(self._p, PROFILES[sp["profile"]], LOADINGS[sp.get("loading", "weight")],
                                        int(sp["ppc"]), float(sp.get("n0", 1.0)), _dp(p),
                                        float(sp.get("temperature", 0.0)),
                                        int(sp.get("seed", 0)) & (2 ** 64 - 1))
        if rc != 0:
            raise ValueError("oracle: unsupported species description")

    def round_storage(self):
        """Round the particle state to what FP32 storage holds (positions as
        FP32 offsets from their patch origin, rounded to nearest and kept
        below the patch's upper face; momenta and weights in FP32), back in
        FP64: the state an FP32 run starts from after loading these particles."""
        _load().orc_round_storage(self._p)

    def add_laser(self, laser: dict):
        """A Gaussian laser through the x = 0 face (2-D, open x)."""
        L = laser
        rc = _load().orc_add_laser(self._p, L["a0"], L.get("omega0", 1.0), L["w0"], L["tau"], L["t0"],
                                   L["x_focus"], L["y_center"], L.get("phase", 0.0),
                                   int(L.get("polarisation", 1)))
        if rc != 0:
            raise ValueError("oracle: unsupported laser")

    def rho(self) -> np.ndarray:
        out = np.zeros(self.fsize)
        _load().orc_rho(self._p, _dp(out))
        return out.reshape(self.fn[2], self.fn[1], self.fn[0])

    # -- evolution --------------------------------------------------------
    def step(self, nsteps: int = 1):
        _load().orc_step(self._p, int(nsteps))

    def maxwell(self):
        """Three-sweep Yee update with the current J and laser row."""
        _load().orc_maxwell(self._p)

    def set_maxwell_order(self, order: int):
        """Field solver of spatial order 2 (Yee, the default) or 6 (staggered
        sixth-order differences; every axis periodic)."""
        if _load().orc_set_maxwell_order(self._p, int(order)) != 0:
            raise ValueError("oracle: unsupported field solver order for this grid")

    def set_window(self, start: int, velocity: float, ppc, density):
        """Moving window along x (2-D, open x faces): it jumps one patch column
        whenever v c (n - start) dt reaches the next multiple of the patch width;
        the new column is filled with ppc = (ppc_x, ppc_y) cold particles per cell
        of the given per-column density (the last entry continues)."""
        dens = _f64(density)
        if _load().orc_set_window(self._p, int(start), float(velocity), int(ppc[0]), int(ppc[1]),
                                  _dp(dens), dens.size) != 0:
            raise ValueError("oracle: unsupported moving window for this grid")
        self._win_dens = dens

    def merge(self, cmax: int, iters: int) -> int:
        """One merge pass now (2-D): cells holding more than cmax particles are
        clustered in momentum into cmax / 2 groups; groups of three or more
        become conserving pairs.  Returns the particles taken out."""
        if self.ndim != 2 or not (4 <= cmax <= 32) or not (1 <= iters <= 64):
            raise ValueError("oracle: unsupported merge request")
        return int(_load().orc_merge(self._p, int(cmax), int(iters)))

    def set_merge(self, every: int, cmax: int = 16, iters: int = 8):
        """Merge after every `every`-th step (0: never)."""
        if _load().orc_set_merge(self._p, int(every), int(cmax), int(iters)) != 0:
            raise ValueError("oracle: unsupported merge request")

    @property
    def merged(self) -> int:
        return int(_load().orc_merged(self._p))

    @property
    def window_shift(self) -> int:
        return int(_load().orc_window_shift(self._p))

    @property
    def next_id(self) -> int:
        return int(_load().orc_next_id(self._p))
    def deposit(self, xa, xb, w, vz):
        a = _f64(list(xa) + [0.0] * (3 - len(xa)))
        b = _f64(list(xb) + [0.0] * (3 - len(xb)))
        _load().orc_deposit(self._p, _dp(a), _dp(b), float(w), float(vz))

    def gather(self, xi) -> np.ndarray:
        a = _f64(list(xi) + [0.0] * (3 - len(xi)))
        out = np.zeros(6)
        _load().orc_gather(self._p, _dp(a), _dp(out))
        return out

    def patch_of(self, xi) -> int:
        a = _f64(list(xi) + [0.0] * (3 - len(xi)))
        return _load().orc_patch_of(self._p, _dp(a))

    @property
    def step_index(self) -> int:
        return _load().orc_step_index(self._p)

    def set_step(self, n: int):
        _load().orc_set_step(self._p, int(n))

    @property
    def removed(self) -> int:
        return _load().orc_removed(self._p)

    def energy(self):
        """(U(E^n, B^n), K^n) of the last completed step n."""
        U = C.c_double()
        K = C.c_double()
        _load().orc_energy(self._p, C.byref(U), C.byref(K))
        return U.value, K.value

    def field_energy(self) -> float:
        return _load().orc_field_energy(self._p)
