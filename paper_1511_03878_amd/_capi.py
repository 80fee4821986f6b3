"""ctypes declarations of the C ABI in include/pic.h (argument marshalling only).

The shared library is built in-tree by ``paper_1511_03878_amd.build``; loading
fails loudly when it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK = 0
ERRORS = {
    -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EBUDGET", -4: "PIC_EHIP", -5: "PIC_EOVERFLOW",
    -6: "PIC_ENAN", -7: "PIC_ECFL", -8: "PIC_ESTATE", -9: "PIC_ENOTSUP",
}
COMPONENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "rho")

# every entry point declared in include/pic.h
EXPORTS = (
    "pic_sim_create", "pic_sim_destroy", "pic_particles_set", "pic_laser_set", "pic_fields_set",
    "pic_step", "pic_sync", "pic_fields_get", "pic_num_particles", "pic_particles_get",
    "pic_patch_counts_get", "pic_diag_get", "pic_residuals", "pic_history_get", "pic_rebin_codes",
    "pic_timing_enable", "pic_timing_get", "pic_batch_create", "pic_batch_destroy",
    "pic_batch_add", "pic_batch_remove", "pic_batch_step", "pic_batch_finished",
    "pic_batch_size", "pic_estimate_bytes", "pic_autotune", "pic_state_save", "pic_state_load",
    "pic_patch_order", "pic_curve_segments", "pic_window_set", "pic_merge_set", "pic_merge",
    "pic_rho_get_noalloc", "pic_species_add", "pic_particles_init", "pic_laser_add",
    "pic_perm_get", "pic_device_bytes", "pic_imbalance", "pic_step_set", "pic_autotune_patch",
    "pic_strerror",
    "pic_last_error",
)


class PicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class SimDesc(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("precision", C.c_int32), ("n", C.c_int32 * 3),
        ("d", C.c_double * 3), ("dt", C.c_double), ("patch", C.c_int32 * 3),
        ("periodic", C.c_int32 * 3), ("q", C.c_double), ("m", C.c_double),
        ("capacity_factor", C.c_double), ("min_capacity", C.c_int32), ("chunk", C.c_int32),
        ("block", C.c_int32), ("field_tile", C.c_int32), ("lane_stride", C.c_int32),
        ("graph", C.c_int32), ("patch_order", C.c_int32),
        ("maxwell_order", C.c_int32), ("deterministic", C.c_int32),
    ]


class SpeciesDesc(C.Structure):
    _fields_ = [
        ("q", C.c_double), ("m", C.c_double), ("profile", C.c_int32), ("loading", C.c_int32),
        ("ppc", C.c_int32), ("reserved", C.c_int32), ("n0", C.c_double), ("param", C.c_double * 6),
        ("temperature", C.c_double), ("seed", C.c_uint64),
    ]


class LaserDesc(C.Structure):
    _fields_ = [
        ("a0", C.c_double), ("omega0", C.c_double), ("w0", C.c_double), ("tau", C.c_double),
        ("t0", C.c_double), ("x_focus", C.c_double), ("y_center", C.c_double), ("phase", C.c_double),
        ("polarisation", C.c_int32), ("face", C.c_int32),
    ]


class TuneResult(C.Structure):
    _fields_ = [
        ("block", C.c_int32), ("field_tile", C.c_int32), ("lane_stride", C.c_int32),
        ("chunk", C.c_int32), ("ms_per_step", C.c_double), ("trials", C.c_int32),
        ("from_cache", C.c_int32), ("patch", C.c_int32 * 3),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("particles", C.c_int64), ("removed", C.c_int64),
        ("field_energy", C.c_double), ("kinetic_energy", C.c_double),
        ("occupancy_min", C.c_int32), ("occupancy_max", C.c_int32),
        ("occupancy_mean", C.c_double), ("flags", C.c_int32), ("relayouts", C.c_int32),
        ("window_cells", C.c_int64), ("merged", C.c_int64), ("device_bytes", C.c_int64),
    ]


class Residuals(C.Structure):
    _fields_ = [("step", C.c_int64), ("gauss", C.c_double), ("continuity", C.c_double),
                ("rho_max", C.c_double), ("rho0_max", C.c_double)]


class Imbalance(C.Structure):
    _fields_ = [("step", C.c_int64), ("items", C.c_int32), ("units", C.c_int32),
                ("device_units", C.c_int32), ("span_us", C.c_double), ("busy_max_us", C.c_double),
                ("busy_mean_us", C.c_double), ("imbalance", C.c_double),
                ("static_imbalance", C.c_double), ("segment_imbalance", C.c_double),
                ("patch_max_us", C.c_double), ("patch_mean_us", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("nkernels", C.c_int32), ("name", C.c_char_p * 8), ("total_ms", C.c_double * 8),
                ("launches", C.c_int64 * 8)]


_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_vp = C.c_void_p


def load() -> C.CDLL:
    """Load libpic.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -m paper_1511_03878_amd.build)")
    # torch ships its own HIP runtime (same soname).  Load it first so the
    # library binds to that single runtime instead of pulling in a second one:
    # device memory and streams come from torch and must live in the same
    # runtime that launches the kernels.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    sig = {
        "pic_sim_create": (C.c_int, [C.POINTER(SimDesc), C.POINTER(Allocator), _vp, C.POINTER(_vp)]),
        "pic_sim_destroy": (None, [_vp]),
        "pic_particles_set": (C.c_int, [_vp, C.c_int64, _D, _D, _D, _D, _D, _D, _D]),
        "pic_laser_set": (C.c_int, [_vp, C.c_int64, _D, _D]),
        "pic_window_set": (C.c_int, [_vp, C.c_int64, C.c_double, C.c_int32, C.c_int32, _D, C.c_int64]),
        "pic_merge_set": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32]),
        "pic_merge": (C.c_int, [_vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]),
        "pic_fields_set": (C.c_int, [_vp, C.c_int, _D, C.c_size_t]),
        "pic_fields_get": (C.c_int, [_vp, C.c_int, _D, C.c_size_t]),
        "pic_step": (C.c_int, [_vp, C.c_int64]),
        "pic_sync": (C.c_int, [_vp]),
        "pic_num_particles": (C.c_int, [_vp, _I64]),
        "pic_particles_get": (C.c_int, [_vp, _D, _D, _D, _D, _D, _D, _D, _I64, C.c_size_t]),
        "pic_patch_counts_get": (C.c_int, [_vp, _I32, C.c_size_t]),
        "pic_diag_get": (C.c_int, [_vp, C.POINTER(Diag)]),
        "pic_residuals": (C.c_int, [_vp, C.POINTER(Residuals)]),
        "pic_rho_get_noalloc": (C.c_int, [_vp, _D, C.c_size_t]),
        "pic_species_add": (C.c_int, [_vp, C.POINTER(SpeciesDesc), _I32]),
        "pic_particles_init": (C.c_int, [_vp, C.c_int32]),
        "pic_laser_add": (C.c_int, [_vp, C.POINTER(LaserDesc)]),
        "pic_perm_get": (C.c_int, [_vp, _I64, C.c_size_t]),
        "pic_device_bytes": (C.c_int, [_vp, _I64]),
        "pic_imbalance": (C.c_int, [_vp, C.POINTER(Imbalance)]),
        "pic_step_set": (C.c_int, [_vp, C.c_int64]),
        "pic_autotune_patch": (C.c_int, [C.POINTER(SimDesc), C.POINTER(SpeciesDesc), C.POINTER(LaserDesc),
                                         _I32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Allocator), _vp,
                                         C.c_char_p, C.POINTER(TuneResult)]),
        "pic_history_get": (C.c_int, [_vp, C.c_int64, C.c_int64, _D, _D, _I64]),
        "pic_rebin_codes": (C.c_int, [_vp, C.POINTER(C.c_uint8), C.c_size_t]),
        "pic_timing_enable": (C.c_int, [_vp, C.c_int]),
        "pic_timing_get": (C.c_int, [_vp, C.POINTER(Timing)]),
        "pic_batch_create": (C.c_int, [C.c_int32, C.c_int32, _vp, C.POINTER(_vp)]),
        "pic_batch_destroy": (None, [_vp]),
        "pic_batch_add": (C.c_int, [_vp, _vp, C.c_int64]),
        "pic_batch_remove": (C.c_int, [_vp, _vp]),
        "pic_batch_step": (C.c_int, [_vp, C.c_int64, _I32]),
        "pic_batch_finished": (C.c_int, [_vp, C.POINTER(_vp), C.c_int32, _I32]),
        "pic_batch_size": (C.c_int, [_vp, _I32]),
        "pic_estimate_bytes": (C.c_int, [C.POINTER(SimDesc), C.c_int64, C.c_int64, _I64]),
        "pic_autotune": (C.c_int, [_vp, C.c_int32, C.c_char_p, C.POINTER(TuneResult)]),
        "pic_state_save": (C.c_int, [_vp, _vp, C.POINTER(C.c_size_t)]),
        "pic_state_load": (C.c_int, [_vp, _vp, C.c_size_t]),
        "pic_patch_order": (C.c_int, [C.c_int32, _I32, _I32, C.c_int64]),
        "pic_curve_segments": (C.c_int, [_I64, C.c_int64, C.c_int32, _I64]),
        "pic_strerror": (C.c_char_p, [C.c_int]),
        "pic_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != PIC_OK:
        lib = load()
        raise PicError(rc, lib.pic_last_error().decode(errors="replace"))
    return rc
