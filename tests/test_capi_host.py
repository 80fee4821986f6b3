"""Host-side checks of the C ABI library (no GPU): it loads, exports every
entry point include/pic.h declares, and rejects bad descriptors before any
device call."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

from paper_1511_03878_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "pic.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_capi.LIB_PATH):
        from paper_1511_03878_amd import build
        build.build()
    return _capi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert set(names) == set(_capi.EXPORTS)


def _desc(**kw):
    d = dict(ndim=2, precision=32, n=(64, 64, 1), d=(0.1, 0.1, 1.0), dt=0.05, patch=(16, 16, 1),
             periodic=(1, 1, 1), q=-1.0, m=1.0, capacity_factor=0.0, min_capacity=0, chunk=0,
             block=0, field_tile=0, lane_stride=0)
    d.update(kw)
    s = _capi.SimDesc()
    s.ndim, s.precision = d["ndim"], d["precision"]
    s.n = (C.c_int32 * 3)(*d["n"])
    s.d = (C.c_double * 3)(*d["d"])
    s.dt = d["dt"]
    s.patch = (C.c_int32 * 3)(*d["patch"])
    s.periodic = (C.c_int32 * 3)(*d["periodic"])
    s.q, s.m = d["q"], d["m"]
    s.capacity_factor, s.min_capacity, s.chunk, s.block, s.field_tile, s.lane_stride = (
        d["capacity_factor"], d["min_capacity"], d["chunk"], d["block"], d["field_tile"],
        d["lane_stride"])
    s.maxwell_order = d.get("maxwell_order", 0)
    s.deterministic = d.get("deterministic", 0)
    return s


@pytest.mark.parametrize("bad,code", [
    (dict(precision=16), -1),
    (dict(ndim=4), -9),
    (dict(patch=(24, 16, 1)), -1),          # does not divide 64
    (dict(patch=(128, 16, 1), n=(128, 64, 1)), -1),  # patch above 64 cells
    (dict(dt=0.2), -1),                      # beyond the Yee limit
    (dict(periodic=(1, 0, 1)), -1),          # only x may be open
    (dict(m=0.0), -1),
    (dict(capacity_factor=0.5), -1),
    (dict(block=128), -1),
    (dict(field_tile=9), -1),
    (dict(lane_stride=65), -1),
    (dict(n=(2, 64, 1), patch=(2, 16, 1)), -1),  # fewer than 4 cells
    (dict(maxwell_order=4), -1),
    (dict(deterministic=2), -1),
    (dict(chunk=16385), -1),                 # the fixed-point current tile of one item
    (dict(maxwell_order=6, periodic=(0, 1, 1)), -1),  # sixth order needs periodic axes
    (dict(maxwell_order=6, dt=0.06), -1),    # within the Yee limit, above the sixth-order one
    (dict(maxwell_order=6, ndim=3, n=(16, 16, 16), patch=(8, 8, 8), d=(0.1, 0.1, 0.1),
          dt=0.05), -1),                     # 3-D: within the Yee limit, above the sixth-order one
])
def test_bad_descriptors_fail_before_device_work(lib, bad, code):
    h = C.c_void_p()
    rc = lib.pic_sim_create(C.byref(_desc(**bad)), None, None, C.byref(h))
    assert rc == code
    assert not h.value
    assert lib.pic_last_error()


def test_null_arguments_are_rejected(lib):
    assert lib.pic_sim_create(None, None, None, None) == -1
    assert lib.pic_step(None, 1) == -1
    assert lib.pic_sync(None) == -1
    assert lib.pic_strerror(-5) == b"patch capacity overflow"
    h = C.c_void_p()
    assert lib.pic_batch_create(2, 48, None, C.byref(h)) == -1


def test_deterministic_mode_charges_its_accumulators(lib):
    """Deterministic deposition holds three 64-bit accumulators per field node:
    the byte estimate (used for admission by the server) grows by exactly that."""
    out0, out1 = C.c_int64(), C.c_int64()
    assert lib.pic_estimate_bytes(C.byref(_desc()), 100000, 0, C.byref(out0)) == 0
    assert lib.pic_estimate_bytes(C.byref(_desc(deterministic=1)), 100000, 0, C.byref(out1)) == 0
    assert out1.value - out0.value == 3 * 8 * 64 * 64
