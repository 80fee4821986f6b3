"""MI355X-native patch-decomposed electromagnetic PIC hot path.

Modules:
  workloads -- seeded synthetic inputs (no method arithmetic)
  _capi     -- ctypes declarations of include/pic.h
  sim       -- Sim / Batch bindings (marshalling only; the step runs in libpic.so)
  build     -- hipcc build of libpic.so for gfx950
"""

__all__ = ["workloads", "sim", "build"]


def __getattr__(name):
    if name in ("Sim", "Batch"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
