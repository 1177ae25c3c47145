"""Two-phase CSR SpGEMM (symbolic + numeric Gustavson) for MI355X / gfx950.

The product runs in libspg.so (hand-written HIP); see include/spg.h for the
C ABI.  ``spgemm`` holds the torch-facing wrapper, ``_lib`` the one-to-one
ctypes binding, ``gen`` seeded synthetic workloads.
"""
from . import gen  # noqa: F401


def __getattr__(name):
    # the torch wrapper is imported lazily so that gen can be used without torch/GPU
    if name in ("SpGEMM", "DeviceCsr", "spgemm"):
        from . import spgemm as _s
        return getattr(_s, name)
    raise AttributeError(name)
