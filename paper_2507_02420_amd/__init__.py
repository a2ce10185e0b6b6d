"""MI355X-native fast generalized tensor transform (GTT).

The transform y = (W kron ... kron W) x runs in hand-written HIP kernels for
gfx950 behind the C ABI declared in include/gtt.h (library libgtt.so).  The
Python layer in ``gtt`` only marshals arguments (device pointers, sizes and
the current HIP stream) into that ABI.
"""

__all__ = ["gtt", "inputs"]


def __getattr__(name):
    if name == "gtt":
        from . import gtt as _gtt
        return _gtt
    raise AttributeError(name)
