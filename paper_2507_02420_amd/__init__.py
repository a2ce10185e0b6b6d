"""MI355X-native fast generalized tensor transform (GTT).

The transform y = (W kron ... kron W) x runs in hand-written HIP kernels for
gfx950 behind the C ABI declared in include/gtt.h (library libgtt.so).  The
Python layer in the ``gtt`` submodule only marshals arguments (device
pointers, sizes and the current HIP stream) into that ABI; import it as
``from paper_2507_02420_amd import gtt``.
"""
