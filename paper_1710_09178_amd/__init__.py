"""MI355X (gfx950) staggered-fermion RHMC hot path: a HIP library behind the C
ABI of include/stag.h, with a thin ctypes binding in ``stag``.

Importing the package does not touch the GPU; ``stag.load_library()`` loads the
in-tree ``libstag.so`` and fails loudly if it has not been built.
"""
