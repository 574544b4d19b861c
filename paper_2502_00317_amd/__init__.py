"""MI355X-native k-clique counting and listing (DIST hot path).

The native library ``libdist.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/dist.h``) does all of the work; ``dist`` is the thin
ctypes binding.  Importing this package loads nothing native: the binding
loads the library on first use and raises if it has not been built.
"""
__all__ = ["dist", "graphgen"]
