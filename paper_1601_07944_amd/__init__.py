"""MI355X-native modal discontinuous Galerkin right-hand side (2D Euler).

The method runs in libdgmi.so (HIP kernels for gfx950 behind the C ABI of
include/dg.h); `binding` is its ctypes binding and `workloads` the seeded
synthetic inputs.  Importing the package loads nothing.
"""
