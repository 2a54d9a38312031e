"""MI355X-native evaluation of the 3D Laplace kernel-independent FMM.

The product path is libkifmm.so (HIP kernels for gfx950 behind the C ABI in
include/kifmm.h) and its thin binding in ``kifmm``.  ``inputs`` holds the
seeded synthetic workloads.
"""
