"""MI355X-native hot path of the 2D Serre-Green-Naghdi Fourier/GMRES solver.

The solver itself is the HIP library libsgn.so (csrc/, C-ABI in
include/sgn.h); `sgn` is its ctypes binding and `build` compiles it.
"""
__all__ = ["sgn", "build"]
