"""MI355X-native FP64 CTU-PPM + HLLC hydrodynamics (gfx950 HIP kernels behind a C ABI).

Modules:
  inputs  seeded synthetic initial conditions and box descriptions (numpy only)
  hydro   ctypes binding of include/hydro.h (libhydro.so); PyTorch supplies
          device memory and streams
  build   in-tree hipcc build of libhydro.so for gfx950
"""
