"""kfmeg: MI355X-native Kalman filter and fixed-interval smoother for dynamic MEG.

Submodules:
  kfmeg   ctypes binding of the HIP library (libkfmeg.so, C ABI in include/kfmeg.h)
  synth   seeded synthetic workloads shaped like the paper's
  build   compiles the HIP sources for gfx950
The binding is imported lazily so that the input generator works without the
library or a GPU.
"""
__all__ = ["kfmeg", "synth", "build"]
