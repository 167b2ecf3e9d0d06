"""Sparse-tiled, fused DG elastic-wave time step on AMD Instinct MI355X.

Submodules:
  dgtile  - ctypes binding of libdgtile.so (the C ABI in include/dgtile.h)
  inputs  - seeded synthetic meshes, materials and sources
  build   - compiles libdgtile.so for gfx950
"""
__all__ = ["dgtile", "inputs", "build"]
