"""MH3D on MI355X: the multi-harmonic forward operator A = P H B, its adjoint and the
nonnegative Tikhonov FISTA solve, as hand-written HIP kernels for gfx950 behind a C ABI.

Submodules are imported lazily:
  mh3d    ctypes binding of libmh3d.so (the C ABI in include/mh3d.h)
  inputs  seeded synthetic phantoms, noise draws and workload configurations
  build   compiles the HIP library in-tree
"""
__all__ = ["mh3d", "inputs", "build"]
