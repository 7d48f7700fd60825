"""MI355X-native batched explicit quadrotor step (libmd) -- Python side.

Submodules:
  md         ctypes binding of include/md.h (same names as the C ABI)
  workloads  seeded synthetic inputs (no physics arithmetic)
  build      hipcc build of libmd.so for gfx950

Nothing is imported eagerly, so importing the package never touches the GPU.
"""
__all__ = ["md", "workloads", "build"]
