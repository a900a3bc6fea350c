"""MI355X-native matrix-free immersed-boundary timestep (hipib).

Submodules:
  inputs  -- seeded synthetic workloads (no method arithmetic)
  hipib   -- ctypes binding of the C-ABI library libhipib.so (HIP, gfx950)
  build   -- hipcc build of libhipib.so
"""
__all__ = ["inputs", "hipib", "build"]
