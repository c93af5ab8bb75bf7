"""MI355X-native MLS-MPM step and adjoint (FluidEngine's hot path).

Submodules:
  scenes  -- seeded synthetic inputs (no method arithmetic)
  build   -- hipcc build of libmpm.so for gfx950
  _lib    -- ctypes binding of include/mpm.h
  sim     -- torch-memory front end: Simulator, MpmRollout, BlobLoss
"""
__all__ = ["scenes", "build", "sim"]
