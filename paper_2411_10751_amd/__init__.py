"""High-order lattice Boltzmann (D2Q37 / D3Q39, Hermite source terms) on AMD
Instinct MI355X.

Submodules:
  holb    -- ctypes binding of libholb.so (the HIP library); importing it
             raises if the library is not built.
  inputs  -- seeded synthetic workloads (initial fields and run parameters).
  build   -- hipcc build step of the library.
"""
__all__ = ["holb", "inputs", "build"]
