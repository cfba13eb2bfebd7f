"""MI355X-native Newton-Krylov solver for the discretised extreme type-II
Ginzburg-Landau equations (Schloemer & Vanroose): the Jacobian solves by
preconditioned MINRES with a smoothed-aggregation AMG V-cycle, as hand-written
HIP kernels for gfx950 behind the C-ABI library libglnk.so.

Submodules:
  glnk    -- ctypes binding of libglnk.so (torch tensors for device memory)
  inputs  -- seeded synthetic input generators
"""
