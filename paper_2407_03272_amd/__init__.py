"""Nesterov-accelerated Jacobi-type solver for consistent SPSD systems on MI355X (gfx950).

Submodules:
  naj        -- ctypes binding of the C-ABI library libnaj.so (loads torch)
  workloads  -- seeded synthetic input generators (numpy/scipy only)
  build      -- compiles libnaj.so with hipcc
"""
__all__ = ["naj", "workloads", "build"]
