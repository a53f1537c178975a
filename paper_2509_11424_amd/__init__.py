"""mgmlmc: multigrid multilevel Monte Carlo trace estimation with orthogonal
projectors (arXiv:2509.11424) on one MI355X (gfx950).

The computation lives in the HIP library libmgmlmc.so (C ABI in
include/mgmlmc.h); this package only marshals arguments.  Importing it does
not load the library; the first call does, and fails loudly if it is missing.
"""
from .api import (Context, Operator, Hierarchy, Net, Deflation, draw_z4, draw_noise, solve_desc, mlmc_allocate, lib,
                  to_dofmajor, from_dofmajor, MgmError, EXPORTED, LIB_PATH)

__all__ = ["Context", "Operator", "Hierarchy", "Net", "Deflation", "draw_z4", "draw_noise", "solve_desc", "mlmc_allocate", "lib",
           "to_dofmajor", "from_dofmajor", "MgmError", "EXPORTED", "LIB_PATH"]
