"""MI355X (gfx950) hot path of ROM-accelerated SIMP minimum-compliance topology
optimisation: matrix-free Jacobi-PCG full-order solves, compliance and sensitivities,
and the Galerkin ROM (per-element MFMA contraction, float64 reduced Cholesky,
residual error indicator), behind the C ABI of include/topo_rom.h.

Python here only marshals arguments to the HIP library; there is no CPU fallback.
"""
from .binding import (FP64, MIXED, Context, TopoError, context, element_stiffness, load,
                      make_mesh)

__all__ = ["FP64", "MIXED", "Context", "TopoError", "context", "element_stiffness", "load",
           "make_mesh"]
