"""Plain, slow, FP64 CPU oracle for the SIMP compliance / ROM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or executes
anything under ``oracle/``; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg do.  The oracle shares no code with the HIP path: it computes the
element stiffness by its own Gauss quadrature, assembles a sparse global matrix,
solves with a sparse direct factorisation (or, beyond direct-solver size, FP64 CG
certified by an independent residual), and builds the reduced operator from the
*assembled* matrix.  Every function cites the passage of the paper it follows
(Yano, Huang & Zahr, "A globally convergent method to accelerate topology
optimization using on-the-fly model reduction").

Parity status: every function here is pinned by tests under ``tests/`` against
closed forms, invariants, brute force or textbook results (see the test modules
``test_oracle_*``); nothing is "parity unpinned".
"""
from .fem import (element_stiffness, constitutive, element_dofs, simp_alpha,
                  simp_alpha_prime, assemble, apply_masked, apply_ebe, apply_rows, solve_direct,
                  solve_cg, compliance, sensitivity, free_dofs)
from .rom import rom_operator, rom_load, rom_solve, rom_residual, rom_eval, rom_gradient
from .basis import pod, gram_schmidt_step, basis_update, SnapshotWindow
from .filter import (filter_forward, filter_adjoint, filter_radius, filter_radius_cited,
                     helmholtz_assemble)
from . import tr

__all__ = [
    "element_stiffness", "constitutive", "element_dofs", "simp_alpha", "simp_alpha_prime",
    "assemble", "apply_masked", "apply_ebe", "apply_rows", "solve_direct", "solve_cg", "compliance",
    "sensitivity", "free_dofs", "rom_operator", "rom_load", "rom_solve", "rom_residual",
    "rom_eval", "rom_gradient", "pod", "gram_schmidt_step", "basis_update", "SnapshotWindow",
    "filter_forward", "filter_adjoint", "filter_radius", "filter_radius_cited", "helmholtz_assemble",
]
