"""Plain, slow, FP64 CPU reference ("oracle") of the quasi-matrix-free hybrid
multigrid of Weinzierl & Weinzierl (arXiv:1607.00648).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library (no kernels, headers,
helpers, tables or generators); the only common code is the seeded input
generator in ``workloads``, which holds none of the method's arithmetic.

The oracle works on sparse matrices over the interior unknowns (SciPy CSR) and
on stencil arrays over the full vertex lattice.  Every function cites the
section, equation or algorithm of the paper it follows.  Readings of passages
that are ambiguous, garbled or silent are listed in the module docstrings where
they are used.

Pins (tests that fix this code against something other than itself) live in
``tests/test_oracle_*.py``.  Functions without such a pin say "parity unpinned"
in their docstring.
"""
from .fem import (element_matrix, geometric_stencil, convection_stencil, offsets, corners,
                  stencil_to_csr, csr_to_stencil, interior_mask, coarsen_eps,
                  rhs_from_f)
from .transfer import (dlinear_P, boxmg_P, injection_R, aggregation_R, boxmg_reference_stepwise,
                       boxmg_reference_Cs, boxmg_reference_matrix)
from .galerkin import rap, definiteness_violations
from . import refine
from .store import quantise, delta_zero, hier_deltas, P_to_parent_weights, bpa_value, bpa_encode
from .solver import (Hierarchy, build_hierarchy, jacobi, residual, vcycle,
                     solve, mixed_solve, direct_solve, raise_coarsest, stagnated,
                     block_jacobi, iota_positions, additive_cycle, solve_additive,
                     bpx_cycle, cpoint_positions)

__all__ = [
    "element_matrix", "geometric_stencil", "convection_stencil", "injection_R", "aggregation_R", "offsets", "corners",
    "stencil_to_csr", "csr_to_stencil", "interior_mask", "coarsen_eps",
    "rhs_from_f", "dlinear_P", "boxmg_P", "boxmg_reference_stepwise",
    "boxmg_reference_Cs", "boxmg_reference_matrix", "rap",
    "definiteness_violations", "quantise", "delta_zero", "hier_deltas",
    "P_to_parent_weights", "bpa_value", "bpa_encode", "raise_coarsest", "stagnated", "block_jacobi", "iota_positions", "additive_cycle", "solve_additive", "bpx_cycle", "cpoint_positions", "Hierarchy", "build_hierarchy", "jacobi",
    "residual", "vcycle", "solve", "mixed_solve", "direct_solve",
    "refine",
]
