"""FP64 CPU oracle for the PFSM subspace-diagonalization step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke entry point and the CPU-baseline leg of the
benchmark call it.  It shares no code with the GPU library (no kernels,
headers, helpers or tables); the only common dependency is the seeded input
generator in ``pfsm_workloads``, which holds none of the method's arithmetic.

Contents:
  * jacobi      -- cyclic two-sided Jacobi full eigensolver (plain C, FP64)
  * pfsm_ref    -- the plain partitioned folded spectrum method, step by step
  * adjoint_ref -- eigen-decomposition adjoint (reverse-mode gradient)
  * refine_ref  -- FP64 Rayleigh-Ritz / Rayleigh-quotient refinement used by
                   the mixed-precision path
"""
from .jacobi import jacobi_eigh, build_jacobi_lib  # noqa: F401
from .pfsm_ref import pfsm_ref, PfsmLayout, window_layout, gershgorin_alpha  # noqa: F401
