"""MI355X-native partitioned folded spectrum method (PFSM) subspace diagonalisation.

The compute path is libpfsm.so (hand-written HIP kernels for gfx950) behind
the C ABI declared in include/pfsm.h; this package is its Python binding.
"""
from .binding import (BatchedPlan, Plan, PFSMFunction, load_library, solve, generalized_to_standard,  # noqa: F401
                      LIB_PATH)
from .scf import FullDiag, SCFDriver, StepRecord  # noqa: F401,E402
