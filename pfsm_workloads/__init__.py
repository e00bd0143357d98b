"""Seeded synthetic workloads for the PFSM subspace-diagonalization step.

This package only draws random numbers and assembles inputs (prescribed
spectra, random orthogonal bases, perturbed previous eigenvectors, SCF-like
sequences, batch layouts, loss weights, overlap matrices).  It holds none of the method's
arithmetic, so both the CPU oracle and the GPU path can consume it.
"""
from .gen import (  # noqa: F401
    CONFIGS,
    WorkloadConfig,
    spectrum,
    householder_q,
    antisym_k,
    expm_small,
    prescribed_problem,
    scf_sequence,
    batch_sizes,
    batch_instance,
    loss_weights,
    random_symmetric_unit,
    uniform_layout,
    overlap_matrix,
)
