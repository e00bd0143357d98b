"""SCF driver with a full-diagonalisation fallback.

PFSM needs previous eigenvectors that nearly diagonalise the current matrix
(Methodology: the rotated matrix is diagonally dominant).  The paper therefore
diagonalises the full matrix in the first SCF steps and only then switches to
PFSM.  This driver applies that policy and guards every later step:

  * steps 0 .. full_steps - 1: full diagonalisation;
  * dominance monitor, before a PFSM step: the residual of the previous
    eigenpairs against the new matrix, ||A_k V - V diag(lambda)||_F / ||A_k||_F,
    measures how far V is from diagonalising A_k; above dominance_tol the step
    is a full diagonalisation;
  * breakdown monitor, after a PFSM step: a device failure report (overlap
    breakdown, non-finite values, eigensolver not converged, lost vector
    length) or a residual of the new eigenpairs above residual_tol sends the
    step to the full diagonalisation.

The full diagonalisation is the library's own: a plan whose single submatrix
is the whole matrix (one slice, no halo, no folded-spectrum iteration), so the
batched block-Jacobi eigensolver diagonalises V^T A V on the GPU and the result
is rotated back by V.  Every decision is recorded in `history`.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import torch

from .binding import Plan


class FullDiag:
    """Full-size eigendecomposition of a symmetric matrix on the GPU (FP64):
    a plan with one submatrix of order n and no folded-spectrum iteration."""

    def __init__(self, n: int, max_sweeps: int = 40):
        self.n = int(n)
        self.plan = Plan(self.n, [0, self.n], halo=0, iterations=0, precision="fp64", max_sweeps=max_sweeps)

    def solve(self, A: torch.Tensor, V_prev: Optional[torch.Tensor] = None, check: bool = True):
        """(lambda ascending, V) with A = V diag(lambda) V^T.  V_prev (orthonormal
        columns) is the basis the eigensolver starts from: the closer it is to
        the eigenvectors, the fewer Jacobi sweeps are needed."""
        if V_prev is None:
            V_prev = torch.eye(self.n, dtype=torch.float64, device=A.device)
        return self.plan.solve(A, V_prev, check=check)

    def diagnostics(self, A, lam, V):
        return self.plan.diagnostics(A, lam, V)


@dataclasses.dataclass
class StepRecord:
    step: int
    method: str                  # "full" or "pfsm"
    reason: str                  # why this method was used
    dominance: Optional[float]   # residual of the previous eigenpairs against this step's matrix
    residual: Optional[float]    # residual of this step's eigenpairs


class SCFDriver:
    """Eigenpairs of a sequence of symmetric matrices A_0, A_1, ... (one call
    of step() per SCF iteration), PFSM when it is safe, full diagonalisation
    otherwise.  `pfsm` and `full` may be given (objects with solve(A, V,
    check=True) and diagnostics(A, lam, V)); by default they are built from the
    plan arguments."""

    def __init__(self, n: int, part_offsets: Sequence[int], halo: int = -1, iterations: int = 3,
                 precision: str = "fp64", full_steps: int = 3, dominance_tol: float = 1e-2,
                 residual_tol: float = 1e-3, max_sweeps_full: int = 40, pfsm=None, full=None):
        if full_steps < 1:
            raise ValueError("full_steps must be >= 1: PFSM needs previous eigenvectors")
        self.n = int(n)
        self.full_steps = int(full_steps)
        self.dominance_tol = float(dominance_tol)
        self.residual_tol = float(residual_tol)
        self.pfsm = pfsm if pfsm is not None else Plan(self.n, part_offsets, halo=halo, iterations=iterations,
                                                       precision=precision)
        self.full = full if full is not None else FullDiag(self.n, max_sweeps_full)
        self.lam = None
        self.V = None
        self.history: List[StepRecord] = []

    def _full(self, A, reason, dominance=None):
        lam, V = self.full.solve(A, self.V, check=True)
        res = self.full.diagnostics(A, lam, V)[0]
        self.history.append(StepRecord(len(self.history), "full", reason, dominance, res))
        self.lam, self.V = lam, V
        return lam, V

    def step(self, A):
        k = len(self.history)
        if self.V is None or k < self.full_steps:
            return self._full(A, "start")
        dom = self.pfsm.diagnostics(A, self.lam, self.V)[0]
        if not (dom <= self.dominance_tol):
            return self._full(A, "dominance", dom)
        try:
            lam, V = self.pfsm.solve(A, self.V, check=True)
        except RuntimeError as e:
            return self._full(A, "breakdown: %s" % e, dom)
        res = self.pfsm.diagnostics(A, lam, V)[0]
        if not (math.isfinite(res) and res <= self.residual_tol):
            return self._full(A, "residual", dom)
        self.history.append(StepRecord(k, "pfsm", "dominant", dom, res))
        self.lam, self.V = lam, V
        return lam, V
