"""Reverse-mode gradient of a symmetric eigendecomposition, FP64.

Oracle code: test infrastructure only.

For A = V diag(lam) V^T with orthonormal V, a loss L(lam, V) with gradients
dlam = dL/dlam and dV = dL/dV pulls back to
    G = V (diag(dlam) + F o (V^T dV)) V^T,   dL/dA = (G + G^T) / 2,
F_ii = 0 and, for i != j, F_ij = 1 / (lam_j - lam_i) (Giles, "An extended
collection of matrix derivative results", 2008).  The 1/gap factor is
broadened to a Lorentzian  F_ij = d / (d^2 + eta^2),  d = lam_j - lam_i,  so an
exactly degenerate pair contributes nothing instead of dividing by zero.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np


def lorentz_f(lam: np.ndarray, eta: float) -> np.ndarray:
    d = lam[None, :] - lam[:, None]  # d_ij = lam_j - lam_i
    F = d / (d * d + eta * eta)
    np.fill_diagonal(F, 0.0)
    return F


def eigh_adjoint(lam: np.ndarray, V: np.ndarray, dlam: Optional[np.ndarray], dV: Optional[np.ndarray],
                 eta: float = 1e-8) -> np.ndarray:
    n = V.shape[0]
    M = np.zeros((n, n))
    if dlam is not None:
        M[np.arange(n), np.arange(n)] += dlam
    if dV is not None:
        M += lorentz_f(lam, eta) * (V.T @ dV)
    G = V @ M @ V.T
    return 0.5 * (G + G.T)


def occupied_loss(lam: np.ndarray, V: np.ndarray, w: np.ndarray, d: np.ndarray) -> float:
    """L = sum_{i<n_occ} w_i lam_i + sum_{j<n_occ} v_j^T diag(d) v_j (n_occ = len(w))."""
    k = len(w)
    return float(w @ lam[:k] + np.sum(d[:, None] * V[:, :k] ** 2))


def occupied_loss_grads(lam: np.ndarray, V: np.ndarray, w: np.ndarray, d: np.ndarray):
    n = V.shape[0]
    k = len(w)
    dlam = np.zeros(n)
    dlam[:k] = w
    dV = np.zeros_like(V)
    dV[:, :k] = 2.0 * d[:, None] * V[:, :k]
    return dlam, dV


def central_fd(loss_of_A: Callable[[np.ndarray], float], A: np.ndarray, E: np.ndarray, h: float,
               order: int = 4) -> float:
    """Central-difference directional derivative of L along E.

    order=2: (L(A+hE) - L(A-hE)) / 2h.  order=4 (default): the Richardson
    combination (8[L(A+hE) - L(A-hE)] - [L(A+2hE) - L(A-2hE)]) / 12h, whose
    O(h^4) truncation stays far below 1e-6 relative for gaps down to ~1e-2 at
    h = 1e-5 ||A||, where the O(h^2) stencil does not."""
    d1 = loss_of_A(A + h * E) - loss_of_A(A - h * E)
    if order == 2:
        return d1 / (2.0 * h)
    d2 = loss_of_A(A + 2.0 * h * E) - loss_of_A(A - 2.0 * h * E)
    return (8.0 * d1 - d2) / (12.0 * h)
