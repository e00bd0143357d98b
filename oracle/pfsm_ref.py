"""Plain FP64 partitioned folded spectrum method (PFSM), step by step.

Oracle code: test infrastructure only (tests, smoke check, CPU baseline).
Every step is written in the order of the paper's Methodology section; NumPy
products and a triangular solve serve as library primitives, nothing is
blocked, fused or reordered.

Steps (with the passage each follows):
  O1  basis change  At = V^T (A V), symmetrised                 (Eq. 12: matrix
      elements of the operator in the current basis; Eq. 3 is the problem)
  O2  alpha from the Gershgorin interval of At                  (Eqs. 8-11)
  O3  overlapping diagonal submatrices B_p of At, B_p y = mu y  (Methodology,
      submatrices of order M; Fig. 1 slice inside its submatrix)
  O4  start vectors = submatrix eigenvectors padded with zeros,
      shifts = submatrix eigenvalues                            (Methodology)
  O5  folded-spectrum iterations x <- x - alpha (At - eps I)^q x (Eq. 11, q=2;
      q=1 is the one-product variant)
  O6  orthonormalisation (Gram-Schmidt == Cholesky-QR)          (Methodology)
  O7  eigenvalues = Rayleigh quotients of the orthonormal vectors
  O8  sign convention, back-rotation V_new = V X, ascending order

Readings where the paper is silent or garbled (alpha rule, window placement,
final eigenvalues, signs) are stated at each step.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
from scipy.linalg import solve_triangular

from .jacobi import jacobi_eigh


@dataclasses.dataclass(frozen=True)
class PfsmLayout:
    """Slice p covers eigen-indices [start, start+size); its submatrix covers
    rows/columns [wstart, wstart+wsize) of At; the slice sits at offset
    `offset` inside the submatrix's ascending eigenvalue ranks."""
    start: int
    size: int
    wstart: int
    wsize: int
    offset: int


def window_layout(n: int, part_offsets: Sequence[int], halo: int) -> List[PfsmLayout]:
    """Submatrix of order M_p = min(n, m_p + 2 h) centred on the slice and
    shifted inward at the ends of the matrix (reading of the overlapping
    diagonal submatrices with the slice inside them)."""
    out = []
    for p in range(len(part_offsets) - 1):
        s = int(part_offsets[p])
        m = int(part_offsets[p + 1]) - s
        M = min(n, m + 2 * halo)
        w = min(max(s - halo, 0), n - M)
        out.append(PfsmLayout(s, m, w, M, s - w))
    return out


def gershgorin_alpha(At: np.ndarray, fs_power: int, alpha_hat: float = 1.0):
    """alpha = alpha_hat / rho^q with rho the width of the Gershgorin interval.

    Reading of Eqs. 8-11: the folded matrix I - alpha (A - eps I)^2 must keep
    every eigenvalue in [0, 1] so that the eigenvector nearest eps dominates;
    alpha (lambda - eps)^2 <= 1 holds for every lambda and every shift inside
    the Gershgorin interval when alpha <= 1/rho^2.
    """
    d = np.diag(At)
    r = np.abs(At).sum(axis=1) - np.abs(d)
    lo = float(np.min(d - r))
    hi = float(np.max(d + r))
    rho = hi - lo
    alpha = alpha_hat / rho ** fs_power if rho > 0 else 0.0
    return alpha, lo, hi


def cholesky_lower(S: np.ndarray):
    """Column-by-column Cholesky S = L L^T.  Returns (L, info); info = k > 0 when
    the k-th pivot (1-based) is not positive, as LAPACK's potrf reports it."""
    n = S.shape[0]
    L = np.zeros_like(S)
    for j in range(n):
        d = S[j, j] - L[j, :j] @ L[j, :j]
        if not d > 0.0:
            return L, j + 1
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (S[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L, 0


def sign_normalize(X: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of every column positive (ties: lowest row)."""
    k = np.argmax(np.abs(X), axis=0)
    sgn = np.where(X[k, np.arange(X.shape[1])] < 0.0, -1.0, 1.0)
    return X * sgn[None, :]


def fs_iterate(At: np.ndarray, X: np.ndarray, eps: np.ndarray, alpha: float, iterations: int,
               fs_power: int = 2, shift_mode: str = "fixed") -> np.ndarray:
    """Folded-spectrum iterations x <- x - alpha (At - eps I)^q x on every column
    (Eq. 11 for q = 2, applied as two shifted products; q = 1 is the
    one-product variant).  shift_mode "fixed" keeps each column's shift (the
    submatrix eigenvalue, Methodology); "rayleigh" replaces it before every
    iteration by the column's Rayleigh quotient x^T At x / x^T x."""
    X = np.array(X, dtype=np.float64, copy=True)
    eps = np.array(eps, dtype=np.float64, copy=True)
    for _ in range(iterations):
        if shift_mode == "rayleigh":
            eps = np.sum(X * (At @ X), axis=0) / np.sum(X * X, axis=0)
        elif shift_mode != "fixed":
            raise ValueError("shift_mode must be 'fixed' or 'rayleigh'")
        if fs_power == 2:
            Y1 = At @ X - X * eps[None, :]
            Y2 = At @ Y1 - Y1 * eps[None, :]
            X = X - alpha * Y2
        elif fs_power == 1:
            X = X - alpha * (At @ X - X * eps[None, :])
        else:
            raise ValueError("fs_power must be 1 or 2")
    return X


def pfsm_ref(A: np.ndarray, V: np.ndarray, part_offsets: Sequence[int], halo: Optional[int] = None,
             iterations: int = 3, fs_power: int = 2, alpha: Optional[float] = None,
             shift_mode: str = "fixed", details: bool = False):
    """One PFSM subspace-diagonalization step.

    A: n x n real symmetric; V: n x n previous eigenvectors (orthonormal
    columns, ascending previous eigenvalues).  part_offsets: P+1 ascending
    slice boundaries 0..n.  halo: rows added on each side of a slice to form
    its submatrix (default: half the largest slice).

    Returns (lam, V_new, info[, det]).  info = 0 on success, k > 0 when the
    overlap matrix is not positive definite at column k, -1 for non-finite
    input.  lam is ascending; V_new's columns are the matching eigenvectors.
    """
    A = np.asarray(A, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    n = A.shape[0]
    part_offsets = [int(x) for x in part_offsets]
    assert part_offsets[0] == 0 and part_offsets[-1] == n
    if halo is None:
        halo = max(part_offsets[p + 1] - part_offsets[p] for p in range(len(part_offsets) - 1)) // 2
    det = {}
    if not (np.all(np.isfinite(A)) and np.all(np.isfinite(V))):
        nan = np.full(n, np.nan)
        out = (nan, np.full((n, n), np.nan), -1)
        return out + (det,) if details else out

    # O1: operator in the basis of the previous eigenvectors.
    W = A @ V
    At = V.T @ W
    At = 0.5 * (At + At.T)
    det["At"] = At

    # O2: step length of the folded-spectrum iteration.
    if alpha is None or alpha <= 0.0:
        alpha_v, glo, ghi = gershgorin_alpha(At, fs_power)
        det["gershgorin"] = (glo, ghi)
    else:
        alpha_v = float(alpha)
    det["alpha"] = alpha_v

    # O3 + O4: submatrix eigenproblems give start vectors and shifts.
    X = np.zeros((n, n))
    eps = np.zeros(n)
    wins = window_layout(n, part_offsets, halo)
    for win in wins:
        B = At[win.wstart:win.wstart + win.wsize, win.wstart:win.wstart + win.wsize]
        mu, Y, _ = jacobi_eigh(B)
        sel = slice(win.offset, win.offset + win.size)
        X[win.wstart:win.wstart + win.wsize, win.start:win.start + win.size] = Y[:, sel]
        eps[win.start:win.start + win.size] = mu[sel]
    det["windows"] = wins
    det["X0"] = X.copy()
    det["eps"] = eps.copy()

    # O5: folded-spectrum iterations, each column with its own shift.
    X = fs_iterate(At, X, eps, alpha_v, iterations, fs_power, shift_mode)
    det["X_fs"] = X.copy()

    # O6: Gram-Schmidt in column order, computed as Cholesky-QR: X <- X L^{-T}.
    S = X.T @ X
    L, info = cholesky_lower(S)
    det["S"] = S
    det["L"] = L
    if info != 0:
        out = (np.full(n, np.nan), np.full((n, n), np.nan), info)
        return out + (det,) if details else out
    X = solve_triangular(L, X.T, lower=True).T
    det["X_orth"] = X.copy()

    # O7: eigenvalue estimates are the Rayleigh quotients x^T At x.
    lam = np.sum(X * (At @ X), axis=0)

    # O8: sign convention, back to the original basis, ascending order.
    X = sign_normalize(X)
    Vn = V @ X
    perm = np.argsort(lam, kind="stable")
    det["lam_unsorted"] = lam.copy()
    det["perm"] = perm
    out = (lam[perm], np.ascontiguousarray(Vn[:, perm]), 0)
    return out + (det,) if details else out


def residual_norm(A: np.ndarray, lam: np.ndarray, V: np.ndarray) -> float:
    """||A V - V diag(lam)||_F / ||A||_F."""
    return float(np.linalg.norm(A @ V - V * lam[None, :]) / np.linalg.norm(A))


def orthogonality(V: np.ndarray) -> float:
    """||V^T V - I||_F."""
    return float(np.linalg.norm(V.T @ V - np.eye(V.shape[1])))


def eig_error(lam: np.ndarray, lam_ref: np.ndarray) -> float:
    """Normwise eigenvalue error max_i |lam_i - ref_i| / max_j |ref_j|."""
    return float(np.max(np.abs(lam - lam_ref)) / np.max(np.abs(lam_ref)))


def clusters(lam: np.ndarray, tol: float) -> List[np.ndarray]:
    """Groups of consecutive (ascending) eigenvalues whose neighbour gaps are <= tol."""
    groups = []
    cur = [0]
    for i in range(1, len(lam)):
        if lam[i] - lam[i - 1] <= tol:
            cur.append(i)
        else:
            groups.append(np.array(cur))
            cur = [i]
    if len(lam):
        groups.append(np.array(cur))
    return groups


def max_subspace_angle(V1: np.ndarray, V2: np.ndarray, groups: List[np.ndarray]) -> float:
    """Largest sine of the angle between span(V1[:, g]) and span(V2[:, g]) over the groups."""
    worst = 0.0
    for g in groups:
        Q1 = V1[:, g]
        Q2 = V2[:, g]
        # sin of the largest principal angle: ||(I - Q2 Q2^T) Q1||_2
        R = Q1 - Q2 @ (Q2.T @ Q1)
        worst = max(worst, float(np.linalg.norm(R, 2)))
    return worst
