"""Oracle (test infrastructure only; never imported by the product path):
conversion of the generalized problem A x = lambda B x to standard form as the
paper's Implementation section describes it (Eqs. 13-15).

Z = B^{-1} A is reached without forming B^{-1}: with D the diagonal of B,

    Z_{n+1} = (I - D^{-1} B) Z_n + D^{-1} A,

whose fixed point satisfies B Z = A (Eq. 15).  The paper takes the identity as
the initial approximation of B^{-1} (B is diagonally dominant, and differs
from I only through the ultrasoft pseudopotential terms), so Z_0 = A.  Each
column of Z evolves on its own.  The iteration converges when the spectral
radius of I - D^{-1} B is below one.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def g2s_ref(A: np.ndarray, B: np.ndarray, iterations: int, cols: Sequence[int] = None
            ) -> Tuple[np.ndarray, List[float], int]:
    """Iterate Eq. 14 `iterations` times from Z_0 = A.

    Returns (Z, res, info): res[k] = ||A - B Z_k||_F / ||A||_F for k < iterations
    (the residual of the iterate each step starts from), info = -5 when a
    diagonal entry of B is not a positive finite number (no iteration then).
    With `cols`, only those columns of Z are computed (columns are independent).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    d = np.diag(B).copy()
    if not np.all(np.isfinite(d) & (d > 0.0)):
        return np.full(A.shape if cols is None else (A.shape[0], len(cols)), np.nan), [], -5
    Acols = A if cols is None else A[:, list(cols)]
    Dinv_B = B / d[:, None]               # D^{-1} B
    Dinv_A = Acols / d[:, None]           # D^{-1} A
    M = np.eye(B.shape[0]) - Dinv_B      # I - D^{-1} B
    Z = Acols.copy()                      # Z_0 = A
    na = np.linalg.norm(Acols)
    res = []
    for _ in range(iterations):
        res.append(float(np.linalg.norm(Acols - B @ Z) / na) if na > 0 else 0.0)
        Z = M @ Z + Dinv_A
    return Z, res, 0
