"""FP64 refinement of approximate eigenpairs against the original matrix.

Oracle code: test infrastructure only.  This is the last step of the
mixed-precision path (not part of the paper, whose method runs in one
precision): the vectors produced with reduced-precision products are
re-evaluated against A in FP64.

  Z = A V;  lambda_j = v_j^T z_j / v_j^T v_j   (Rayleigh quotients)
  order the estimates; runs of neighbours with gaps <= tau max|lambda| form
  clusters; each cluster's estimates are replaced by the Ritz pairs of the
  pencil (V_c^T Z_c, V_c^T V_c); isolated vectors are normalised.

Readings (the refinement is not in the paper; these choices define it):
  * tau = 1e-4: estimates closer than this (relative to max|lambda|) may have
    been mixed by the reduced-precision products, whose eigenvector error
    grows like (product error) / gap; wider clusters cost more Rayleigh-Ritz
    work without changing the eigenvalues at the 1e-8 level;
  * kmax = 32: a run longer than kmax is refined in consecutive pieces of at
    most kmax estimates (the Rayleigh-Ritz block size; vectors inside one
    piece are mixed freely, across pieces they are not);
  * each Ritz vector's sign makes its largest-magnitude coefficient on the
    piece's input vectors positive (lowest index on ties), so the output does
    not depend on the signs an eigensolver happens to return.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def cluster_bounds(lam_sorted: np.ndarray, tau: float):
    thr = tau * np.max(np.abs(lam_sorted))
    starts = [0] + [i for i in range(1, len(lam_sorted)) if not (lam_sorted[i] - lam_sorted[i - 1] <= thr)]
    ends = starts[1:] + [len(lam_sorted)]
    return list(zip(starts, ends))


def refine_ref(A: np.ndarray, V: np.ndarray, tau: float = 1e-4, kmax: int = 32):
    """Return (lam, V_out) -- ascending Ritz values and orthonormalised vectors."""
    Z = A @ V
    d = np.sum(V * Z, axis=0)
    nn = np.sum(V * V, axis=0)
    lam = d / nn
    perm = np.argsort(lam, kind="stable")
    lam_s = lam[perm]
    Vs = V[:, perm]
    Zs = Z[:, perm]
    out_l = lam_s.copy()
    out_V = Vs / np.sqrt(nn[perm])[None, :]
    for s, e in cluster_bounds(lam_s, tau):
        for p0 in range(s, e, kmax):
            p1 = min(e, p0 + kmax)
            if p1 - p0 < 2:
                continue
            Vc, Zc = Vs[:, p0:p1], Zs[:, p0:p1]
            G = Vc.T @ Zc
            G = 0.5 * (G + G.T)
            M = Vc.T @ Vc
            mu, Y = scipy.linalg.eigh(G, M)
            big = np.argmax(np.abs(Y), axis=0)  # first maximum: lowest index
            Y = Y * np.where(Y[big, np.arange(Y.shape[1])] < 0.0, -1.0, 1.0)[None, :]
            out_l[p0:p1] = mu
            out_V[:, p0:p1] = Vc @ Y
    return out_l, out_V
