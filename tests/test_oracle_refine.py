"""Pins of the FP64 refinement oracle: exact eigenvectors are fixed points;
a small rotation of the exact eigenvectors leaves Rayleigh quotients with a
second-order error that the cluster Rayleigh-Ritz removes inside clusters;
degenerate clusters come back exactly; a 2x2 case matches its closed form."""
import numpy as np
import scipy.linalg

from oracle.refine_ref import cluster_bounds, refine_ref
from pfsm_workloads import antisym_k, expm_small, householder_q, spectrum


def _problem(n, seed, clusters=False):
    lam = spectrum(n, n // 4, seed, clusters)
    Q = householder_q(n, seed + 1).numpy()
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), lam, Q


def test_exact_vectors_fixed_point():
    A, lam, Q = _problem(96, 11)
    l, V = refine_ref(A, Q)
    assert np.max(np.abs(l - lam)) <= 1e-14
    assert np.max(np.abs(np.abs(np.sum(V * Q, 0)) - 1)) <= 1e-13


def test_rotated_vectors_second_order():
    n = 128
    A, lam, Q = _problem(n, 21, clusters=True)
    for kappa in (1e-3, 1e-4):
        R = expm_small(antisym_k(n, kappa, 5)).numpy()
        V = (Q @ R) * (1.0 + 1e-6 * np.arange(n))[None, :]  # unnormalised on purpose
        l, Vo = refine_ref(A, V)
        # Rayleigh quotients are second order in the vector error (Weyl-type bound kappa^2 ||A||)
        assert np.max(np.abs(l - lam)) <= 4 * kappa ** 2 * np.max(np.abs(lam))
        assert np.max(np.abs(np.sum(Vo * Vo, 0) - 1)) <= 1e-13
    # exactly degenerate clusters (3-fold every 32 levels) come back exactly from a mixed basis
    V = Q.copy()
    c = V[:, 0:3] @ scipy.linalg.expm(np.array([[0, 0.3, -0.2], [-0.3, 0, 0.5], [0.2, -0.5, 0]]))
    V[:, 0:3] = c
    l, _ = refine_ref(A, V)
    assert np.max(np.abs(l[:3] - lam[:3])) <= 1e-14


def test_close_pair_resolved_by_cluster():
    # two eigenvalues 1e-9 apart, vectors mixed by 45 degrees: Rayleigh quotients alone give the
    # midpoint, the 2x2 Ritz problem gives both exactly
    lam = np.array([-1.0, 0.5, 0.5 + 1e-9, 2.0])
    Q = householder_q(4, 3).numpy()
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    V = Q.copy()
    c, s = np.cos(np.pi / 4), np.sin(np.pi / 4)
    V[:, 1], V[:, 2] = c * Q[:, 1] + s * Q[:, 2], -s * Q[:, 1] + c * Q[:, 2]
    l, Vo = refine_ref(A, V, tau=1e-6)
    assert np.max(np.abs(l - lam)) <= 1e-15 * 4
    l_nocluster, _ = refine_ref(A, V, tau=0.0)
    assert abs(l_nocluster[1] - 0.5 - 0.5e-9) < 1e-12  # midpoint without the cluster step


def test_cluster_bounds():
    lam = np.array([0.0, 1e-6, 2e-6, 1.0, 1.0, 3.0])
    assert cluster_bounds(lam, 1e-5) == [(0, 3), (3, 5), (5, 6)]
    assert cluster_bounds(lam, 0.0) == [(0, 1), (1, 2), (2, 3), (3, 5), (5, 6)]
