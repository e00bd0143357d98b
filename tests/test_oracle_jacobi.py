"""Pins of the cyclic-Jacobi oracle against facts fixed by the mathematics:
the 2x2 closed form, prescribed spectra (Weyl), trace / Frobenius invariants,
orthonormality, and brute force against two independent routines (LAPACK's
eigh through numpy, and bisection on the inertia of an LDL^T factorisation)."""
import numpy as np
import pytest
import scipy.linalg

from oracle.jacobi import jacobi_eigh
from pfsm_workloads import householder_q, spectrum

U64 = 2.0 ** -53


def _sym(n, seed):
    g = np.random.default_rng(seed)
    G = g.standard_normal((n, n))
    return 0.5 * (G + G.T)


@pytest.mark.parametrize("a,b,c", [(1.0, 0.5, -2.0), (3.0, 0.0, 3.0), (2.0, 1e-9, 2.0), (-1.0, 4.0, 7.0),
                                   (0.0, 1.0, 0.0), (5.0, -2.5, 1.0)])
def test_2x2_closed_form(a, b, c):
    lam, U, _ = jacobi_eigh(np.array([[a, b], [b, c]]))
    m = 0.5 * (a + c)
    r = np.hypot(0.5 * (a - c), b)
    assert np.allclose(lam, [m - r, m + r], rtol=0, atol=4 * U64 * max(abs(a), abs(b), abs(c)))
    A = np.array([[a, b], [b, c]])
    assert np.abs(A @ U - U * lam).max() <= 8 * U64 * max(abs(a), abs(b), abs(c))


@pytest.mark.parametrize("n,clusters", [(48, False), (96, True), (160, True)])
def test_prescribed_spectrum(n, clusters):
    lam_ex = spectrum(n, n // 2, 11 + n, clusters)
    Q = householder_q(n, 12 + n).numpy()
    A = (Q * lam_ex) @ Q.T
    A = 0.5 * (A + A.T)
    lam, U, sweeps = jacobi_eigh(A)
    normA = np.linalg.norm(A, 2)
    # Weyl: a backward-stable result is within c * n * u * ||A|| of the exact spectrum.
    assert np.max(np.abs(lam - lam_ex)) <= 4 * n * U64 * normA
    assert np.abs(U.T @ U - np.eye(n)).max() <= 4 * n * U64
    assert np.linalg.norm(A @ U - U * lam) <= 4 * n * U64 * np.linalg.norm(A)
    assert 1 <= sweeps <= 20


@pytest.mark.parametrize("n", [3, 17, 64])
def test_invariants(n):
    A = _sym(n, n)
    lam, U, _ = jacobi_eigh(A)
    assert abs(lam.sum() - np.trace(A)) <= 8 * n * U64 * np.abs(A).sum()
    assert abs(np.sum(lam ** 2) - np.sum(A ** 2)) <= 8 * n * U64 * np.sum(A ** 2)
    assert np.all(np.diff(lam) >= 0)
    assert np.allclose(U @ np.diag(lam) @ U.T, A, rtol=0, atol=8 * n * U64 * np.abs(A).max())


def _count_below(A, sigma):
    """Number of eigenvalues < sigma from the inertia of LDL^T(A - sigma I) (Sylvester)."""
    _, D, _ = scipy.linalg.ldl(A - sigma * np.eye(A.shape[0]))
    return int(np.sum(np.linalg.eigvalsh(D) < 0))  # D is block diagonal with 1x1 / 2x2 blocks


def _bisect_eigs(A, tol=1e-13):
    n = A.shape[0]
    r = np.abs(A).sum(axis=1).max()
    out = []
    for k in range(n):  # k-th smallest: smallest sigma with count_below(sigma) > k
        lo, hi = -r - 1.0, r + 1.0
        while hi - lo > tol * max(1.0, r):
            mid = 0.5 * (lo + hi)
            if _count_below(A, mid) > k:
                hi = mid
            else:
                lo = mid
        out.append(0.5 * (lo + hi))
    return np.array(out)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 16])
def test_brute_force_small(n):
    for seed in range(3):
        A = _sym(n, 100 * n + seed)
        lam, U, _ = jacobi_eigh(A)
        ref = np.linalg.eigh(A)
        assert np.max(np.abs(lam - ref[0])) <= 16 * n * U64 * max(1.0, np.abs(ref[0]).max())
        # eigenvectors agree up to sign for the (generically simple) spectrum
        dots = np.abs(np.sum(U * ref[1], axis=0))
        assert np.all(np.abs(dots - 1.0) <= 1e-10)
        bis = _bisect_eigs(A)
        assert np.max(np.abs(lam - bis)) <= 1e-11 * max(1.0, np.abs(lam).max())


def test_degenerate_cluster_and_diagonal():
    n = 40
    lam_ex = np.repeat(np.linspace(-1, 1, 10), 4)
    Q = householder_q(n, 77).numpy()
    A = (Q * lam_ex) @ Q.T
    A = 0.5 * (A + A.T)
    lam, U, _ = jacobi_eigh(A)
    assert np.max(np.abs(lam - lam_ex)) <= 1e-13
    for c in range(10):  # each 4-dim eigenspace is spanned exactly
        cols = U[:, 4 * c:4 * c + 4]
        P_ex = Q[:, 4 * c:4 * c + 4]
        assert np.linalg.norm(cols - P_ex @ (P_ex.T @ cols), 2) <= 1e-12
    d = np.array([3.0, -1.0, 2.0, 0.0])
    lam, U, sweeps = jacobi_eigh(np.diag(d))
    assert sweeps == 1 and np.array_equal(lam, np.sort(d))
    assert np.array_equal(np.abs(U), np.eye(4)[:, np.argsort(d, kind="stable")])


def test_empty_and_scalar():
    lam, U, _ = jacobi_eigh(np.zeros((0, 0)))
    assert lam.shape == (0,)
    lam, U, _ = jacobi_eigh(np.array([[2.5]]))
    assert lam[0] == 2.5 and U[0, 0] == 1.0
