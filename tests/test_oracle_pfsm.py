"""Pins of the plain PFSM oracle against what the paper and the mathematics fix.

Each test checks a different part through a route that does not repeat the
oracle's own arithmetic: closed forms (basis change, folded-spectrum map in
the eigenbasis), library special cases (Householder QR for Gram-Schmidt),
exact special cases (one full window, unperturbed basis, block-diagonal
operator, exact eigenpair as fixed point), the failure modes the paper names,
and the paper's qualitative claim that wider submatrices approach full
diagonalisation."""
import numpy as np
import pytest
import scipy.linalg

from oracle.jacobi import jacobi_eigh
from fractions import Fraction

from oracle.pfsm_ref import (clusters, eig_error, fs_iterate, gershgorin_alpha, max_subspace_angle, orthogonality,
                             pfsm_ref, residual_norm, sign_normalize, window_layout)
from pfsm_workloads import antisym_k, householder_q, prescribed_problem, spectrum, uniform_layout


@pytest.fixture(scope="module")
def c1():
    A, V, lam, Q = prescribed_problem(256, 128, 1e-2, 1000)
    return A.numpy(), V.numpy(), lam, Q.numpy()


def test_window_layout_reading():
    w = window_layout(256, [0, 64, 128, 192, 256], 32)
    assert [(x.wstart, x.wsize, x.offset) for x in w] == [(0, 128, 0), (32, 128, 32), (96, 128, 32), (128, 128, 64)]
    w = window_layout(100, [0, 30, 70, 100], 10)  # uneven slices
    assert [(x.start, x.size, x.wstart, x.wsize, x.offset) for x in w] == [
        (0, 30, 0, 50, 0), (30, 40, 20, 60, 10), (70, 30, 50, 50, 20)]
    for x in w:
        assert x.wstart <= x.start and x.start + x.size <= x.wstart + x.wsize


def test_basis_change_closed_form(c1):
    A, V, lam, Q = c1
    K = antisym_k(256, 1e-2, 1003).numpy()
    # V = Q exp(K) and A = Q diag(lam) Q^T  =>  V^T A V = exp(-K) diag(lam) exp(K), independent of Q.
    E = scipy.linalg.expm(K)
    At_cf = E.T @ np.diag(lam) @ E
    _, _, _, det = pfsm_ref(A, V, uniform_layout(256, 64), 32, details=True)
    assert np.abs(det["At"] - At_cf).max() <= 1e-13
    assert np.array_equal(det["At"], det["At"].T)


def test_gershgorin_alpha_bounds(c1):
    A, V, lam, Q = c1
    _, _, _, det = pfsm_ref(A, V, uniform_layout(256, 64), 32, details=True)
    lo, hi = det["gershgorin"]
    ev = np.linalg.eigvalsh(det["At"])
    assert lo <= ev.min() and ev.max() <= hi  # Gershgorin circle theorem
    assert det["alpha"] * (hi - lo) ** 2 == pytest.approx(1.0, rel=1e-15)
    # every folded eigenvalue 1 - alpha (l - eps)^2 lies in [0, 1] for all shifts
    fold = 1.0 - det["alpha"] * (ev[:, None] - det["eps"][None, :]) ** 2
    assert fold.min() >= 0.0 and fold.max() <= 1.0
    a1, lo1, hi1 = gershgorin_alpha(np.diag([1.0, 3.0]), 1)
    assert (a1, lo1, hi1) == (0.5, 1.0, 3.0)


def test_single_full_window_is_exact(c1):
    A, V, lam, Q = c1
    lam_p, Vn, info = pfsm_ref(A, V, [0, 256], halo=0)
    assert info == 0
    assert eig_error(lam_p, lam) <= 1e-13
    assert residual_norm(A, lam_p, Vn) <= 1e-13 and orthogonality(Vn) <= 1e-12


def test_unperturbed_basis_is_exact(c1):
    A, V, lam, Q = c1
    lam_p, Vn, info, det = pfsm_ref(A, Q, uniform_layout(256, 64), 32, details=True)
    assert info == 0 and eig_error(lam_p, lam) <= 1e-14
    # every output vector is a column of Q with its sign: in the rotated basis the
    # vectors are unit vectors e_j (up to rounding), whose largest entry the sign
    # convention makes positive, so V_new = Q X = Q without any sign flip
    assert np.abs(np.sum(Vn * Q, axis=0) - 1.0).max() <= 1e-13


def test_block_diagonal_operator_is_exact():
    n, m, h = 96, 24, 8
    offs = uniform_layout(n, m)
    blocks = []
    for p in range(n // m):  # separated spectra: block p lives in [p, p + 0.5]
        Qb = householder_q(m, 900 + p).numpy()
        lb = p + 0.5 * np.random.default_rng(p).random(m)
        blocks.append((Qb * lb) @ Qb.T)
    A = scipy.linalg.block_diag(*blocks)
    A = 0.5 * (A + A.T)
    lam_p, Vn, info = pfsm_ref(A, np.eye(n), offs, halo=h)
    ref = np.linalg.eigvalsh(A)
    assert info == 0 and np.abs(lam_p - ref).max() <= 1e-13
    assert residual_norm(A, lam_p, Vn) <= 1e-13


def test_zero_iterations_is_householder_qr(c1):
    A, V, lam, Q = c1
    _, _, _, det = pfsm_ref(A, V, uniform_layout(256, 64), 32, iterations=0, details=True)
    Qr, R = np.linalg.qr(det["X0"])
    Qr = Qr * np.sign(np.diag(R))[None, :]  # Gram-Schmidt convention: diag(R) > 0
    assert np.abs(det["X_orth"] - Qr).max() <= 1e-12


@pytest.mark.parametrize("q", [1, 2])
def test_folded_spectrum_closed_form(c1, q):
    A, V, lam, Q = c1
    nit = 3
    _, _, _, det = pfsm_ref(A, V, uniform_layout(256, 64), 32, iterations=nit, fs_power=q, details=True)
    At, X0, eps, alpha = det["At"], det["X0"], det["eps"], det["alpha"]
    w, U = np.linalg.eigh(At)
    # In At's eigenbasis the map multiplies component k of column i by (1 - alpha (w_k - eps_i)^q)^nit.
    f = (1.0 - alpha * (w[:, None] - eps[None, :]) ** q) ** nit
    X_cf = U @ (f * (U.T @ X0))
    assert np.abs(det["X_fs"] - X_cf).max() <= 1e-12


def test_exact_eigenpair_is_fixed_point():
    n = 64
    lam_ex = np.linspace(-1, 1, n)
    A = np.diag(lam_ex)  # V = I: every start vector from a window of a diagonal matrix is exact
    _, _, _, det = pfsm_ref(A, np.eye(n), uniform_layout(n, 16), 8, iterations=5, details=True)
    assert np.array_equal(np.abs(det["X_fs"]), np.abs(det["X0"]))


def test_wider_windows_and_more_iterations_approach_full_diagonalisation(c1):
    A, V, lam, Q = c1
    offs = uniform_layout(256, 64)
    errs = [eig_error(pfsm_ref(A, V, offs, halo=h)[0], lam) for h in (0, 16, 32, 64, 96)]
    assert all(errs[i + 1] <= errs[i] * 1.05 for i in range(len(errs) - 1))
    assert errs[-1] < 0.5 * errs[0]
    errs_it = [eig_error(pfsm_ref(A, V, offs, halo=16, iterations=k)[0], lam) for k in (0, 3, 30)]
    assert errs_it[2] < errs_it[1] < errs_it[0]
    lam_full = pfsm_ref(A, V, offs, halo=128)[0]  # every window is the whole matrix
    assert eig_error(lam_full, lam) <= 1e-13


def test_outputs_sorted_orthonormal_and_residual(c1):
    A, V, lam, Q = c1
    for q in (1, 2):
        lam_p, Vn, info = pfsm_ref(A, V, uniform_layout(256, 64), 32, fs_power=q)
        assert info == 0 and np.all(np.diff(lam_p) >= 0)
        assert orthogonality(Vn) <= 1e-12
        # the method error is far below the spacing but not zero
        assert 1e-12 < eig_error(lam_p, lam) < 1e-6
        assert residual_norm(A, lam_p, Vn) < 1e-3


def test_rayleigh_shift_mode_runs(c1):
    A, V, lam, Q = c1
    lam_p, Vn, info = pfsm_ref(A, V, uniform_layout(256, 64), 32, shift_mode="rayleigh")
    assert info == 0 and eig_error(lam_p, lam) < 1e-6


def _fs_exact(w, x0, alpha, iterations, q, rayleigh):
    """Folded-spectrum iterations on a diagonal operator diag(w) in exact rational
    arithmetic: component k of x is multiplied by 1 - alpha (w_k - eps)^q, the
    shift being the Rayleigh quotient sum w_k x_k^2 / sum x_k^2 of the current
    vector (refreshed shift) or the given one (fixed shift)."""
    x = [Fraction(v) for v in x0]
    eps = Fraction(rayleigh[1]) if not rayleigh[0] else None
    for _ in range(iterations):
        if rayleigh[0]:
            eps = sum(wk * xk * xk for wk, xk in zip(w, x)) / sum(xk * xk for xk in x)
        x = [(1 - alpha * (wk - eps) ** q) * xk for wk, xk in zip(w, x)]
    return [float(v) for v in x]


@pytest.mark.parametrize("q", [1, 2])
def test_rayleigh_shift_hand_case(q):
    # At = diag(0, 1, 3), x0 = (1, 1, 1): the refreshed shift of the first
    # iteration is 4/3; alpha = 1/10.  After one q = 2 iteration the vector is
    # (74, 89, 65)/90 and the next shift 20596/17622.
    w = [Fraction(0), Fraction(1), Fraction(3)]
    alpha = Fraction(1, 10)
    At = np.diag([0.0, 1.0, 3.0])
    x0 = np.ones((3, 1))
    X1 = fs_iterate(At, x0, np.array([0.5]), 0.1, 1, q, "rayleigh")  # the given shift is replaced
    if q == 2:
        assert np.allclose(X1[:, 0], [74 / 90, 89 / 90, 65 / 90], rtol=0, atol=1e-15)
    for it in (1, 2, 4):
        X = fs_iterate(At, x0, np.array([0.5]), 0.1, it, q, "rayleigh")
        ref = _fs_exact(w, [1, 1, 1], alpha, it, q, (True, None))
        assert np.abs(X[:, 0] - ref).max() <= 1e-14
        # the fixed shift keeps 0.5 for every iteration
        Xf = fs_iterate(At, x0, np.array([0.5]), 0.1, it, q, "fixed")
        assert np.abs(Xf[:, 0] - _fs_exact(w, [1, 1, 1], alpha, it, q, (False, Fraction(1, 2)))).max() <= 1e-14
        assert np.abs(Xf - X).max() > 1e-3  # the two shift rules differ on this vector


@pytest.mark.parametrize("q", [1, 2])
def test_rayleigh_shift_closed_form(c1, q):
    A, V, lam, Q = c1
    nit = 3
    _, _, _, det = pfsm_ref(A, V, uniform_layout(256, 64), 32, iterations=nit, fs_power=q, shift_mode="rayleigh",
                            details=True)
    At, X0, alpha = det["At"], det["X0"], det["alpha"]
    w, U = np.linalg.eigh(At)
    # in At's eigenbasis the Rayleigh quotient of a column c is sum w_k c_k^2 / sum c_k^2, and the
    # iteration scales component k by 1 - alpha (w_k - eps)^q
    C = U.T @ X0
    for _ in range(nit):
        eps = np.sum(w[:, None] * C * C, axis=0) / np.sum(C * C, axis=0)
        C = (1.0 - alpha * (w[:, None] - eps[None, :]) ** q) * C
    assert np.abs(det["X_fs"] - U @ C).max() <= 1e-12


def test_sign_convention_hand_built_columns():
    # largest |entry| positive; among equal magnitudes the lowest row decides
    X = np.array([[1.0, -3.0, 2.0, -2.0, 0.0, 0.0],
                  [-2.0, 1.0, -2.0, 2.0, 0.0, 0.0],
                  [0.5, 2.0, 1.0, 0.0, -1e-300, 0.0]])
    Y = sign_normalize(X)
    assert np.array_equal(Y, X * np.array([-1.0, -1.0, 1.0, -1.0, -1.0, 1.0])[None, :])
    # idempotent, and a column and its negative map to the same column
    assert np.array_equal(sign_normalize(Y), Y)
    assert np.array_equal(sign_normalize(-X), Y)


def test_uneven_slices(c1):
    A, V, lam, Q = c1
    lam_p, Vn, info = pfsm_ref(A, V, [0, 40, 100, 180, 256], halo=24)
    assert info == 0 and eig_error(lam_p, lam) < 1e-6 and orthogonality(Vn) <= 1e-12


def test_failure_modes(c1):
    A, V, lam, Q = c1
    offs = uniform_layout(256, 64)
    V2 = V.copy()
    V2[:, 5] = V2[:, 4]  # duplicated previous eigenvector: the overlap matrix is singular
    assert pfsm_ref(A, V2, offs, 32)[2] > 0
    A2 = A.copy()
    A2[3, 7] = np.nan
    assert pfsm_ref(A2, V, offs, 32)[2] == -1
    # A randomly mixed basis (not diagonally dominant): estimates fail to resolve the spectrum.
    R = householder_q(256, 4242).numpy()
    lam_bad, _, info = pfsm_ref(A, R, offs, 32)
    assert info != 0 or eig_error(lam_bad, lam) > 1e-3


def test_cluster_helpers():
    lam = np.array([0.0, 0.0, 1e-12, 1.0, 2.0, 2.0 + 1e-11])
    g = clusters(lam, 1e-10)
    assert [list(x) for x in g] == [[0, 1, 2], [3], [4, 5]]
    V = np.eye(6)
    W = V.copy()
    W[:, [0, 1]] = W[:, [1, 0]]
    assert max_subspace_angle(V, W, g) == 0.0
