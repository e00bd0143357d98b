"""Pins of the generalized -> standard conversion oracle (Eqs. 13-15) against
facts that do not reuse its recurrence: the closed-form solution B^{-1} A, the
matrix-power form of the error, exact special cases and column independence."""
import numpy as np
import pytest

from oracle.generalized_ref import g2s_ref


def _problem(n, delta, seed):
    g = np.random.default_rng(seed)
    G = g.standard_normal((n, n))
    B = np.eye(n) + delta * (G @ G.T) / n          # SPD overlap, D^{-1}B close to I
    H = g.standard_normal((n, n))
    A = 0.5 * (H + H.T)
    return A, B


def test_converges_to_closed_form():
    A, B = _problem(60, 0.05, 1)
    Z, res, info = g2s_ref(A, B, 60)
    assert info == 0
    ref = np.linalg.solve(B, A)
    assert np.max(np.abs(Z - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(B @ Z - A)) <= 1e-12 * np.max(np.abs(A))  # Eq. 15: B Z = A


def test_error_equals_matrix_power_form():
    # Z_k - Z* = (I - D^{-1}B)^k (Z_0 - Z*): the k-step error from a matrix power
    A, B = _problem(40, 0.1, 2)
    Zs = np.linalg.solve(B, A)
    Mi = np.eye(40) - B / np.diag(B)[:, None]
    for k in (0, 1, 2, 5):
        Z, _, _ = g2s_ref(A, B, k)
        pred = Zs + np.linalg.matrix_power(Mi, k) @ (A - Zs)
        assert np.max(np.abs(Z - pred)) <= 1e-13 * np.max(np.abs(A))


def test_identity_overlap_is_exact():
    A, _ = _problem(30, 0.0, 3)
    Z, res, info = g2s_ref(A, np.eye(30), 4)
    assert info == 0 and np.array_equal(Z, A) and all(r == 0.0 for r in res)


def test_diagonal_overlap_one_step():
    A, _ = _problem(30, 0.0, 4)
    d = np.linspace(0.5, 2.0, 30)
    Z, res, _ = g2s_ref(A, np.diag(d), 1)
    assert np.max(np.abs(Z - A / d[:, None])) <= 1e-15 * np.max(np.abs(A / d[:, None]))
    Z2, res2, _ = g2s_ref(A, np.diag(d), 3)
    assert np.max(np.abs(Z2 - Z)) <= 1e-15 * np.max(np.abs(Z)) and res2[1] <= 1e-15


def test_residual_contracts():
    A, B = _problem(50, 0.05, 5)
    _, res, _ = g2s_ref(A, B, 8)
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(50) - B / np.diag(B)[:, None])))
    assert rho < 1
    for k in range(1, 8):
        assert res[k] < res[k - 1]
    assert res[-1] <= 10 * rho ** 7 * res[0]


def test_columns_are_independent():
    A, B = _problem(40, 0.05, 6)
    Z, _, _ = g2s_ref(A, B, 5)
    cols = [3, 17, 39]
    Zc, _, _ = g2s_ref(A, B, 5, cols=cols)
    assert np.array_equal(Zc, Z[:, cols]) or np.max(np.abs(Zc - Z[:, cols])) <= 1e-15 * np.max(np.abs(Z))


@pytest.mark.parametrize("bad", [0.0, -1.0, np.nan])
def test_nonpositive_diagonal_reported(bad):
    A, B = _problem(10, 0.05, 7)
    B[4, 4] = bad
    Z, res, info = g2s_ref(A, B, 3)
    assert info == -5 and res == [] and np.all(np.isnan(Z))
