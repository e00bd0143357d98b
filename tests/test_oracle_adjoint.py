"""Pins of the eigen-adjoint oracle: the Hellmann-Feynman special case,
central finite differences through an exact forward solve, symmetry, and a
finite result at an exact degeneracy."""
import numpy as np
import pytest

from oracle.adjoint_ref import central_fd, eigh_adjoint, lorentz_f, occupied_loss, occupied_loss_grads
from oracle.jacobi import jacobi_eigh
from pfsm_workloads import householder_q, loss_weights, random_symmetric_unit, spectrum


def _problem(n, seed):
    lam = spectrum(n, n // 2, seed, clusters=False)
    Q = householder_q(n, seed + 1).numpy()
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T)


def test_hellmann_feynman():
    A = _problem(24, 31)
    lam, V, _ = jacobi_eigh(A)
    w = np.random.default_rng(0).random(24)
    G = eigh_adjoint(lam, V, w, None)
    assert np.allclose(G, (V * w) @ V.T, atol=1e-14)
    assert np.array_equal(G, G.T)


def test_finite_differences_occupied_loss():
    n, nocc = 64, 32
    A = _problem(n, 5000)
    w, d = loss_weights(nocc, n, 5000)

    def loss(M):
        lam, V, _ = jacobi_eigh(M)
        return occupied_loss(lam, V, w, d)

    lam, V, _ = jacobi_eigh(A)
    dlam, dV = occupied_loss_grads(lam, V, w, d)
    G = eigh_adjoint(lam, V, dlam, dV, eta=1e-8)
    h = 1e-5 * np.linalg.norm(A, 2)
    for k in range(8):
        E = random_symmetric_unit(n, 7000 + k)
        fd = central_fd(loss, A, E, h)
        assert abs(np.sum(G * E) - fd) / max(abs(fd), 1e-12) <= 1e-6


def test_degenerate_pair_is_finite():
    lam = np.array([0.0, 1.0, 1.0, 2.0])
    F = lorentz_f(lam, 1e-8)
    assert F[1, 2] == 0.0 and F[2, 1] == 0.0 and F[0, 1] == pytest.approx(1.0)
    V = np.eye(4)
    G = eigh_adjoint(lam, V, np.ones(4), np.ones((4, 4)))
    assert np.all(np.isfinite(G))


def test_lorentzian_matches_plain_inverse_away_from_degeneracy():
    lam = np.array([-1.0, -0.25, 0.5, 3.0])
    F = lorentz_f(lam, 1e-8)
    plain = 1.0 / (lam[None, :] - lam[:, None] + np.eye(4)) * (1 - np.eye(4))
    assert np.allclose(F, plain, rtol=1e-15, atol=0)
