"""Switching rule of the SCF driver (host logic, no GPU): full diagonalisation
for the first steps, PFSM while the previous eigenpairs nearly diagonalise the
new matrix, and a fall back to full diagonalisation on a dominance, breakdown
or residual failure."""
import math

import pytest

from paper_1502_07806_amd.scf import SCFDriver


class FakeSolver:
    """Scripted stand-in: solve() returns a tag per call or raises; diagnostics()
    returns the next scripted residual."""

    def __init__(self, name, residuals, fail_steps=()):
        self.name = name
        self.residuals = list(residuals)
        self.fail_steps = set(fail_steps)
        self.calls = 0
        self.seen_V = []

    def solve(self, A, V, check=True):
        self.seen_V.append(V)
        self.calls += 1
        if A in self.fail_steps:
            raise RuntimeError("pfsm device info -3: submatrix eigensolver did not converge")
        return ("lam", self.name, A), ("V", self.name, A)

    def diagnostics(self, A, lam, V):
        return self.residuals.pop(0), 0.0


def test_policy_sequence():
    full = FakeSolver("full", [1e-14] * 10)
    # pfsm diagnostics: (dominance, residual) per attempted step, dominance only when it fails
    pfsm = FakeSolver("pfsm", [1e-4, 1e-6,      # step 2: PFSM accepted
                               0.5,             # step 3: previous pairs too far -> full
                               1e-4,            # step 4: PFSM raises -> full
                               1e-4, math.nan,  # step 5: non-finite residual -> full
                               1e-4, 1e-2,      # step 6: residual above tolerance -> full
                               1e-3, 1e-5],     # step 7: accepted
                      fail_steps={4})
    d = SCFDriver(8, [0, 8], full_steps=2, dominance_tol=1e-2, residual_tol=1e-3, pfsm=pfsm, full=full)
    outs = [d.step(k) for k in range(8)]
    methods = [(h.method, h.reason.split(":")[0]) for h in d.history]
    assert methods == [("full", "start"), ("full", "start"), ("pfsm", "dominant"), ("full", "dominance"),
                       ("full", "breakdown"), ("full", "residual"), ("full", "residual"), ("pfsm", "dominant")]
    assert [o[0][1] for o in outs] == [m for m, _ in methods]
    # the first full step starts from no basis, later ones from the previous eigenvectors
    assert full.seen_V[0] is None and full.seen_V[1] == ("V", "full", 0)
    # PFSM always rotates from the eigenvectors of the step before
    assert pfsm.seen_V[0] == ("V", "full", 1) and pfsm.seen_V[-1] == ("V", "full", 6)
    assert d.history[2].dominance == 1e-4 and d.history[2].residual == 1e-6
    assert d.history[3].dominance == 0.5
    assert not pfsm.residuals and full.calls == 6


def test_policy_rejects_no_start_steps():
    with pytest.raises(ValueError):
        SCFDriver(8, [0, 8], full_steps=0, pfsm=FakeSolver("p", []), full=FakeSolver("f", []))
