"""SCF driver with the full-diagonalisation fallback on the GPU: the full
diagonalisation (a plan whose single submatrix is the whole matrix) against the
oracle's step with that layout and against LAPACK; a PFSM sequence that starts
with full steps; and a fall back when the previous eigenvectors no longer fit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle.pfsm_ref import eig_error, orthogonality, pfsm_ref, residual_norm  # noqa: E402
from pfsm_workloads import prescribed_problem, scf_sequence, uniform_layout  # noqa: E402


@pytest.fixture(scope="module")
def pf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_1502_07806_amd as pf
    pf.load_library()
    return pf


def _random_symmetric(n, seed):
    g = np.random.default_rng(seed)
    G = g.standard_normal((n, n))
    return 0.5 * (G + G.T)


def _random_orthogonal(n, seed):
    g = np.random.default_rng(seed)
    Q, R = np.linalg.qr(g.standard_normal((n, n)))
    return Q * np.sign(np.diag(R))[None, :]


@pytest.mark.parametrize("n,basis", [(300, "identity"), (640, "identity"), (640, "orthogonal")])
def test_full_diag_parity(pf, n, basis):
    dev = torch.device("cuda:0")
    A = _random_symmetric(n, n)
    V = np.eye(n) if basis == "identity" else _random_orthogonal(n, n + 1)
    fd = pf.FullDiag(n)
    lam, Vo = fd.solve(torch.from_numpy(A).to(dev), torch.from_numpy(V).to(dev))
    lam, Vo = lam.cpu().numpy(), Vo.cpu().numpy()
    lam_ref, V_ref, info = pfsm_ref(A, V, [0, n], halo=0, iterations=0)
    assert info == 0
    assert eig_error(lam, lam_ref) <= 1e-13
    assert eig_error(lam, np.linalg.eigvalsh(A)) <= 1e-13
    # the block Jacobi leaves off-diagonal entries below its noise floor of
    # 256 u ||B||, so residual and orthogonality scale like 256 u n
    floor = 256 * 2.0 ** -53 * n
    assert residual_norm(A, lam, Vo) <= floor
    assert orthogonality(Vo) <= floor
    # non-degenerate random spectrum: each eigenvector agrees with the oracle's (same signs)
    gaps = np.diff(lam_ref)
    tol = 1e-13 * np.abs(lam_ref).max() / np.minimum(np.r_[gaps, np.inf], np.r_[np.inf, gaps])
    assert np.all(np.abs(Vo - V_ref).max(axis=0) <= 100 * tol + 1e-12)


def test_scf_sequence_switches_to_pfsm(pf):
    dev = torch.device("cuda:0")
    n = 1024
    A0 = prescribed_problem(n, n // 2, 1e-2, 2500, clusters=True, device=dev)[0]
    seq = [A0] + scf_sequence(A0, 4, 2500)
    offs = uniform_layout(n, 128)
    drv = pf.SCFDriver(n, offs, halo=64, iterations=3, full_steps=2)
    V_prev = None
    for k, A in enumerate(seq):
        Ac = A.t().contiguous().t()
        lam, V = drv.step(Ac)
        An = A.cpu().numpy()
        lam_n = lam.cpu().numpy()
        # full steps are exact to rounding; PFSM steps carry the method's own
        # truncation (three folded-spectrum iterations), checked for parity below
        assert eig_error(lam_n, np.linalg.eigvalsh(An)) <= (1e-13 if k < 2 else 1e-7)
        if k >= 2:  # PFSM step: parity with the oracle from the same previous eigenvectors
            lam_ref, _, info = pfsm_ref(An, V_prev, offs, 64, 3, 2)
            assert info == 0 and eig_error(lam_n, lam_ref) <= 1e-10
        V_prev = V.cpu().numpy()
    assert [h.method for h in drv.history] == ["full", "full", "pfsm", "pfsm", "pfsm"]
    res = [h.residual for h in drv.history]
    assert all(r <= 256 * 2.0 ** -53 * n for r in res[:2]), res
    assert all(r <= drv.residual_tol for r in res[2:]), res


def test_scf_falls_back_when_basis_no_longer_fits(pf):
    dev = torch.device("cuda:0")
    n = 512
    A0 = prescribed_problem(n, n // 2, 1e-2, 2600, device=dev)[0]
    R = _random_symmetric(n, 2601)
    drv = pf.SCFDriver(n, uniform_layout(n, 128), halo=64, full_steps=1)
    drv.step(A0.t().contiguous().t())
    lam, V = drv.step(torch.from_numpy(R).to(dev))
    assert [(h.method, h.reason) for h in drv.history] == [("full", "start"), ("full", "dominance")]
    assert drv.history[1].dominance > 1e-2
    assert eig_error(lam.cpu().numpy(), np.linalg.eigvalsh(R)) <= 1e-13
    assert residual_norm(R, lam.cpu().numpy(), V.cpu().numpy()) <= 256 * 2.0 ** -53 * n
