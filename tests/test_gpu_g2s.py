"""Generalized -> standard conversion on the GPU (Implementation section,
Eqs. 13-15) against the oracle: element-wise parity of Z and of the residual
history on ragged sizes, the even/odd iterate buffer handling, padded leading
dimensions, the bad-diagonal report, and sampled columns at N = 8192."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle.generalized_ref import g2s_ref  # noqa: E402
from pfsm_workloads import overlap_matrix, prescribed_problem  # noqa: E402


@pytest.fixture(scope="module")
def pf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_1502_07806_amd as pf
    pf.load_library()
    return pf


def _problem(n, delta, seed, dev):
    A = prescribed_problem(n, n // 2, 1e-2, seed)[0]
    B = overlap_matrix(n, delta, seed + 7)
    return A, B, A.to(dev), B.to(dev)


# rounding of one FP64 product per step, amplified by at most 1/(1 - rho) over the steps
TOL = 1e-13


@pytest.mark.parametrize("n,it", [(300, 6), (1000, 5), (129, 1), (257, 0)])
def test_g2s_parity(pf, n, it):
    dev = torch.device("cuda:0")
    A, B, Ad, Bd = _problem(n, 0.05, 6000 + n, dev)
    Z, res, info = pf.generalized_to_standard(Ad, Bd, it, residuals=True)
    Zr, resr, infor = g2s_ref(A.numpy(), B.numpy(), it)
    assert int(info.item()) == infor == 0
    Zg = Z.cpu().numpy()
    assert np.max(np.abs(Zg - Zr)) <= TOL * np.max(np.abs(Zr))
    assert np.allclose(res.cpu().numpy(), np.array(resr), rtol=1e-10, atol=1e-14)
    if it == 0:
        assert np.array_equal(Zg, A.numpy())


def test_g2s_converges_to_solution(pf):
    """Enough steps reach B^{-1} A (Eq. 15) to rounding."""
    dev = torch.device("cuda:0")
    A, B, Ad, Bd = _problem(512, 0.05, 6100, dev)
    Z, res, _ = pf.generalized_to_standard(Ad, Bd, 30, residuals=True)
    ref = np.linalg.solve(B.numpy(), A.numpy())
    assert np.max(np.abs(Z.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    r = res.cpu().numpy()
    assert np.all(np.diff(r[:10]) < 0)


def test_g2s_padded_leading_dims(pf):
    dev = torch.device("cuda:0")
    n = 200
    A, B, Ad, Bd = _problem(n, 0.05, 6200, dev)
    big = torch.zeros((n, n + 13), dtype=torch.float64, device=dev)
    big[:, :n] = Ad.t()
    A_view = big[:, :n].t()  # column-major with stride(1) = n + 13
    assert A_view.stride(0) == 1 and A_view.stride(1) == n + 13
    zbig = torch.zeros((n, n + 5), dtype=torch.float64, device=dev)
    Z_out = zbig[:, :n].t()
    Z, info = pf.generalized_to_standard(A_view, Bd, 4, out=Z_out)
    Zr, _, _ = g2s_ref(A.numpy(), B.numpy(), 4)
    assert np.max(np.abs(Z.cpu().numpy() - Zr)) <= TOL * np.max(np.abs(Zr))
    assert torch.all(zbig[:, n:] == 0)  # the padding columns of Z's storage are untouched


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan")])
def test_g2s_bad_diagonal(pf, bad):
    dev = torch.device("cuda:0")
    A, B, Ad, Bd = _problem(128, 0.05, 6300, dev)
    Bd[17, 17] = bad
    with pytest.raises(RuntimeError, match="-5"):
        pf.generalized_to_standard(Ad, Bd, 3)
    assert g2s_ref(A.numpy(), Bd.cpu().numpy(), 3)[2] == -5


def test_g2s_full_size_sampled_columns(pf):
    """N = 8192 (the benchmark's size and step count): sampled columns against
    the oracle, which computes only those columns (they are independent)."""
    dev = torch.device("cuda:0")
    n, it = 8192, 8
    A = prescribed_problem(n, n // 4, 5e-3, 3000, clusters=True, device=dev)[0]
    B = overlap_matrix(n, 0.05, 6007, device=dev)
    Z, res, info = pf.generalized_to_standard(A, B, it, residuals=True)
    cols = [0, 1, 777, 4095, 4096, 8191]
    Zr, resr, _ = g2s_ref(A.cpu().numpy(), B.cpu().numpy(), it, cols=cols)
    Zs = Z[:, cols].cpu().numpy()
    assert np.max(np.abs(Zs - Zr)) <= TOL * np.max(np.abs(Zr))
    assert res.cpu().numpy()[-1] < 1e-5 * res.cpu().numpy()[0]
