"""GPU refinement of the mixed path (digits of A and V on the int8 matrix
cores, Z = A V, Rayleigh quotients, cluster Rayleigh-Ritz) against the FP64
oracle refinement (oracle/refine_ref.py) fed the same estimates V.

A and V are first rounded onto grids that make their digit expansions finite
(A: ceil((s+1)/2) digits on one global grid; V: the remaining digits on each
column's own grid), so every digit pair the product keeps covers every
nonzero pair: the int8 product then equals A V up to the rounding of its
final FP64 sums, and the two refinements can be compared to 1e-12."""
import ctypes

import numpy as np
import pytest
import scipy.linalg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.refine_ref import cluster_bounds, refine_ref  # noqa: E402
from pfsm_workloads import antisym_k, householder_q, spectrum  # noqa: E402

from hooks_util import lib  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    return torch.device("cuda:0")


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _quantize_global(A, digits):
    e = int(np.max(np.frexp(np.max(np.abs(A), axis=0))[1]))
    g = np.ldexp(1.0, e - 6 - 7 * (digits - 1))
    return np.round(A / g) * g


def _quantize_cols(V, digits):
    e = np.frexp(np.max(np.abs(V), axis=0))[1]
    g = np.ldexp(1.0, e - 6 - 7 * (digits - 1))
    Vq = np.round(V / g[None, :]) * g[None, :]
    assert np.array_equal(np.frexp(np.max(np.abs(Vq), axis=0))[1], e)  # grids unchanged by the rounding
    return Vq


def _problem(n, seed, group=(300, 340)):
    """Prescribed spectrum with 3-fold clusters, plus one run of 40 eigenvalues
    1e-9 apart; V = Q exp(K) with the run's vectors strongly mixed."""
    lam = spectrum(n, n // 4, seed, clusters=True)
    a, b = group
    lam[a:b] = lam[a] + 1e-9 * np.arange(b - a)
    assert np.all(np.diff(lam) >= 0)
    Q = householder_q(n, seed + 1).numpy()
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    K = antisym_k(n, 1e-3, seed + 2).numpy()
    Kg = antisym_k(b - a, 1.0, seed + 3).numpy()
    K[a:b, a:b] += Kg
    V = Q @ scipy.linalg.expm(K)
    return A, V


def _gpu_refine(dev, A, V):
    L = lib()
    n = A.shape[0]
    s = L.pfsm_test_refine_slices()
    planes = torch.zeros(2 * L.pfsm_test_oz_plane_bytes(n, s), dtype=torch.uint8, device=dev)
    expo = torch.zeros(2 * n, dtype=torch.int32, device=dev)
    Z = torch.zeros(n * n, dtype=torch.float64, device=dev)
    rb = torch.zeros(7 * n + 8, dtype=torch.float64, device=dev)
    lam = torch.zeros(n, dtype=torch.float64, device=dev)
    Vout = torch.zeros((n, n), dtype=torch.float64, device=dev).t()  # column-major
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    dA = torch.from_numpy(A).to(dev).t().contiguous().t()
    dV = torch.from_numpy(V).to(dev).t().contiguous().t()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.pfsm_test_refine(n, _p(dA), n, _p(dV), n, _p(planes), _p(expo), _p(Z), _p(rb), _p(lam), _p(Vout), n,
                              _p(info), st) == 0
    torch.cuda.synchronize()
    ri = rb.cpu().numpy().view(np.int32)
    cnt = int(ri[2 * 7 * n])
    cstart = ri[2 * 5 * n: 2 * 5 * n + cnt]
    csize = ri[2 * 6 * n: 2 * 6 * n + cnt]
    return int(info.item()), lam.cpu().numpy(), Vout.cpu().numpy(), list(zip(cstart, cstart + csize))


@pytest.mark.parametrize("n,seed", [(640, 6401), (1100, 11001)])
def test_refine_matches_oracle_refinement(dev, n, seed):
    L = lib()
    s = L.pfsm_test_refine_slices()
    tau = L.pfsm_test_refine_tau()
    kmax = L.pfsm_test_refine_kmax()
    sa = (s + 2) // 2
    A, V = _problem(n, seed)
    A = _quantize_global(A, sa)
    V = _quantize_cols(V, s + 1 - sa)
    info, lam, Vo, bounds = _gpu_refine(dev, A, V)
    lam_ref, V_ref = refine_ref(A, V, tau=tau, kmax=kmax)
    assert info == 0
    # the same clusters of close estimates, one of them longer than a Rayleigh-Ritz piece
    d = np.sum(V * (A @ V), axis=0) / np.sum(V * V, axis=0)
    ref_bounds = cluster_bounds(np.sort(d), tau)
    assert [tuple(map(int, b)) for b in bounds] == ref_bounds
    assert max(e - b for b, e in ref_bounds) > kmax
    # eigenvalues element by element
    scale = np.max(np.abs(lam_ref))
    assert np.max(np.abs(lam - lam_ref)) <= 1e-12 * scale
    # vectors: every Rayleigh-Ritz piece as a subspace; singletons column by column (signs included)
    for b, e in ref_bounds:
        for p0 in range(b, e, kmax):
            p1 = min(e, p0 + kmax)
            if p1 - p0 == 1:
                assert np.max(np.abs(Vo[:, p0] - V_ref[:, p0])) <= 1e-12
                continue
            Q1, Q2 = Vo[:, p0:p1], V_ref[:, p0:p1]
            assert np.linalg.norm(Q1 - Q2 @ (Q2.T @ Q1), 2) <= 1e-10
            assert np.max(np.abs(Q1.T @ Q1 - np.eye(p1 - p0))) <= 1e-12
            # Ritz vectors whose Ritz values are well apart inside the piece: column by column
            mu = lam_ref[p0:p1]
            gap = np.minimum(np.r_[np.inf, np.diff(mu)], np.r_[np.diff(mu), np.inf])
            sep = gap > 1e-6 * scale
            if np.any(sep):
                assert np.max(np.abs(Q1[:, sep] - Q2[:, sep])) <= 1e-9
