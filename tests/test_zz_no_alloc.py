"""pfsm_solve_static (the entry point that allocates nothing: its workspace is
the library's own device array) against pfsm_solve with a caller workspace,
through the C ABI, on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from pfsm_workloads import prescribed_problem, uniform_layout  # noqa: E402

STATIC_BYTES = 64 << 20


@pytest.fixture(scope="module")
def pf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_1502_07806_amd as pf
    pf.load_library()
    return pf


@pytest.mark.parametrize("precision", ["fp64", "mixed_bf16"])
def test_static_matches_workspace_solve(pf, precision):
    dev = torch.device("cuda:0")
    for n, slice_, halo, seed in [(256, 64, 32, 1000), (128, 32, 16, 1128)]:  # second call: smaller
        print("static solve: precision %s n %d" % (precision, n), flush=True)
        A, V, _, _ = prescribed_problem(n, n // 2, 1e-2, seed)
        A, V = A.to(dev), V.to(dev)
        offs = uniform_layout(n, slice_)
        plan = pf.Plan(n, offs, halo=halo, precision=precision)
        assert plan.workspace_bytes <= STATIC_BYTES
        lam_w, V_w = plan.solve(A, V)
        lam_w, V_w = lam_w.clone(), V_w.clone()
        lam_s, V_s = plan.solve_static(A, V)
        torch.cuda.synchronize()
        assert int(plan.info.item()) == 0
        scale = torch.max(torch.abs(lam_w)).item()
        dl = torch.max(torch.abs(lam_s - lam_w)).item() / scale
        dv = torch.max(torch.abs(V_s - V_w)).item()
        print("  max eigenvalue difference %.3e (relative), max vector difference %.3e, bitwise equal: %s"
              % (dl, dv, torch.equal(lam_s, lam_w) and torch.equal(V_s, V_w)), flush=True)
        tol = 1e-12 if precision == "fp64" else 1e-10
        assert dl <= tol and dv <= tol


def test_static_rejects_large_plan(pf):
    """A plan whose workspace exceeds the static array is refused before anything is enqueued."""
    lib = pf.load_library()
    n = 2048
    plan = pf.Plan(n, uniform_layout(n, 256), halo=128)
    assert plan.workspace_bytes > STATIC_BYTES
    st = lib.pfsm_solve_static(plan._h, ctypes.c_void_p(8), n, ctypes.c_void_p(8), n, ctypes.c_void_p(8),
                               ctypes.c_void_p(8), n, ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert st == 5  # PFSM_WORKSPACE_TOO_SMALL
