"""GPU parity of the mixed-precision path (BF16 matrix-core products with FP32
accumulation, FP64 submatrix eigensolver, first-order or FP64 Cholesky-QR
orthonormalisation, FP64 refinement against A) against the FP64 CPU oracle:
eigenvalues within 1e-8 (normwise relative) after refinement; eigenvectors
within a Davis-Kahan bound of the oracle's, per group of close eigenvalues.

Eigenvector tolerance.  The mixed vectors and the oracle's follow the same
iteration; they differ by the effect of the reduced-precision products, which
act like a perturbation E of the rotated operator of size about
2^-16 ||A|| (hi/lo split BF16 products keep about 16 significant bits).  For a
group g of eigenvalues separated by gap_g from the rest of the spectrum the
Davis-Kahan sin-theta theorem bounds the angle between the two spans by
||E|| / gap_g, so the test checks sin_g * gap_g / ||A||_2 <= 2^-16 (measured:
at most 0.07 * 2^-16 at N = 256 ... 8192; the values are printed)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.pfsm_ref import clusters, eig_error, orthogonality, pfsm_ref, residual_norm  # noqa: E402
from oracle.refine_ref import refine_ref  # noqa: E402
from pfsm_workloads import CONFIGS, householder_q, prescribed_problem, uniform_layout  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL_MIXED = 1e-8
U_SPLIT = 2.0 ** -16
C_DK = 1.0


def vector_parity(A, lam_ref, V_ref, Vo):
    """Largest sin of the angle between the mixed and oracle spans over groups of
    eigenvalues closer than 1e-10 and 1e-6 times max|lambda|, and the largest
    Davis-Kahan product sin_g * gap_g / ||A||_2 over those groups."""
    scale = np.max(np.abs(lam_ref))
    a2 = np.max(np.abs(lam_ref))  # ||A||_2 (A symmetric, lam_ref its eigenvalue estimates)
    out = {}
    for tol in (1e-10, 1e-6):
        worst_sin, worst_dk = 0.0, 0.0
        for g in clusters(lam_ref, tol * scale):
            lo, hi = g[0], g[-1]
            gap = min(lam_ref[lo] - lam_ref[lo - 1] if lo > 0 else np.inf,
                      lam_ref[hi + 1] - lam_ref[hi] if hi + 1 < len(lam_ref) else np.inf)
            Q1, Q2 = Vo[:, g], V_ref[:, g]
            sn = float(np.linalg.norm(Q1 - Q2 @ (Q2.T @ Q1), 2))
            worst_sin = max(worst_sin, sn)
            worst_dk = max(worst_dk, sn * gap / a2)
        out[tol] = (worst_sin, worst_dk)
    return out


@pytest.fixture(scope="module")
def pf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_1502_07806_amd as pf
    pf.load_library()
    return pf


def _run(pf, A, V, offs, halo, **kw):
    dev = torch.device("cuda:0")
    plan = pf.Plan(A.shape[0], offs, halo=halo, precision="mixed_bf16", **kw)
    lam, Vo = plan.solve(torch.from_numpy(A).to(dev), torch.from_numpy(V).to(dev), check=False)
    torch.cuda.synchronize()
    return plan, int(plan.info.item()), lam.cpu().numpy(), Vo.cpu().numpy()


@pytest.mark.parametrize("n,offs,halo,clusters_,q", [
    (256, uniform_layout(256, 64), 32, False, 2),
    (256, uniform_layout(256, 64), 32, False, 1),
    (300, [0, 50, 130, 220, 300], 20, False, 2),     # uneven slices, ragged 256-tiles
    (300, [0, 50, 130, 220, 300], 20, True, 2),      # overlap 0.12 from the identity: FP64 Cholesky-QR
    (1000, uniform_layout(1000, 100), 50, True, 2),
    (2048, uniform_layout(2048, 256), 128, True, 2),  # the N=8192 recipe at N=2048
])
def test_mixed_parity(pf, n, offs, halo, clusters_, q):
    A, V, lam_ex, _ = prescribed_problem(n, n // 4, 5e-3, 3000 + n, clusters=clusters_)
    A, V = A.numpy(), V.numpy()
    lam_ref, V_ref, info_ref = pfsm_ref(A, V, offs, halo, 3, q)
    plan, info, lam, Vo = _run(pf, A, V, offs, halo, fs_power=q)
    assert info == info_ref == 0
    assert eig_error(lam, lam_ref) <= TOL_MIXED
    assert abs(residual_norm(A, lam, Vo) - residual_norm(A, lam_ref, V_ref)) <= 1e-6
    assert orthogonality(Vo) <= 1e-3
    # the refinement is the FP64 oracle's refinement applied to comparable vectors:
    # refining the oracle's own PFSM vectors changes nothing beyond 1e-8 either
    lam_rr, _ = refine_ref(A, V_ref)
    assert eig_error(lam_rr, lam_ref) <= TOL_MIXED
    vp = vector_parity(A, lam_ref, V_ref, Vo)
    print("n=%d clusters=%s q=%d vector parity (group tol: max sin, max sin*gap/||A||): %s" % (n, clusters_, q, vp))
    for tol, (sn, dk) in vp.items():
        assert dk <= C_DK * U_SPLIT, (tol, sn, dk)


@pytest.mark.parametrize("n,offs,halo", [
    (1000, uniform_layout(1000, 100), 50),
    (300, [0, 50, 130, 220, 300], 20),
])
def test_mixed_fs_split_and_plain(pf, n, offs, halo):
    """The folded-spectrum products on plain BF16 operands (default) and on
    split operands (PFSM_FLAG_FS_SPLIT): both within the mixed bar of the
    oracle after the FP64 refinement, and close to each other."""
    # (with clusters and these narrow submatrices the N = 300 overlap is 0.12 from
    # the identity: the FP64 Cholesky-QR replaces the first-order step)
    A, V, _, _ = prescribed_problem(n, n // 4, 5e-3, 3000 + n, clusters=True)
    A, V = A.numpy(), V.numpy()
    lam_ref, V_ref, _ = pfsm_ref(A, V, offs, halo, 3, 2)
    _, info_p, lam_p, V_p = _run(pf, A, V, offs, halo)
    _, info_s, lam_s, V_s = _run(pf, A, V, offs, halo, fs_split=True)
    assert info_p == info_s == 0
    assert eig_error(lam_p, lam_ref) <= TOL_MIXED and eig_error(lam_s, lam_ref) <= TOL_MIXED
    assert eig_error(lam_p, lam_s) <= 1e-9
    assert abs(residual_norm(A, lam_p, V_p) - residual_norm(A, lam_s, V_s)) <= 1e-6


def test_mixed_unrefined_result(pf):
    A, V, _, _ = prescribed_problem(512, 128, 5e-3, 3512, clusters=True)
    A, V = A.numpy(), V.numpy()
    offs = uniform_layout(512, 128)
    lam_ref, _, _ = pfsm_ref(A, V, offs, 64, 3, 2)
    plan, info, lam, Vo = _run(pf, A, V, offs, 64, refine=False)
    assert info == 0
    err = eig_error(lam, lam_ref)
    assert 1e-9 < err <= 1e-4  # split-BF16 products alone: ~1e-5 (reported as the FP32 result)


def test_mixed_full_size(pf):
    """N = 8192 workload in the benchmark's launch configuration against the
    stored oracle eigenvalues; properties at full size."""
    gp = os.path.join(ROOT, "tests", "golden", "c3_n8192_oracle_lambda.txt")
    if not os.path.exists(gp):
        pytest.skip("oracle eigenvalues for N=8192 not generated (tests/golden/make_golden.py)")
    golden = np.loadtxt(gp)
    cfg = CONFIGS["c3_n8192"]
    dev = torch.device("cuda:0")
    A, V, lam_ex, _ = prescribed_problem(cfg.n, cfg.n_occ, cfg.kappa, cfg.seed_base, cfg.clusters, device=dev)
    plan = pf.Plan(cfg.n, uniform_layout(cfg.n, cfg.slice_size), halo=cfg.halo, iterations=cfg.iterations,
                   precision="mixed_bf16")
    lam, Vo = plan.solve(A, V)
    lam_np = lam.cpu().numpy()
    assert eig_error(lam_np, golden) <= TOL_MIXED
    # eigenvectors of 8 well separated eigenvalues (column by column, signs
    # included) and of one 3-fold cluster (as a subspace) against the oracle's
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "c3_n8192_oracle_vec_cols.txt"))
    Vref = np.load(os.path.join(ROOT, "tests", "golden", "c3_n8192_oracle_vectors.npy")).T
    cols = rows[:, 0].astype(np.int64)
    Vg = Vo[:, torch.from_numpy(cols).to(dev)].cpu().numpy()
    a2 = np.max(np.abs(golden))
    for grp in np.unique(rows[:, 1]):
        sel = np.flatnonzero(rows[:, 1] == grp)
        for j in (sel if grp < 0 else [sel]):
            j = np.atleast_1d(j)
            gap = rows[j[0], 2]
            if grp < 0:  # sign fixed: |v - v_ref| = 2 sin(theta / 2) <= sqrt(2) sin(theta)
                err = float(np.linalg.norm(Vg[:, j[0]] - Vref[:, j[0]])) / np.sqrt(2.0)
            else:
                Q1, Q2 = Vg[:, j], Vref[:, j]
                err = float(np.linalg.norm(Q1 - Q2 @ (Q2.T @ Q1), 2))
            print("n=8192 columns %s gap %.2e: sin %.2e, sin*gap/||A|| %.2e (bound %.2e)" %
                  (cols[j].tolist(), gap, err, err * gap / a2, C_DK * U_SPLIT))
            assert err * gap / a2 <= C_DK * U_SPLIT
    r, o = plan.diagnostics(A, lam, Vo)
    assert r <= 1e-3 and o <= 1e-2
    cols = torch.tensor([0, 1, 2, 31, 2047, 2048, 4096, 8191], device=dev)
    Vs = Vo[:, cols]
    nrm = torch.linalg.vector_norm(Vs, dim=0).cpu().numpy()
    assert np.max(np.abs(nrm - 1.0)) <= 1e-12
    # returned eigenvalues are the Rayleigh quotients of the returned vectors, up
    # to the error of the refinement product A V_new (int8 digit product with s
    # digits: about (s + 1) 2^-7s sqrt(n) 2^e 2^f per entry, e and f the
    # exponents of the row and column maxima, and about the same on a Rayleigh
    # quotient; a factor 8 over that estimate is allowed)
    s_dig = int(pf.load_library().pfsm_refine_digit_count())
    rq_tol = 8 * (s_dig + 1) * 2.0 ** (-7 * s_dig) * np.sqrt(cfg.n) * 2.0 ** np.frexp(
        torch.max(torch.abs(A)).item())[1]
    vmax = torch.max(torch.abs(Vs), dim=0).values.cpu().numpy()
    rq = torch.sum(Vs * (A @ Vs), dim=0).cpu().numpy()
    diff = np.abs(rq - lam_np[cols.cpu().numpy()])
    print("n=8192 Rayleigh quotients vs eigenvalues: max %.2e (allowed %.2e per unit 2^f)" % (diff.max(), rq_tol))
    assert np.all(diff <= rq_tol * 2.0 ** np.frexp(vmax)[1])
    # the largest groups of close estimates (refined together by a Rayleigh-Ritz
    # solve, several blocks of columns wide): Ritz vectors orthonormal to FP64
    # rounding, eigenvalues equal to their Rayleigh quotients
    thr = 1e-4 * np.abs(lam_np).max()
    starts = np.flatnonzero(np.r_[True, np.diff(lam_np) > thr])
    sizes = np.diff(np.r_[starts, cfg.n])
    big = np.argsort(-sizes, kind="stable")[:3]
    assert sizes[big[0]] >= 5
    for b in big:
        cl = torch.arange(int(starts[b]), int(starts[b] + sizes[b]), device=dev)
        Vc = Vo[:, cl]
        assert torch.max(torch.abs(Vc.T @ Vc - torch.eye(len(cl), dtype=Vc.dtype, device=dev))).item() <= 1e-12
        rq = torch.sum(Vc * (A @ Vc), dim=0).cpu().numpy()
        vmax = torch.max(torch.abs(Vc), dim=0).values.cpu().numpy()
        assert np.all(np.abs(rq - lam_np[cl.cpu().numpy()]) <= rq_tol * 2.0 ** np.frexp(vmax)[1])


def test_mixed_failure_modes(pf):
    A, V, _, _ = prescribed_problem(256, 64, 5e-3, 3256)
    A, V = A.numpy(), V.numpy()
    offs = uniform_layout(256, 64)
    A2 = A.copy()
    A2[3, 7] = np.nan
    assert _run(pf, A2, V, offs, 32)[1] == -1
    V2 = V.copy()
    V2[:, 5] = V2[:, 4]
    # V_prev not orthonormal: Cholesky breakdown or a collapsed output vector
    info = _run(pf, A, V2, offs, 32)[1]
    assert info == -4 or info > 0
    R = householder_q(256, 4242).numpy()
    plan, info, lam, Vo = _run(pf, A, R, offs, 32)
    assert info != 0 or eig_error(lam, np.linalg.eigvalsh(A)) > 1e-3


def test_mixed_deterministic(pf):
    A, V, _, _ = prescribed_problem(768, 192, 5e-3, 3768, clusters=True)
    dev = torch.device("cuda:0")
    plan = pf.Plan(768, uniform_layout(768, 128), halo=64, precision="mixed_bf16")
    A, V = A.to(dev), V.to(dev)
    l1, V1 = plan.solve(A, V)
    l1, V1 = l1.clone(), V1.clone()
    l2, V2 = plan.solve(A, V)
    assert torch.equal(l1, l2) and torch.equal(V1, V2)


def test_mixed_eigh_floor(pf):
    """The mixed path's submatrix eigensolver leaves off-diagonal entries below
    2^-24 of the Gershgorin bound unrotated (its projected matrix carries
    split-BF16 rounding, its start vectors are stored in FP32), where the FP64
    path rotates them down to its rounding floor; the eigenvalues still meet
    the mixed bar against the oracle."""
    n, offs, halo = 512, uniform_layout(512, 128), 64
    g = np.random.default_rng(91)
    E = g.standard_normal((n, n)) * 1e-10
    A = np.diag(np.sort(g.uniform(-1.0, 1.0, n))) + (E + E.T)
    V = np.eye(n)
    lam_ref, _, info_ref = pfsm_ref(A, V, offs, halo, 3, 2)
    plan_m, info_m, lam_m, _ = _run(pf, A, V, offs, halo)
    dev = torch.device("cuda:0")
    plan_d = pf.Plan(n, offs, halo=halo, precision="fp64")
    plan_d.solve(torch.from_numpy(A).to(dev), torch.from_numpy(V).to(dev))
    torch.cuda.synchronize()
    assert info_ref == info_m == 0
    assert all(s == 1 for s in plan_m.debug_stats()["converged_sweep"])  # sweep 0 rotated nothing
    assert all(s >= 2 for s in plan_d.debug_stats()["converged_sweep"])
    assert eig_error(lam_m, lam_ref) <= 1e-8


def test_mixed_band_form_gate(pf):
    """Folded-spectrum products (and the orthonormalisation correction) in the
    band form: taken for a basis close to the eigenvectors (every product),
    refused by the device gate for one farther from them (the dropped far terms
    would not be negligible), and within the mixed bar of the oracle either way."""
    n, offs, halo = 1024, uniform_layout(1024, 128), 64
    # kappa = 0.03: the start vectors have no rows outside their submatrices, so
    # the first product takes the band form; the far rows it produces, times the
    # off-diagonal row sums of At, exceed the gate's bound, and the rest run in
    # full
    for kappa, expect_band in ((5e-3, True), (0.03, False)):
        A, V, _, _ = prescribed_problem(n, n // 4, kappa, 3700, clusters=True)
        A, V = A.numpy(), V.numpy()
        lam_ref, _, info_ref = pfsm_ref(A, V, offs, halo, 3, 2)
        plan, info, lam, Vo = _run(pf, A, V, offs, halo)
        st = plan.debug_stats()
        nb = st["fs_band_products"]
        assert info == info_ref == 0
        assert (nb == 6) if expect_band else (1 <= nb < 6), (kappa, nb)
        if expect_band:  # the orthonormalisation correction's band form too
            assert st["correction_band"] == 1
        assert eig_error(lam, lam_ref) <= TOL_MIXED, kappa
        assert orthogonality(Vo) <= 1e-3
    # the split folded-spectrum products have no band form
    plan, info, _, _ = _run(pf, A, V, offs, halo, fs_split=True)
    st = plan.debug_stats()
    assert info == 0 and st["fs_band_products"] == 0 and st["correction_band"] == 0
