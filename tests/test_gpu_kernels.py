"""Kernel-level parity (through libpfsm_testhooks.so): the FP64 MFMA GEMM in
all transpose combinations and epilogues against NumPy FP64 products, and
the split-BF16 GEMM against an FP64 product of the same split operands, on
ragged shapes that are not tile multiples."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from hooks_util import lib, split_hi_lo  # noqa: E402

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    lib()
    return torch.device("cuda:0")


def _cm(x, dev):
    """column-major device copy of a 2-D numpy array"""
    return torch.from_numpy(np.asarray(x)).to(dev).t().contiguous().t()


def _np(t):
    return t.cpu().numpy()


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(129, 257, 70), (300, 1, 33), (1, 5, 400), (256, 256, 256)])
def test_gemm_f64_store(dev, ta, tb, M, N, K):
    g = np.random.default_rng(M * 7 + N + K)
    A = g.standard_normal((K, M) if ta else (M, K))
    B = g.standard_normal((N, K) if tb else (K, N))
    C0 = g.standard_normal((M, N))
    dA, dB, dC = _cm(A, dev), _cm(B, dev), _cm(C0, dev)
    rc = lib().pfsm_test_gemm_f64(ta, tb, 0, M, N, K, _p(dA), dA.stride(1), _p(dB), dB.stride(1), _p(dC), dC.stride(1),
                                  -0.5, 2.0, None, None, 0, None, 0, _stream())
    assert rc == 0
    ref = -0.5 * ((A.T if ta else A) @ (B.T if tb else B)) + 2.0 * C0
    bound = 2 * K * U64 * (np.abs(A).max() * np.abs(B).max() * K + np.abs(C0).max())
    assert np.max(np.abs(_np(dC) - ref)) <= bound


def test_gemm_f64_epilogues(dev):
    n = 300
    g = np.random.default_rng(5)
    At = g.standard_normal((n, n))
    At = 0.5 * (At + At.T)
    X = g.standard_normal((n, n))
    D = g.standard_normal((n, n))
    eps = g.standard_normal(n)
    dA, dX, dD, de = _cm(At, dev), _cm(X, dev), _cm(D, dev), torch.from_numpy(eps).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev).t()
    L = lib()
    assert L.pfsm_test_gemm_f64(0, 0, 1, n, n, n, _p(dA), n, _p(dX), n, _p(C), n, 1.0, 0.0, _p(de), None, 0, None, 0,
                                _stream()) == 0
    tol = 4 * n * U64 * np.abs(At).max() * np.abs(X).max() * n
    assert np.max(np.abs(_np(C) - (At @ X - X * eps))) <= tol
    assert L.pfsm_test_gemm_f64(0, 0, 2, n, n, n, _p(dA), n, _p(dX), n, _p(C), n, 0.3, 0.0, _p(de), _p(dD), n, None,
                                0, _stream()) == 0
    assert np.max(np.abs(_np(C) - (D - 0.3 * (At @ X - X * eps)))) <= tol
    tiles_m = (n + 127) // 128
    part = torch.empty(tiles_m * n, dtype=torch.float64, device=dev)
    assert L.pfsm_test_gemm_f64(0, 0, 3, n, n, n, _p(dA), n, _p(dX), n, None, n, 1.0, 0.0, None, _p(dX), n,
                                _p(part), 0, _stream()) == 0
    rq = _np(part).reshape(tiles_m, n).sum(0)
    assert np.max(np.abs(rq - np.sum(X * (At @ X), 0))) <= tol * 10
    # lower tiles only: entries on and below the diagonal are right, the rest untouched
    C2 = torch.zeros((n, n), dtype=torch.float64, device=dev).t()
    assert L.pfsm_test_gemm_f64(1, 0, 0, n, n, n, _p(dX), n, _p(dX), n, _p(C2), n, 1.0, 0.0, None, None, 0, None, 1,
                                _stream()) == 0
    S = X.T @ X
    low = np.tril_indices(n)
    assert np.max(np.abs(_np(C2)[low] - S[low])) <= tol


def _pack(x, by_rows, dev, flags_extra=0):
    L = lib()
    m, n = x.shape
    R, K = (m, n) if by_rows else (n, m)
    ldp = L.pfsm_test_x3_row_stride(K)
    P = torch.empty(R * ldp, dtype=torch.int16, device=dev)
    dx = _cm(x, dev)
    assert L.pfsm_test_pack_x3(_p(dx), 1, m, n, dx.stride(1), (1 if by_rows else 0) | flags_extra, _p(P), ldp,
                               _stream()) == 0
    return P, ldp


def test_pack_roundtrip(dev):
    g = np.random.default_rng(9)
    x = g.standard_normal((70, 45)) * np.exp(g.standard_normal((70, 45)))
    P, ldp = _pack(x, False, dev)
    raw = P.cpu().numpy().view(np.uint16).reshape(45, ldp).astype(np.uint32) << 16
    vals = raw.view(np.float32).astype(np.float64)
    K = 70
    hi = np.concatenate([vals[:, 64 * c:64 * c + 32] for c in range((K + 31) // 32)], axis=1)[:, :K]
    lo = np.concatenate([vals[:, 64 * c + 32:64 * c + 64] for c in range((K + 31) // 32)], axis=1)[:, :K]
    rec = (hi + lo).T
    assert np.max(np.abs(rec - x) / np.abs(x)) <= 2.0 ** -16
    h_ref, l_ref = split_hi_lo(x)
    assert np.array_equal(hi.T, h_ref) and np.array_equal(lo.T, l_ref)


def _unpack(P, R, K, ldp):
    raw = P.cpu().numpy().view(np.uint16).reshape(R, ldp).astype(np.uint32) << 16
    vals = raw.view(np.float32).astype(np.float64)
    nc = (K + 31) // 32
    hi = np.concatenate([vals[:, 64 * c:64 * c + 32] for c in range(nc)], axis=1)
    lo = np.concatenate([vals[:, 64 * c + 32:64 * c + 64] for c in range(nc)], axis=1)
    return hi, lo


@pytest.mark.parametrize("src_double", [0, 1])
@pytest.mark.parametrize("by_rows", [False, True])
@pytest.mark.parametrize("m,n,ld,flags", [(300, 300, 300, 2 | 4 | 16), (300, 300, 301, 2 | 8), (77, 130, 77, 0),
                                          (257, 64, 259, 4)])
def test_pack_flags_layouts(dev, src_double, by_rows, m, n, ld, flags):
    """Both packing kernels (with and without transpose), FP32 and FP64
    sources, aligned and unaligned leading dimensions, and the triangle /
    identity / half-diagonal flags against the same transformation in numpy;
    chunks past K hold zeros."""
    L = lib()
    g = np.random.default_rng(m + n + ld + flags)
    x = g.standard_normal((m, n)) * np.exp(g.standard_normal((m, n)))
    dt = torch.float64 if src_double else torch.float32
    buf = torch.from_numpy(np.zeros((n, ld))).to(dt)
    buf[:, :m] = torch.from_numpy(x.T).to(dt)
    dx = buf.to(dev)  # column-major m x n with leading dimension ld
    xs = buf[:, :m].numpy().T.astype(np.float64)  # the values as stored
    ref = xs.copy()
    rr, cc = np.indices((m, n))
    if flags & 4:
        ref[rr < cc] = 0.0
    if flags & 8:
        ref[rr > cc] = 0.0
    d = np.arange(min(m, n))
    if flags & 2:
        ref[d, d] -= 1.0
    if flags & 16:
        ref[d, d] *= 0.5
    R, K = (m, n) if by_rows else (n, m)
    ldp = L.pfsm_test_x3_row_stride(K)
    P = torch.full((R * ldp,), -1, dtype=torch.int16, device=dev)
    assert L.pfsm_test_pack_x3(_p(dx), src_double, m, n, ld, (1 if by_rows else 0) | flags, _p(P), ldp,
                               _stream()) == 0
    hi, lo = _unpack(P, R, K, ldp)
    want = ref if by_rows else ref.T  # packed row r, k along the row
    h_ref, l_ref = split_hi_lo(want)
    assert np.array_equal(hi[:, :K], h_ref) and np.array_equal(lo[:, :K], l_ref)
    assert np.all(hi[:, K:] == 0) and np.all(lo[:, K:] == 0)


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("M,N,K", [(300, 270, 100), (256, 512, 64), (33, 600, 257)])
def test_gemm_x3(dev, cfg, M, N, K):
    g = np.random.default_rng(M + N + K + cfg)
    A = g.standard_normal((M, K))
    B = g.standard_normal((K, N))
    Ap, lda = _pack(A, True, dev)     # rows of A
    Bp, ldb = _pack(B, False, dev)    # columns of B
    C = torch.empty((N, M), dtype=torch.float64, device=dev).t()  # column-major M x N
    assert lib().pfsm_test_gemm_x3(0, cfg, 0, M, N, K, _p(Ap), lda, _p(Bp), ldb, _p(C), M, 1, 1.0, 0.0, None, 0, None,
                                   0, 0, None, None, _stream()) == 0
    ah, al = split_hi_lo(A)
    bh, bl = split_hi_lo(B)
    ref3 = ah @ bh + ah @ bl + al @ bh
    # FP32 accumulation of K products of magnitude |a||b|
    tol = 4 * K * 2.0 ** -24 * np.abs(A).max() * np.abs(B).max()
    assert np.max(np.abs(_np(C) - ref3)) <= tol
    assert np.max(np.abs(_np(C) - A @ B)) <= 2.0 ** -14 * np.sqrt(K) * np.abs(A).max() * np.abs(B).max() + tol


def _pack_plain(x, dev):
    """Plain layout of the columns of x (K x R): bf16(x) along k, zero-filled to 32."""
    L = lib()
    K, R = x.shape
    ldq = L.pfsm_test_x3_plain_stride(K)
    P = torch.full((R * ldq,), -1, dtype=torch.int16, device=dev)
    dx = _cm(x, dev)
    assert L.pfsm_test_pack_x3(_p(dx), 1, K, R, dx.stride(1), 32, _p(P), ldq, _stream()) == 0
    return P, ldq


def test_pack_plain_layout(dev):
    g = np.random.default_rng(5)
    K, R = 100, 37
    x = g.standard_normal((K, R))
    P, ldq = _pack_plain(x, dev)
    assert ldq == 128
    torch.cuda.synchronize()
    got = P.cpu().numpy().view(np.uint16).reshape(R, ldq)
    h_ref, _ = split_hi_lo(x.T)
    hi = (got[:, :K].astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.array_equal(hi, h_ref)
    assert np.all(got[:, K:] == 0)
    # the transposing pack in the plain layout: rows of x (K rows of length R)
    ldr = lib().pfsm_test_x3_plain_stride(R)
    Q = torch.full((K * ldr,), -1, dtype=torch.int16, device=dev)
    dx = _cm(x, dev)
    assert lib().pfsm_test_pack_x3(_p(dx), 1, K, R, K, 1 | 32, _p(Q), ldr, _stream()) == 0
    torch.cuda.synchronize()
    got = Q.cpu().numpy().view(np.uint16).reshape(K, ldr)
    h_ref, _ = split_hi_lo(x)
    assert np.array_equal((got[:, :R].astype(np.uint32) << 16).view(np.float32).astype(np.float64), h_ref)
    assert np.all(got[:, R:] == 0)


@pytest.mark.parametrize("epi", [1, 2])  # X3_SHIFT, X3_FSUPD
@pytest.mark.parametrize("M,N,K", [(300, 270, 100), (512, 512, 512), (33, 600, 257)])
def test_gemm_x3_plain_product(dev, epi, M, N, K):
    """One BF16 product from plain operands (the folded-spectrum products of the
    mixed path): equal to bf16(A) bf16(B) within FP32 accumulation, with the
    SHIFT / FSUPD epilogue; refused for other epilogues."""
    L = lib()
    g = np.random.default_rng(M + N + K + epi)
    A = g.standard_normal((M, K))
    B = g.standard_normal((K, N))
    Ap, lda = _pack_plain(A.T, dev)   # rows of A
    Bp, ldb = _pack_plain(B, dev)     # columns of B
    B32 = torch.from_numpy(g.standard_normal((N, M))).float().to(dev).t()
    D32 = torch.from_numpy(g.standard_normal((N, M))).float().to(dev).t()
    eps = torch.from_numpy(g.standard_normal(N)).to(dev)
    C = torch.empty((N, M), dtype=torch.float32, device=dev).t()
    alpha = 0.3
    assert L.pfsm_test_gemm_x3_fs(epi, 1, 0, M, N, K, _p(Ap), lda, _p(Bp), ldb, _p(C), M, _p(B32), M, _p(D32), M,
                                  _p(eps), alpha, _stream()) == 0
    torch.cuda.synchronize()
    ah, _ = split_hi_lo(A)
    bh, _ = split_hi_lo(B)
    prod = ah @ bh
    b32, d32, e = _np(B32).astype(np.float64), _np(D32).astype(np.float64), eps.cpu().numpy()
    ref = prod - b32 * e[None, :]
    if epi == 2:
        ref = d32 - alpha * ref
    tol = (4 * K * 2.0 ** -24 * np.abs(ah).max() * np.abs(bh).max() + 2.0 ** -23 * np.abs(ref).max()) * (1 + alpha)
    assert np.max(np.abs(_np(C).astype(np.float64) - ref)) <= tol
    assert L.pfsm_test_gemm_x3_fs(0, 1, 0, M, N, K, _p(Ap), lda, _p(Bp), ldb, _p(C), M, None, 0, None, 0, None,
                                  1.0, _stream()) != 0
    assert L.pfsm_test_gemm_x3_fs(epi, 1, 1, M, N, K, _p(Ap), lda, _p(Bp), ldb, _p(C), M, _p(B32), M, _p(D32), M,
                                  _p(eps), alpha, _stream()) != 0  # no lower-triangle tiles


@pytest.mark.parametrize("n", [600, 512])
def test_gemm_x3_plain_correction(dev, n):
    """The orthonormalisation correction X <- X - X Phi^T of the mixed path from
    plain operands packed by rows (transposing pack), k-prefix tiles: equal to
    D - bf16(X) bf16(Phi)^T within FP32 accumulation for a lower-triangular Phi."""
    L = lib()
    g = np.random.default_rng(n)
    X = g.standard_normal((n, n))
    Phi = np.tril(g.standard_normal((n, n))) * 1e-3
    ldq = L.pfsm_test_x3_plain_stride(n)
    dX, dPhi = _cm(X, dev), _cm(Phi, dev)
    Xp = torch.full((n * ldq,), -1, dtype=torch.int16, device=dev)
    Pp = torch.full((n * ldq,), -1, dtype=torch.int16, device=dev)
    assert L.pfsm_test_pack_x3(_p(dX), 1, n, n, n, 1 | 32, _p(Xp), ldq, _stream()) == 0    # rows of X
    assert L.pfsm_test_pack_x3(_p(dPhi), 1, n, n, n, 1 | 32, _p(Pp), ldq, _stream()) == 0  # rows of Phi
    torch.cuda.synchronize()
    rows = Xp.cpu().numpy().view(np.uint16).reshape(n, ldq)
    h_ref, _ = split_hi_lo(X)
    assert np.array_equal((rows[:, :n].astype(np.uint32) << 16).view(np.float32).astype(np.float64), h_ref)
    assert np.all(rows[:, n:] == 0)
    D = torch.from_numpy(g.standard_normal((n, n))).float().to(dev).t().contiguous().t()
    C = torch.empty((n, n), dtype=torch.float32, device=dev).t()
    assert L.pfsm_test_gemm_x3_fs(3, 1, 3, n, n, n, _p(Xp), ldq, _p(Pp), ldq, _p(C), n, None, 0, _p(D), n, None,
                                  -1.0, _stream()) == 0
    torch.cuda.synchronize()
    xh, _ = split_hi_lo(X)
    ph, _ = split_hi_lo(Phi)
    ref = _np(D).astype(np.float64) - xh @ ph.T
    tol = 4 * n * 2.0 ** -24 * np.abs(xh).max() * np.abs(ph).max() + 2.0 ** -23 * np.abs(ref).max()
    assert np.max(np.abs(_np(C).astype(np.float64) - ref)) <= tol


@pytest.mark.parametrize("c_double,beta", [(1, 0.5), (0, 0.0)])
def test_gemm_x3_lower_ksplit(dev, c_double, beta):
    """Lower-triangle product whose last wave is split along K (23 x 23 tiles =
    276 > 256 compute units): equal to the unsplit launch within FP32
    accumulation, and the split tail tiles (the last tile row) equal to the
    split-BF16 expansion; the upper tiles stay untouched."""
    L = lib()
    n = 5800
    assert L.pfsm_test_x3_split_bytes(4096) == 0
    nbytes = L.pfsm_test_x3_split_bytes(n)
    assert nbytes > 0
    ws = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    g = np.random.default_rng(77)
    X = g.standard_normal((n, n))
    Xp, ldx = _pack(X, False, dev)  # columns of X: C = X^T X
    dt = torch.float64 if c_double else torch.float32
    outs = []
    for use_ws in (False, True):
        C = torch.full((n, n), 1.0, dtype=dt, device=dev)  # symmetric fill: layout irrelevant
        assert L.pfsm_test_gemm_x3_ws(0, 5, 1, n, n, n, _p(Xp), ldx, _p(Xp), ldx, _p(C), n, c_double, 1.0, beta, None,
                                      0, None, 0, 0, None, None, _p(ws) if use_ws else None,
                                      nbytes if use_ws else 0, _stream()) == 0
        torch.cuda.synchronize()
        outs.append(_np(C).T.astype(np.float64))  # column-major element (i, j) at [i, j]
    ti = np.arange(n) // 256
    lower = ti[:, None] >= ti[None, :]
    tol = 4 * n * 2.0 ** -24 * np.abs(X).max() ** 2 + (0 if c_double else 2.0 ** -23 * n * 1.5)
    assert np.all(outs[1][~lower] == 1.0)
    assert np.max(np.abs(outs[1][lower] - outs[0][lower])) <= tol
    xh, xl = split_hi_lo(X)
    rows = np.arange(22 * 256, n)
    ref = xh[:, rows].T @ xh + xh[:, rows].T @ xl + xl[:, rows].T @ xh + beta
    assert np.max(np.abs(outs[1][rows] - ref)) <= tol


# ------------------------------------------------------------ Cholesky (overlap factor)
def _spd(n, seed):
    g = np.random.default_rng(seed)
    G = g.standard_normal((n, n))
    return np.eye(n) + G @ G.T / n


@pytest.mark.parametrize("n", [64, 200, 1100])
def test_cholesky_blocked_vs_oracle(dev, n):
    """Blocked FP64 factor (64-wide register blocks, 512-wide panels) against the
    oracle's column Cholesky, on sizes with a ragged last block and two panels."""
    from oracle.pfsm_ref import cholesky_lower
    S0 = _spd(n, n)
    S = _cm(S0, dev)
    T = torch.empty(((n + 63) // 64) * 4096, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    assert lib().pfsm_test_cholesky(_p(S), n, n, _p(T), _p(info), _stream()) == 0
    torch.cuda.synchronize()
    L_ref, info_ref = cholesky_lower(S0)
    assert int(info.item()) == info_ref == 0
    L = np.tril(_np(S))
    assert np.max(np.abs(L - L_ref)) <= 64 * n * U64 * np.abs(L_ref).max()
    # X <- X L^{-T} with the same factor and block inverses
    m = 150
    X0 = np.random.default_rng(n + 1).standard_normal((m, n))
    X = _cm(X0, dev)
    assert lib().pfsm_test_trsm(_p(S), n, _p(X), m, n, m, _p(T), _stream()) == 0
    torch.cuda.synchronize()
    ref = np.linalg.solve(L_ref, X0.T).T
    assert np.max(np.abs(_np(X) - ref)) <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("n,m", [(64, 64), (200, 200), (300, 150), (1100, 1100)])
def test_cholesky_qr_gated_vs_oracle(dev, n, m):
    """Fallback orthonormalisation of the mixed path: one launch per 64-wide block
    column factors [S; X] left-looking, giving L in place of S and X L^{-T} in
    place of X.  Against the oracle's column Cholesky and a solve with its
    factor, on ragged sizes; with the gate off nothing is written."""
    from oracle.pfsm_ref import cholesky_lower
    S0 = _spd(n, n)
    X0 = np.random.default_rng(n + 7).standard_normal((m, n))
    L_ref, info_ref = cholesky_lower(S0)
    assert info_ref == 0
    ref = np.linalg.solve(L_ref, X0.T).T
    nblk = (n + 63) // 64
    for g in (0, 1):
        S = _cm(S0, dev)
        X = _cm(X0, dev)
        T = torch.zeros(nblk * 4096, dtype=torch.float64, device=dev)
        Bc = torch.zeros(nblk * 4096, dtype=torch.float64, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        gate = torch.tensor([g], dtype=torch.int32, device=dev)
        assert lib().pfsm_test_cholesky_qr_gated(_p(S), n, _p(X), m, n, m, _p(T), _p(Bc), _p(info), _p(gate),
                                                 _stream()) == 0
        torch.cuda.synchronize()
        if g == 0:
            assert np.array_equal(_np(S), S0) and np.array_equal(_np(X), X0)
            continue
        assert int(info.item()) == 0
        L = np.tril(_np(S))
        assert np.max(np.abs(L - L_ref)) <= 64 * n * U64 * np.abs(L_ref).max()
        assert np.max(np.abs(_np(X) - ref)) <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("n,k", [(200, 0), (200, 130), (1100, 777)])
def test_cholesky_qr_gated_breakdown(dev, n, k):
    """The fallback reports a non-positive pivot at global column k as info = k + 1."""
    from oracle.pfsm_ref import cholesky_lower
    S0 = np.eye(n)
    S0[k, k] = -1.0
    S0[min(k + 5, n - 1), min(k + 5, n - 1)] = -2.0
    nblk = (n + 63) // 64
    S = _cm(S0, dev)
    X = _cm(np.eye(n), dev)
    T = torch.zeros(nblk * 4096, dtype=torch.float64, device=dev)
    Bc = torch.zeros(nblk * 4096, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    gate = torch.ones(1, dtype=torch.int32, device=dev)
    assert lib().pfsm_test_cholesky_qr_gated(_p(S), n, _p(X), n, n, n, _p(T), _p(Bc), _p(info), _p(gate),
                                             _stream()) == 0
    torch.cuda.synchronize()
    assert int(info.item()) == cholesky_lower(S0)[1] == k + 1


@pytest.mark.parametrize("n,k", [(200, 0), (200, 130), (1100, 777)])
def test_cholesky_breakdown_column(dev, n, k):
    """A non-positive pivot at global column k reports info = k + 1 (first one wins)."""
    from oracle.pfsm_ref import cholesky_lower
    S0 = np.eye(n)
    S0[k, k] = -1.0
    S0[min(k + 5, n - 1), min(k + 5, n - 1)] = -2.0
    S = _cm(S0, dev)
    T = torch.empty(((n + 63) // 64) * 4096, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    assert lib().pfsm_test_cholesky(_p(S), n, n, _p(T), _p(info), _stream()) == 0
    torch.cuda.synchronize()
    assert int(info.item()) == cholesky_lower(S0)[1] == k + 1


@pytest.mark.parametrize("n,eps", [(600, 1e-4), (300, 1e-3)])
def test_first_order_orthonormalisation(dev, n, eps):
    """The mixed path's X <- X L^{-T} for S = X^T X near the identity: the rows
    of Phi(S - I) packed straight from S (identity removed, lower triangle,
    half diagonal), then X - X Phi(S - I)^T with the ADD epilogue (alpha = -1)
    on KPREFIX tiles.  Equal to that expression in FP64 up to the split-BF16
    rounding of the product, and orthonormal up to O(eps^2)."""
    L = lib()
    g = np.random.default_rng(n)
    X = np.eye(n) + eps * g.standard_normal((n, n)) / np.sqrt(n) * 3
    S = X.T @ X
    E = S - np.eye(n)
    Phi = np.tril(E, -1) + 0.5 * np.diag(np.diag(E))
    Xp, ldx = _pack(X, True, dev)                   # rows of X
    Sp, lds = _pack(S, True, dev, 2 | 4 | 16)       # rows of Phi(S - I) = columns of Phi^T
    dX = _cm(X, dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev).t()
    assert L.pfsm_test_gemm_x3(3, 5, 3, n, n, n, _p(Xp), ldx, _p(Sp), lds, _p(C), n, 1, -1.0, 0.0, None, 0, _p(dX),
                               n, 1, None, None, _stream()) == 0
    torch.cuda.synchronize()
    out = _np(C)
    ref = X - X @ Phi.T
    prod = np.abs(X) @ np.abs(Phi).T
    assert np.max(np.abs(out - ref)) <= 2.0 ** -14 * prod.max() + 1e-15
    # the first-order correction leaves an O(eps^2) overlap error, and the
    # rounding of the product adds little to it
    e1 = np.abs(E).max()
    r_ref = np.abs(ref.T @ ref - np.eye(n)).max()
    assert r_ref <= 0.05 * e1
    assert np.abs(out.T @ out - np.eye(n)).max() <= r_ref + 2.0 ** -10 * e1


# ------------------------------------------------------------ int8 digit GEMM (FP64-accurate products)
def _oz_split_dev(X, s, dev):
    """GPU digits of the columns of X: (planes as numpy [s, ncols, ldp] int8, exponents, info)."""
    K, nc = X.shape
    ldp = int(lib().pfsm_test_oz_row_stride(K))
    P = torch.full((s * nc * ldp,), 7, dtype=torch.int8, device=dev)
    ex = torch.empty(nc, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    Xd = _cm(X, dev)
    assert lib().pfsm_test_oz_split(_p(Xd), K, K, nc, s, _p(P), _p(ex), _p(info), _stream()) == 0
    torch.cuda.synchronize()
    return P, P.cpu().numpy().reshape(s, nc, ldp), ex.cpu().numpy(), int(info.item()), ldp, ex


@pytest.mark.parametrize("K,nc", [
    (300, 70),   # columns held in registers, 16-byte loads, ragged tail
    (301, 9),    # odd leading dimension: 8-byte loads
    (8200, 7),   # longer than the register-held column: two reads
])
def test_oz_split_digits(dev, K, nc):
    from hooks_util import oz_digits
    g = np.random.default_rng(21 + K)
    s = 6
    X = g.standard_normal((K, nc)) * np.exp(3 * g.standard_normal((1, nc))) * np.exp(g.standard_normal((K, nc)))
    X[:, 5] = 0.0
    X[:, 6] = 0.5  # exact power of two at the maximum
    _, planes, ex, info, ldp, _ = _oz_split_dev(X, s, dev)
    D, e = oz_digits(X, s)
    assert info == 0
    assert np.array_equal(ex, e)
    for p in range(s):
        assert np.array_equal(planes[p, :, :K].astype(np.float64), D[p].T)
        assert np.all(planes[p, :, K:] == 0)
        assert np.abs(planes[p]).max() <= 64
    rec = sum(np.ldexp(D[p], (e - 6 - 7 * p)[None, :]) for p in range(s))
    assert np.all(np.abs(rec - X) <= np.ldexp(1.0, e - 7 * s)[None, :])


def test_oz_split_nonfinite(dev):
    X = np.ones((130, 3))
    X[7, 1] = np.nan
    _, planes, ex, info, _, _ = _oz_split_dev(X, 3, dev)
    assert info == -1
    assert np.all(planes[:, 1, :] == 0)
    assert np.all(planes[0, 0, :130] == 32) and np.all(planes[1:, 0, :] == 0)  # 1 = 32 * 2^(1 - 6)


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("M,N,K,s", [(300, 270, 1000, 6), (256, 512, 128, 4), (33, 600, 257, 5), (520, 130, 700, 5)])
def test_gemm_oz(dev, cfg, M, N, K, s):
    """C = A B from digits: equal (to FP64 rounding of the group sums) to the same
    truncated digit expansion evaluated in FP64 from digits made on the host, and
    within the truncation bound of the FP64 product."""
    from hooks_util import oz_digits
    g = np.random.default_rng(M + N + K + s)
    A = g.standard_normal((M, K)) * np.exp(g.standard_normal((M, 1)))
    B = g.standard_normal((K, N)) * np.exp(g.standard_normal((1, N)))
    Ap, _, ea_h, info_a, _, ea = _oz_split_dev(A.T, s, dev)   # rows of A
    Bp, _, eb_h, info_b, _, eb = _oz_split_dev(B, s, dev)     # columns of B
    assert info_a == info_b == 0
    C = torch.empty((N, M), dtype=torch.float64, device=dev).t()
    assert lib().pfsm_test_gemm_oz(M, N, K, s, _p(Ap), _p(ea), _p(Bp), _p(eb), _p(C), M, cfg, _stream()) == 0
    torch.cuda.synchronize()
    Da, e_a = oz_digits(A.T, s)
    Db, e_b = oz_digits(B, s)
    ref = np.zeros((M, N))
    for grp in range(s + 1, 1, -1):
        G = sum(Da[p - 1].T @ Db[grp - p - 1] for p in range(max(1, grp - s), min(s, grp - 1) + 1))
        ref += np.ldexp(G, -12 - 7 * (grp - 2))  # integer-valued G: exact in FP64
    ref = ref * np.ldexp(1.0, e_a)[:, None] * np.ldexp(1.0, e_b)[None, :]
    out = _np(C)
    scale = np.ldexp(1.0, e_a)[:, None] * np.ldexp(1.0, e_b)[None, :]
    assert np.max(np.abs(out - ref) / scale) <= 8 * U64 * K
    assert np.max(np.abs(out - A @ B) / scale) <= 2 * s * K * 2.0 ** (-7 * s)


@pytest.mark.parametrize("M,N,K,s", [(300, 270, 1000, 5), (640, 384, 2048, 5), (200, 333, 512, 4), (129, 64, 128, 3)])
def test_gemm_oz_multi_matches_fused(dev, M, N, K, s):
    """The all-groups kernel (configuration 5) performs the fused kernel's FP64
    additions in the same order: the two products agree bit for bit."""
    g = np.random.default_rng(7 * M + N + K + s)
    A = g.standard_normal((M, K)) * np.exp(g.standard_normal((M, 1)))
    B = g.standard_normal((K, N)) * np.exp(g.standard_normal((1, N)))
    Ap, _, _, info_a, _, ea = _oz_split_dev(A.T, s, dev)
    Bp, _, _, info_b, _, eb = _oz_split_dev(B, s, dev)
    assert info_a == info_b == 0
    out = []
    for cfg in (4, 5, 6):
        C = torch.full((N, M), np.nan, dtype=torch.float64, device=dev).t()
        assert lib().pfsm_test_gemm_oz(M, N, K, s, _p(Ap), _p(ea), _p(Bp), _p(eb), _p(C), M, cfg, _stream()) == 0
        torch.cuda.synchronize()
        out.append(_np(C))
    assert np.all(np.isfinite(out[1]))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


@pytest.mark.parametrize("n", [512, 700])
@pytest.mark.parametrize("by_rows,flags", [(False, 32), (False, 2), (True, 32)])
def test_pack_band_and_gated_far(dev, n, by_rows, flags):
    """The two-part packs of the band forms: the band part writes exactly the
    rows of the packed operand inside each 256-row tile's K range, bitwise as
    the full pack does, and nothing else; the far part writes nothing while
    the gate lets the band form run, and completes the full pack when it does
    not.  Plain column packs (the folded-spectrum operands), split column packs
    (X - I of the back-rotation, band part only) and plain row packs (the
    correction's operand); n = 700 has zero padding past K."""
    L = lib()
    g = np.random.default_rng(n + 10 * flags + by_rows)
    x = g.standard_normal((n, n)).astype(np.float32)
    plain = bool(flags & 32)
    ld = L.pfsm_test_x3_plain_stride(n) if plain else L.pfsm_test_x3_row_stride(n)
    kpad = (n + 31) // 32 * 32
    tiles = (n + 255) // 256
    kr = []
    for _ in range(tiles):  # a random band per 256-row tile of the packed operand
        lo = int(g.integers(0, kpad // 32)) * 32
        hi = min(kpad, lo + 32 * int(g.integers(1, 9)))
        kr += [lo, hi]
    chunks = max((kr[2 * t + 1] - kr[2 * t]) // 32 for t in range(tiles))
    dkr = torch.tensor(kr, dtype=torch.int32, device=dev)
    dx = torch.from_numpy(x).to(dev).t().contiguous().t()  # column-major FP32
    fl = flags | (1 if by_rows else 0)
    full = torch.full((n * ld,), -1, dtype=torch.int16, device=dev)
    assert L.pfsm_test_pack_x3(_p(dx), 0, n, n, dx.stride(1), fl, _p(full), ld, _stream()) == 0
    part = torch.full((n * ld,), -1, dtype=torch.int16, device=dev)
    assert L.pfsm_test_pack_x3_part(_p(dx), 0, n, n, dx.stride(1), fl, _p(part), ld, _p(dkr), chunks, 0, None, None,
                                    _stream()) == 0
    torch.cuda.synchronize()
    F, Pp = full.view(n, ld).cpu().numpy(), part.view(n, ld).cpu().numpy()
    band = np.zeros((n, ld), dtype=bool)  # packed positions of the k inside each row's band
    for r in range(n):
        lo, hi = kr[2 * (r // 256)], kr[2 * (r // 256) + 1]
        k = np.arange(lo, hi)
        if plain:
            band[r, k] = True
        else:
            band[r, (k >> 5) * 64 + (k & 31)] = True
            band[r, (k >> 5) * 64 + (k & 31) + 32] = True
    assert np.array_equal(Pp[band], F[band])
    assert np.all(Pp[~band] == -1)
    if not plain:
        return  # the split column layout has no far part (the back-rotation's plain product covers those rows)
    open_gate = torch.tensor([0], dtype=torch.int32, device=dev)  # m = 0: c m <= limit
    closed_gate = torch.tensor([np.float32(2.0).view(np.int32)], dtype=torch.int32, device=dev)  # m = 2
    cl = torch.tensor([1.0, 1.0], dtype=torch.float64, device=dev)
    assert L.pfsm_test_pack_x3_part(_p(dx), 0, n, n, dx.stride(1), fl, _p(part), ld, _p(dkr), chunks, 1,
                                    _p(open_gate), _p(cl), _stream()) == 0
    torch.cuda.synchronize()
    assert np.array_equal(part.view(n, ld).cpu().numpy(), Pp)
    assert L.pfsm_test_pack_x3_part(_p(dx), 0, n, n, dx.stride(1), fl, _p(part), ld, _p(dkr), chunks, 1,
                                    _p(closed_gate), _p(cl), _stream()) == 0
    torch.cuda.synchronize()
    assert np.array_equal(part.view(n, ld).cpu().numpy(), F)
