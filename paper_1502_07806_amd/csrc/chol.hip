// Blocked FP64 Cholesky of the overlap matrix S = X^T X and the right-side
// triangular solve X <- X L^{-T} (the orthonormalisation step, computed as
// Cholesky-QR).  Block width 64: a single-workgroup kernel factors each
// 64x64 diagonal block in LDS and writes both L_kk and L_kk^{-T}; the panel
// and trailing updates are MFMA GEMMs.
#include "common.h"
#include "chol.h"

namespace pfsm {
namespace {

constexpr int NB = CHOL_NB;
constexpr int LS = NB + 1;

// Factor S[k0:k0+nb, k0:k0+nb] (lower triangle) in place; write T = L^{-T}
// (upper triangular, column-major nb x nb).  A non-positive or non-finite
// pivot records info = global column (1-based), first error wins.
__global__ __launch_bounds__(256) void potrf_diag(double* S, int64_t lds, int64_t k0, int nb, double* T, int* info) {
  __shared__ double L[NB][LS];
  __shared__ double Xi[NB][LS];
  const int tid = threadIdx.x;
  double* Sk = S + k0 + k0 * lds;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    int r = idx % NB, c = idx / NB;
    double v = 0.0;
    if (r < nb && c < nb && r >= c) v = Sk[r + c * lds];
    if (r >= nb && r == c) v = 1.0;  // ragged last block: identity padding
    L[r][c] = v;
    Xi[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (tid == 0) {
      double d = L[j][j];
      if (!(d > 0.0)) {
        if (j < nb) atomicCAS(info, 0, (int)(k0 + j + 1));
        d = __builtin_nan("");
      }
      L[j][j] = sqrt(d);
    }
    __syncthreads();
    const double djj = L[j][j];
    for (int i = j + 1 + tid; i < NB; i += 256) L[i][j] /= djj;
    __syncthreads();
    const int m = NB - j - 1;
    for (int idx = tid; idx < m * m; idx += 256) {
      int i = j + 1 + idx % m, c = j + 1 + idx / m;
      if (c <= i) L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  // Xi <- L^{-1} by right-looking forward substitution on the identity.
  for (int i = 0; i < NB; ++i) {
    const double lii = L[i][i];
    for (int c = tid; c <= i; c += 256) Xi[i][c] /= lii;
    __syncthreads();
    const int m = NB - i - 1;
    for (int idx = tid; idx < m * (i + 1); idx += 256) {
      int r = i + 1 + idx % m, c = idx / m;
      Xi[r][c] -= L[r][i] * Xi[i][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < NB * NB; idx += 256) {
    int r = idx % NB, c = idx / NB;
    if (r < nb && c < nb) {
      if (r >= c) Sk[r + c * lds] = L[r][c];
      T[r + c * NB] = Xi[c][r];  // T = (L^{-1})^T
    } else {
      T[r + c * NB] = (r == c) ? 1.0 : 0.0;
    }
  }
}

}  // namespace

hipError_t cholesky_factor(double* S, int64_t lds, int64_t n, double* Tbuf, int* info, hipStream_t s) {
  // S: n x n (lower triangle valid) -> L in place; Tbuf receives the inverse-transposed diagonal blocks.
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t k0 = b * NB;
    const int nb = (int)std::min<int64_t>(NB, n - k0);
    double* T = Tbuf + b * NB * NB;
    hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(256), 0, s, S, lds, k0, nb, T, info);
    const int64_t rest = n - k0 - nb;
    if (rest > 0) {
      GemmArgs g = {};
      // panel: L21 = S21 * T  (in place; one column tile per row tile)
      g.M = rest; g.N = nb; g.K = nb;
      g.A = S + (k0 + nb) + k0 * lds; g.lda = lds;
      g.B = T; g.ldb = NB;
      g.C = S + (k0 + nb) + k0 * lds; g.ldc = lds;
      g.alpha = 1.0; g.beta = 0.0;
      hipError_t e = gemm_f64(false, false, EPI_STORE, g, s);
      if (e != hipSuccess) return e;
      // trailing: S22 -= L21 L21^T (lower tiles)
      GemmArgs h = {};
      h.M = rest; h.N = rest; h.K = nb;
      h.A = S + (k0 + nb) + k0 * lds; h.lda = lds;
      h.B = S + (k0 + nb) + k0 * lds; h.ldb = lds;
      h.C = S + (k0 + nb) + (k0 + nb) * lds; h.ldc = lds;
      h.alpha = -1.0; h.beta = 1.0; h.lower_only = 1;
      e = gemm_f64(false, true, EPI_STORE, h, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t cholesky_qr(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m,
                       double* Tbuf, int* info, hipStream_t s) {
  // S: n x n overlap (lower triangle valid) -> L.  X: m x n, overwritten by X L^{-T}.
  const int64_t nblk = (n + NB - 1) / NB;
  hipError_t e0 = cholesky_factor(S, lds, n, Tbuf, info, s);
  if (e0 != hipSuccess) return e0;
  // X <- X L^{-T}: right-looking over column blocks.
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t k0 = b * NB;
    const int nb = (int)std::min<int64_t>(NB, n - k0);
    GemmArgs g = {};
    g.M = m; g.N = nb; g.K = nb;
    g.A = X + k0 * ldx; g.lda = ldx;
    g.B = Tbuf + b * NB * NB; g.ldb = NB;
    g.C = X + k0 * ldx; g.ldc = ldx;
    g.alpha = 1.0; g.beta = 0.0;
    hipError_t e = gemm_f64(false, false, EPI_STORE, g, s);
    if (e != hipSuccess) return e;
    const int64_t rest = n - k0 - nb;
    if (rest > 0) {
      GemmArgs h = {};
      h.M = m; h.N = rest; h.K = nb;
      h.A = X + k0 * ldx; h.lda = ldx;
      h.B = S + (k0 + nb) + k0 * lds; h.ldb = lds;   // op(B) = L[k0+nb:, k0:k0+nb]^T
      h.C = X + (k0 + nb) * ldx; h.ldc = ldx;
      h.alpha = -1.0; h.beta = 1.0;
      e = gemm_f64(false, true, EPI_STORE, h, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

}  // namespace pfsm
