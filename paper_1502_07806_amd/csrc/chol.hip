// Blocked FP64 Cholesky of the overlap matrix S = X^T X and the right-side
// triangular solve X <- X L^{-T} (the orthonormalisation step, computed as
// Cholesky-QR).
//
// Two-level blocking: 64-wide diagonal blocks are factored by one wavefront
// with each lane holding one row in registers (column values are broadcast
// through LDS), which also forms L_kk^{-T}; the 64-wide panel solve is an
// MFMA GEMM with that inverse; updates inside a 512-wide panel are rank-64
// GEMMs restricted to the panel, and the rest of the matrix receives one
// rank-512 update per panel, so the trailing matrix is streamed N/512 times
// instead of N/64 times.
#include "common.h"
#include "chol.h"

namespace pfsm {
namespace {

constexpr int NB = CHOL_NB;      // 64
constexpr int NB2 = CHOL_NB2;    // 512

// One wavefront: factor S[k0:k0+nb, k0:k0+nb] (lower triangle) in place and
// write T = L^{-T} (upper triangular, 64 x 64 column-major; identity padding
// past nb).  The block lives in LDS (row-major, padded); lane i updates row i,
// and the column being eliminated is read as a broadcast (all lanes read the
// same address).  With a single-wave workgroup each barrier is cheap.  A
// non-positive or non-finite pivot records info = global column (1-based),
// first error wins, and the factorisation continues with NaN.
__global__ __launch_bounds__(64) void potrf_diag(double* S, int64_t lds, int64_t k0, int nb, double* T, int* info) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int i = threadIdx.x;  // this lane's row
  double* Sk = S + k0 + k0 * lds;
  for (int c = 0; c < NB; ++c) {
    double v = (i == c) ? 1.0 : 0.0;
    if (i < nb && c < nb && c <= i) v = Sk[i + c * lds];
    L[i][c] = v;
    X[i][c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  // right-looking Cholesky: column j is finished at step j
  for (int j = 0; j < NB; ++j) {
    double d = L[j][j];
    if (!(d > 0.0)) {
      if (i == 0 && j < nb) atomicCAS(info, 0, (int)(k0 + j + 1));
      d = __builtin_nan("");
    }
    const double sj = sqrt(d);
    const double lij = (i == j) ? sj : L[i][j] / sj;
    __syncthreads();
    if (i >= j) L[i][j] = lij;
    __syncthreads();
#pragma unroll 4
    for (int c = j + 1; c < NB; ++c) {
      const double lcj = L[c][j];
      if (i >= c) L[i][c] -= lij * lcj;
    }
    __syncthreads();
  }
  // X = L^{-1}: right-looking forward substitution on the identity (row k final at step k)
  for (int k = 0; k < NB; ++k) {
    const double lkk = L[k][k];
    if (i <= k) X[k][i] /= lkk;  // lane c scales X[k][c]
    __syncthreads();
    const double lik = L[i][k];
#pragma unroll 4
    for (int c = 0; c <= k; ++c) {
      const double xkc = X[k][c];
      if (i > k) X[i][c] -= lik * xkc;
    }
    __syncthreads();
  }
  for (int c = 0; c < NB; ++c) {
    if (i < nb && c < nb && c <= i) Sk[i + c * lds] = L[i][c];
  }
  // T(r, c) = (L^{-1})(c, r): lane i writes column i of T = row i of L^{-1}
  for (int r = 0; r < NB; ++r) {
    double v;
    if (i < nb && r < nb) v = (r <= i) ? X[i][r] : 0.0;
    else v = (r == i) ? 1.0 : 0.0;
    T[r + i * NB] = v;
  }
}

hipError_t gemm_store(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, bool tb, const double* B,
                      int64_t ldb, double* C, int64_t ldc, double alpha, double beta, int lower, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  GemmArgs g = {};
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.lower_only = lower;
  return gemm_f64(false, tb, EPI_STORE, g, s);
}

#define CHK(x)                           \
  do {                                   \
    hipError_t _e = (x);                 \
    if (_e != hipSuccess) return _e;     \
  } while (0)

}  // namespace

hipError_t cholesky_factor(double* S, int64_t lds, int64_t n, double* Tbuf, int* info, hipStream_t s) {
  // S: n x n (lower triangle valid) -> L in place; Tbuf receives the inverse-transposed diagonal blocks.
  for (int64_t K0 = 0; K0 < n; K0 += NB2) {
    const int64_t w = std::min<int64_t>(NB2, n - K0);
    for (int64_t k0 = K0; k0 < K0 + w; k0 += NB) {
      const int nb = (int)std::min<int64_t>(NB, K0 + w - k0);
      double* T = Tbuf + (k0 / NB) * NB * NB;
      hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(64), 0, s, S, lds, k0, nb, T, info);
      const int64_t rest = n - k0 - nb;
      double* L21 = S + (k0 + nb) + k0 * lds;
      // panel: L21 = S21 T (in place; one column tile per row tile)
      CHK(gemm_store(rest, nb, nb, L21, lds, false, T, NB, L21, lds, 1.0, 0.0, 0, s));
      // update the remaining columns of this 512-wide panel: S[k0+nb:, k0+nb:K0+w] -= L21 L21[:pc]^T
      const int64_t pc = K0 + w - (k0 + nb);
      CHK(gemm_store(rest, pc, nb, L21, lds, true, L21, lds, S + (k0 + nb) + (k0 + nb) * lds, lds, -1.0, 1.0, 0, s));
    }
    // one rank-w update of the trailing matrix (lower tiles)
    const int64_t rest2 = n - K0 - w;
    double* P = S + (K0 + w) + K0 * lds;
    CHK(gemm_store(rest2, rest2, w, P, lds, true, P, lds, S + (K0 + w) + (K0 + w) * lds, lds, -1.0, 1.0, 1, s));
  }
  return hipGetLastError();
}

hipError_t trsm_right_lt(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t n, int64_t m,
                         const double* Tbuf, hipStream_t s) {
  // X (m x n) <- X L^{-T}, same two-level blocking over column blocks.
  for (int64_t K0 = 0; K0 < n; K0 += NB2) {
    const int64_t w = std::min<int64_t>(NB2, n - K0);
    for (int64_t k0 = K0; k0 < K0 + w; k0 += NB) {
      const int nb = (int)std::min<int64_t>(NB, K0 + w - k0);
      double* Xk = X + k0 * ldx;
      CHK(gemm_store(m, nb, nb, Xk, ldx, false, Tbuf + (k0 / NB) * NB * NB, NB, Xk, ldx, 1.0, 0.0, 0, s));
      const int64_t pc = K0 + w - (k0 + nb);
      CHK(gemm_store(m, pc, nb, Xk, ldx, true, L + (k0 + nb) + k0 * ldl, ldl, X + (k0 + nb) * ldx, ldx, -1.0, 1.0, 0, s));
    }
    const int64_t rest2 = n - K0 - w;
    CHK(gemm_store(m, rest2, w, X + K0 * ldx, ldx, true, L + (K0 + w) + K0 * ldl, ldl, X + (K0 + w) * ldx, ldx, -1.0,
                   1.0, 0, s));
  }
  return hipGetLastError();
}

hipError_t cholesky_qr(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m, double* Tbuf, int* info,
                       hipStream_t s) {
  CHK(cholesky_factor(S, lds, n, Tbuf, info, s));
  return trsm_right_lt(S, lds, X, ldx, n, m, Tbuf, s);
}

}  // namespace pfsm
