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

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Factor S[k0:k0+nb, k0:k0+nb] (lower triangle) in place and write
// T = L^{-T} (upper triangular, 64 x 64 column-major; identity padding past
// nb).  512 threads in two groups of four waves.  Factor group: thread
// (w, i) holds row i of L, columns 16w .. 16w+15, in registers.  Step j:
// the wave owning column j takes the pivot from lane j (readlane), scales
// the column by one reciprocal square root (as LAPACK's unblocked Cholesky
// does) and publishes it through an LDS column buffer; after one barrier
// every factor wave updates its own columns past j.  Entries above the
// diagonal are left as scratch (never read back).  Inverse group: forms
// L^{-1} one step behind, by right-looking forward substitution on the
// identity (wave owning columns 16w.. of L^{-1}, row k taken from lane k by
// readlane), so it runs in the time the factor group spends waiting on the
// pivot chain.  The j loop is unrolled by 16 so that register indices are
// static and finished columns cost nothing.  Two column buffers suffice: the
// last read of column j (the inverse step) comes before the barrier after
// which column j+2 is written.  A non-positive or non-finite pivot records
// info = global column (1-based), first error wins, and the factorisation
// continues with NaN.
__global__ __launch_bounds__(512) void potrf_diag(double* S, int64_t lds, int64_t k0, int nb, double* T, int* info) {
  constexpr int CW = NB / 4;  // columns per wave
  __shared__ __attribute__((aligned(16))) double colbuf[2][NB];
  __shared__ double rdiag[NB];
  __shared__ double Lsh[NB][NB + 1];
  const bool fac = threadIdx.x < 256;
  const int w = (threadIdx.x >> 6) & 3, i = threadIdx.x & 63;
  const int cbase = w * CW;
  double* Sk = S + k0 + k0 * lds;
  double r[CW];  // factor group: row i of L; inverse group: row i of L^{-1}
#pragma unroll
  for (int t = 0; t < CW; ++t) {
    const int c = cbase + t;
    double v = (i == c) ? 1.0 : 0.0;
    if (fac && i < nb && c < nb && c <= i) v = Sk[i + c * lds];
    r[t] = v;
  }
#pragma unroll 1
  for (int jb = 0; jb < NB / CW; ++jb) {
#pragma unroll
    for (int jl = 0; jl < CW; ++jl) {
      const int j = jb * CW + jl;
      double* colj = colbuf[j & 1];
      if (fac) {
        if (w == jb) {
          double d = readlane_d(r[jl], j);
          if (!(d > 0.0)) {
            if (i == 0 && j < nb) atomicCAS(info, 0, (int)(k0 + j + 1));
            d = __builtin_nan("");
          }
          // 1/sqrt(d): hardware estimate refined by two Newton steps (the
          // correctly rounded sqrt and division sequences are far longer)
          double inv = __builtin_amdgcn_rsq(d);
          inv = inv * (1.5 - 0.5 * d * inv * inv);
          inv = inv * (1.5 - 0.5 * d * inv * inv);
          const double lij = (i == j) ? d * inv : r[jl] * inv;
          if (i >= j) r[jl] = lij;
          colj[i] = (i >= j) ? lij : 0.0;
          if (i == 0) rdiag[j] = inv;
        }
      } else if (j > 0) {
        // inverse step k = j - 1 (its column and pivot were published last step)
        const int k = j - 1, kb = k / CW, kl = k % CW;  // kl is static after unrolling
        if (w <= kb) {
          const double lik = (i > k) ? colbuf[k & 1][i] : 0.0;
          if (i == k) {
            const double rk = rdiag[k];
#pragma unroll
            for (int t = 0; t < CW; ++t) r[t] *= rk;
          }
#pragma unroll
          for (int t = 0; t < CW; ++t)
            if (w < kb || t <= kl) r[t] -= lik * readlane_d(r[t], k);
        }
      }
      __syncthreads();
      if (fac && w >= jb) {
        const double li = colj[i];  // L(i, j); zero above the diagonal
        double v[CW];
#pragma unroll
        for (int t = 0; t < CW; t += 2) {
          const double2 p2 = *(const double2*)&colj[cbase + t];
          v[t] = p2.x;
          v[t + 1] = p2.y;
        }
#pragma unroll
        for (int t = 0; t < CW; ++t)
          if (w > jb || t > jl) r[t] -= li * v[t];
      }
    }
  }
  if (fac) {
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int c = cbase + t;
      if (i < nb && c < nb && c <= i) Sk[i + c * lds] = r[t];
    }
  } else {
    // last inverse step k = NB - 1 only scales row NB - 1; then stage
    // T(c, i) = (L^{-1})(i, c) through LDS so the stores are contiguous
    if (i == NB - 1) {
      const double rk = rdiag[NB - 1];
#pragma unroll
      for (int t = 0; t < CW; ++t) r[t] *= rk;
    }
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int c = cbase + t;
      Lsh[c][i] = (i < nb && c < nb) ? (c <= i ? r[t] : 0.0) : (i == c ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  if (!fac) {
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int col = cbase + t;  // column col of T, row i
      T[i + col * NB] = Lsh[i][col];
    }
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
      hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(512), 0, s, S, lds, k0, nb, T, info);
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
