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
#include "gemm_x3.h"
#include "refine.h"

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

// One fixed-point step of the near-identity Cholesky, column j per block:
// out = I + Phi(S - I - P) on the lower triangle (P = K K^T of the previous
// iterate); with prev (the previous I + K), colmax[j] = max |out - prev|.
// out may alias S (each element is read before it is written).
__global__ __launch_bounds__(256) void k_chol_fp_step(const double* S, int64_t lds, const double* P, int64_t ldp,
                                                      double* out, int64_t ldo, const double* prev, int64_t ldprev,
                                                      double* colmax, int64_t n) {
  __shared__ double sh[256];
  const int64_t j = blockIdx.x;
  double m = 0.0;
  for (int64_t i = j + threadIdx.x; i < n; i += 256) {
    const double e = S[i + j * lds] - (i == j ? 1.0 : 0.0) - P[i + j * ldp];
    const double o = (i == j) ? 1.0 + 0.5 * e : e;
    if (prev) {
      const double d = fabs(o - prev[i + j * ldprev]);
      m = (d > m || d != d) ? d : m;
    }
    out[i + j * ldo] = o;
  }
  if (!prev) return;
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = sh[threadIdx.x + w];
      sh[threadIdx.x] = (o > sh[threadIdx.x] || o != o) ? o : sh[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) colmax[j] = sh[0];
}

__global__ __launch_bounds__(256) void k_colmax_check(const double* colmax, int64_t n, double limit, int code,
                                                      int* info) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = colmax[i];
    m = (v > m || v != v) ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = sh[threadIdx.x + w];
      sh[threadIdx.x] = (o > sh[threadIdx.x] || o != o) ? o : sh[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(sh[0] <= limit)) atomicCAS(info, 0, code);
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

hipError_t cholesky_near_identity(double* S, int64_t lds, int64_t n, bf16_t* pk, int64_t ldp, double* P, double* L1,
                                  int64_t ldw, double* colmax, double tol, int x3_cfg, float* split_ws,
                                  size_t split_bytes, int* info, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  X3Args g = {};
  g.M = n; g.N = n; g.K = n; g.Ap = pk; g.ldap = ldp; g.Bp = pk; g.ldbp = ldp; g.C = P; g.ldc = ldw;
  g.c_double = 1; g.alpha = 1.0; g.tiles = X3_LOWER; g.cfg = x3_cfg;
  g.split_ws = split_ws; g.split_bytes = split_bytes;
  // step 1: K0 = Phi(S - I) packed by rows; L1 = I + Phi(S - I - K0 K0^T)
  CHK(pack_x3(S, 1, n, n, lds, PACK_BY_ROWS | PACK_LOWER | PACK_SUB_I | PACK_HALF_DIAG, pk, ldp, s));
  CHK(gemm_x3(X3_STORE, g, s));
  hipLaunchKernelGGL(k_chol_fp_step, dim3((unsigned)n), dim3(256), 0, s, S, lds, P, ldw, L1, ldw, nullptr, 0,
                     nullptr, n);
  // step 2: K1 = L1 - I; S <- I + Phi(S - I - K1 K1^T), change against L1 checked
  CHK(pack_x3(L1, 1, n, n, ldw, PACK_BY_ROWS | PACK_LOWER | PACK_SUB_I, pk, ldp, s));
  CHK(gemm_x3(X3_STORE, g, s));
  hipLaunchKernelGGL(k_chol_fp_step, dim3((unsigned)n), dim3(256), 0, s, S, lds, P, ldw, S, lds, L1, ldw, colmax, n);
  hipLaunchKernelGGL(k_colmax_check, dim3(1), dim3(256), 0, s, colmax, n, tol, PFSM_INFO_SERIES, info);
  return hipGetLastError();
}

}  // namespace pfsm
