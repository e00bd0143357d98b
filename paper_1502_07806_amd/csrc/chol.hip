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
__device__ inline void potrf_block(double* S, int64_t lds, int64_t k0, int nb, double* T, int* info) {
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

__global__ __launch_bounds__(512) void potrf_diag(double* S, int64_t lds, int64_t k0, int nb, double* T, int* info) {
  potrf_block(S, lds, k0, nb, T, info);
}

// ------------------------------------------------------------------------
// Gated Cholesky-QR with one launch per 64-wide block column (left-looking).
//
// The rows of X are treated as extra rows below S: factoring the stacked
// matrix [S; X] by columns gives L in the S rows and X L^{-T} in the X rows
// (the panel solve of a Cholesky step is exactly the triangular solve of the
// rows below it).  Launch t (t = 0 .. nblk), one workgroup per row block of
// rows at or below block t of S and one per row block of X:
//   1. (t >= 1) its own rows of block column t-1 are solved: R_{i,t-1} <-
//      R~_{i,t-1} T_{t-1}, T_{t-1} = L_{t-1,t-1}^{-T} from the previous launch;
//   2. (t < nblk) block column t is brought up to date, left-looking:
//      R~_{i,t} = R_{i,t} - sum_{j<t} R_{i,j} L_{t,j}^T.  The factor row
//      L_{t,j} is final in memory for j < t-1; L_{t,t-1} is recomputed by every
//      workgroup from a copy of the unsolved block R~_{t,t-1} (written by the
//      workgroup of row block t in the previous launch), because that
//      workgroup overwrites the block itself in step 1 of this launch;
//   3. the workgroup of row block t factors the diagonal block (potrf_block),
//      writing L_{t,t} and T_t; the one of row block t+1 also writes the copy
//      of R~_{t+1,t} for the next launch.
// Every workgroup writes only its own row block (and the one copy), so the
// launches need no synchronisation beyond their order on the stream.  The
// products run on the FP64 vector units (8 outputs per thread); this path is
// a fallback and is sized for correctness, not speed.
//
// Every kernel of the fallback returns at once when *gate == 0, so a fixed
// launch sequence (capturable into one graph) serves both cases.

constexpr int CK = 16;  // k chunk of the tile products

// acc (4 x 2 per thread, rows 4 (tid % 16) + u, columns 2 (tid / 16) + v of a
// 64 x 64 tile) += sgn * sum_k A(r, k) B(c, k) for k < K, with
// A(r, k) = A[r + k lda] for r < ra (else 0) and B(c, k) = B[c sbc + k sbk]
// for c < cb (else 0).  B may point to LDS (generic address).  512 threads.
__device__ inline void tile_gemm(double (&acc)[4][2], double sgn, const double* A, int64_t lda, int ra,
                                 const double* B, int64_t sbc, int64_t sbk, int cb, int64_t K, double (*As)[64],
                                 double (*Bs)[64]) {
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  const int lr = tid & 63, lk = tid >> 6;  // loader: row lr, k = lk and lk + 8
  for (int64_t k0 = 0; k0 < K; k0 += CK) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = lk + 8 * h;
      const int64_t k = k0 + kk;
      As[kk][lr] = (k < K && lr < ra) ? A[lr + k * lda] : 0.0;
      Bs[kk][lr] = (k < K && lr < cb) ? B[(int64_t)lr * sbc + k * sbk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < CK; ++kk) {
      double a[4], b[2];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][4 * tr + u];
#pragma unroll
      for (int v = 0; v < 2; ++v) b[v] = Bs[kk][2 * tc + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] += sgn * a[u] * b[v];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(512) void k_chol_ll(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m,
                                                 int t, double* Tbuf, double* Bcopy, int* info, const int* gate) {
  if (*gate == 0) return;
  __shared__ double As[CK][64], Bs[CK][64];
  __shared__ double Lt[64 * 64];  // L_{t,t-1}, Lt[c + 64 k]
  const int nblk = (int)((n + NB - 1) / NB);
  const int nS = nblk - t;  // S row blocks t .. nblk - 1
  const int b = blockIdx.x;
  const bool isS = b < nS;
  const int64_t r0 = isS ? (int64_t)(t + b) * NB : (int64_t)(b - nS) * NB;
  double* R = isS ? S : X;
  const int64_t ldr = isS ? lds : ldx;
  const int ra = (int)min<int64_t>(NB, (isS ? n : m) - r0);
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  double acc[4][2];
  auto zero = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) acc[u][v] = 0.0;
  };
  // writes acc to the 64 x cw block at (rows r0.., column c0) of R (ld ldr), rows < ra
  auto store = [&](double* D, int64_t ldd, int64_t c0, int cw, int rows) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int r = 4 * tr + u, c = 2 * tc + v;
        if (r < rows && c < cw) D[r + (c0 + c) * ldd] = acc[u][v];
      }
  };
  if (t >= 1) {
    // 1. own rows of block column t-1: R <- R~ T_{t-1}
    const int64_t c0 = (int64_t)(t - 1) * NB;
    const int cw = (int)min<int64_t>(NB, n - c0);
    const double* Tk = Tbuf + (int64_t)(t - 1) * NB * NB;  // T(k, c) = Tk[k + 64 c]
    zero();
    tile_gemm(acc, 1.0, R + r0 + c0 * ldr, ldr, ra, Tk, NB, 1, cw, cw, As, Bs);
    store(R + r0, ldr, c0, cw, ra);
    if (t < nblk) {
      // 2a. L_{t,t-1} = R~_{t,t-1} T_{t-1} from the copy (64 x 64, column-major)
      const int rt = (int)min<int64_t>(NB, n - (int64_t)t * NB);
      zero();
      tile_gemm(acc, 1.0, Bcopy + (int64_t)(t - 1) * NB * NB, NB, rt, Tk, NB, 1, cw, cw, As, Bs);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) Lt[(4 * tr + u) + 64 * (2 * tc + v)] = acc[u][v];
    }
    __syncthreads();  // own solved block and Lt visible to the whole workgroup
  }
  if (t >= nblk) return;
  // 2b. block column t, left-looking
  const int64_t ct = (int64_t)t * NB;
  const int cwt = (int)min<int64_t>(NB, n - ct);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int r = 4 * tr + u, c = 2 * tc + v;
      acc[u][v] = (r < ra && c < cwt) ? R[r0 + r + (ct + c) * ldr] : 0.0;
    }
  if (t >= 2)  // sum over j < t-1: own rows against the final factor rows of block t
    tile_gemm(acc, -1.0, R + r0, ldr, ra, S + ct, 1, lds, cwt, (int64_t)(t - 1) * NB, As, Bs);
  if (t >= 1) {  // j = t-1: own solved rows against L_{t,t-1} (LDS)
    const int64_t c0 = (int64_t)(t - 1) * NB;
    tile_gemm(acc, -1.0, R + r0 + c0 * ldr, ldr, ra, Lt, 1, 64, cwt, NB, As, Bs);
  }
  store(R + r0, ldr, ct, cwt, ra);
  if (isS && b == 1) store(Bcopy + (int64_t)t * NB * NB - ct * NB, NB, ct, cwt, ra);  // copy of R~_{t+1,t}
  if (isS && b == 0) {
    __syncthreads();  // the updated diagonal block is in memory
    potrf_block(S, lds, ct, cwt, Tbuf + (int64_t)t * NB * NB, info);
  }
}

// X64 (m x n) = X32 when *gate != 0.
__global__ __launch_bounds__(256) void k_f32_to_f64_gated(const float* X, int64_t ldx, double* Y, int64_t ldy, int64_t m,
                                                          int64_t n, const int* gate) {
  if (*gate == 0) return;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
      Y[i + j * ldy] = (double)X[i + j * ldx];
}
__global__ __launch_bounds__(256) void k_f64_to_f32_gated(const double* Y, int64_t ldy, float* X, int64_t ldx, int64_t m,
                                                          int64_t n, const int* gate) {
  if (*gate == 0) return;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
      X[i + j * ldx] = (float)Y[i + j * ldy];
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

hipError_t cholesky_qr_gated(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m, double* Tbuf,
                             double* Bcopy, int* info, const int* gate, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nblk = (int)((n + NB - 1) / NB);
  const int xb = (int)((m + NB - 1) / NB);
  for (int t = 0; t <= nblk; ++t) {
    const unsigned grid = (unsigned)((nblk - t) + xb);
    if (grid == 0) continue;
    hipLaunchKernelGGL(k_chol_ll, dim3(grid), dim3(512), 0, s, S, lds, X, ldx, n, m, t, Tbuf, Bcopy, info, gate);
  }
  return hipGetLastError();
}

hipError_t convert_f32_f64_gated(const float* X32, int64_t ld32, double* X64, int64_t ld64, int64_t m, int64_t n,
                                 int to_f64, const int* gate, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  // a modest grid, columns in a stride loop: when the gate is off every workgroup only reads it
  const dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 16), (unsigned)std::min<int64_t>(n, 128));
  if (to_f64)
    hipLaunchKernelGGL(k_f32_to_f64_gated, grid, dim3(256), 0, s, X32, ld32, X64, ld64, m, n, gate);
  else
    hipLaunchKernelGGL(k_f64_to_f32_gated, grid, dim3(256), 0, s, X64, ld64, (float*)X32, ld32, m, n, gate);
  return hipGetLastError();
}


}  // namespace pfsm
