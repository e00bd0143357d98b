// Conversion of the generalized problem A x = lambda B x to standard form
// (Implementation section, Eqs. 13-15): Z = B^{-1} A without forming B^{-1},
// by the stationary iteration Z_{k+1} = (I - D^{-1} B) Z_k + D^{-1} A with D
// the diagonal of B, started from Z_0 = A (the identity approximates B^{-1}
// for a diagonally dominant overlap).  It is evaluated as
// Z_{k+1} = Z_k + D^{-1}(A - B Z_k): one FP64 MFMA GEMM per step whose
// epilogue applies the row scaling and the update and accumulates the
// squared residual of Z_k per column.  Columns of Z evolve independently.
// B is an overlap matrix, symmetric: the product is taken as B^T Z.
#include "g2s.h"
#include "misc.h"

#include <algorithm>

namespace pfsm {
namespace {

constexpr int NT = 256;

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ __launch_bounds__(NT) void k_g2s_dinv(const double* B, int64_t ldb, int64_t n, double* dinv, int* info) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double d = B[i + i * ldb];
  if (!(d > 0.0 && d <= 1.7976931348623157e308)) {
    atomicCAS(info, 0, PFSM_INFO_B_DIAG);
    dinv[i] = __builtin_nan("");
    return;
  }
  dinv[i] = 1.0 / d;
}

__global__ __launch_bounds__(NT) void k_copy_cols(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t m) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (int64_t)gridDim.x * NT)
    Y[i + j * ldy] = X[i + j * ldx];
}

constexpr int RB = 256;  // blocks of the first reduction stage

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// blk[b] = sum of part[i] over the i that block b strides over (fixed order).
__global__ __launch_bounds__(NT) void k_g2s_res_part(const double* part, int64_t count, double* blk) {
  __shared__ double sh[NT];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < count; i += (int64_t)RB * NT) a += part[i];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) blk[blockIdx.x] = a;
}

// res[k] = sqrt(sum blk / sum anorm2); a non-finite result records info = -1.
__global__ __launch_bounds__(NT) void k_g2s_res(const double* blk, const double* anorm2, int64_t n, double* res,
                                                int* info) {
  __shared__ double sh[NT];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < RB; i += NT) a += blk[i];
  for (int64_t i = threadIdx.x; i < n; i += NT) b += anorm2[i];
  a = block_sum(a, sh);
  __syncthreads();
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    const double r = b > 0.0 ? sqrt(a / b) : sqrt(a);
    if (res) *res = r;
    if (!(r <= 1.7976931348623157e308)) atomicCAS(info, 0, -1);
  }
}

}  // namespace

size_t g2s_workspace_bytes(int64_t n) {
  const int64_t tiles_m = (n + GEMM_BM - 1) / GEMM_BM;
  return al256((size_t)n * n * sizeof(double)) + al256((size_t)n * sizeof(double)) +
         al256((size_t)tiles_m * n * sizeof(double)) + al256((size_t)n * sizeof(double)) +
         al256((size_t)RB * sizeof(double));
}

G2SWork g2s_carve(void* base, int64_t n) {
  const int64_t tiles_m = (n + GEMM_BM - 1) / GEMM_BM;
  char* p = (char*)base;
  G2SWork w;
  w.zbuf = (double*)p;
  p += al256((size_t)n * n * sizeof(double));
  w.dinv = (double*)p;
  p += al256((size_t)n * sizeof(double));
  w.part = (double*)p;
  p += al256((size_t)tiles_m * n * sizeof(double));
  w.anorm2 = (double*)p;
  p += al256((size_t)n * sizeof(double));
  w.blk = (double*)p;
  return w;
}

hipError_t g2s_run(int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb, int iterations, double* Z,
                   int64_t ldz, G2SWork w, double* res, int* info, hipStream_t s) {
  const int64_t tiles_m = (n + GEMM_BM - 1) / GEMM_BM;
  hipError_t e = fill_i32(info, 1, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_g2s_dinv, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, B, ldb, n, w.dinv, info);
  e = col_norm2(A, n, n, lda, w.anorm2, s);
  if (e != hipSuccess) return e;
  // the iterate pair: Z_K must end in Z, so Z_0 goes to Z when K is even
  double* cur = (iterations % 2 == 0) ? Z : w.zbuf;
  int64_t ldc = (iterations % 2 == 0) ? ldz : n;
  double* nxt = (iterations % 2 == 0) ? w.zbuf : Z;
  int64_t ldn = (iterations % 2 == 0) ? n : ldz;
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)std::min<int64_t>((n + NT - 1) / NT, 64), (unsigned)n), dim3(NT), 0,
                     s, A, lda, cur, ldc, n);
  for (int k = 0; k < iterations; ++k) {
    GemmArgs g = {};
    g.M = n; g.N = n; g.K = n; g.A = B; g.lda = ldb; g.B = cur; g.ldb = ldc; g.C = nxt; g.ldc = ldn;
    g.D = A; g.ldd = lda; g.eps = w.dinv; g.part = w.part;
    e = gemm_f64(true, false, EPI_G2S, g, s);  // B symmetric: B^T Z = B Z in the faster TN layout
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_g2s_res_part, dim3(RB), dim3(NT), 0, s, w.part, tiles_m * n, w.blk);
    hipLaunchKernelGGL(k_g2s_res, dim3(1), dim3(NT), 0, s, w.blk, w.anorm2, n, res ? res + k : nullptr, info);
    std::swap(cur, nxt);
    std::swap(ldc, ldn);
  }
  return hipGetLastError();
}

}  // namespace pfsm
