// Internal declarations shared by the HIP translation units of libpfsm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace pfsm {

// Band forms of the mixed path's products (folded-spectrum products and the
// orthonormalisation correction): the terms a product restricted to the
// submatrix rows drops must stay below this bound, relative to the scale of
// the product's output (2^-20, far below the 2^-9 rounding of the plain BF16
// products of the whole matrix that the full forms compute).
constexpr double PFSM_BAND_TOL = 9.5367431640625e-07;

// ---------------------------------------------------------------- GEMM (FP64)
// C = op(A) op(B) with a fused epilogue.  Column-major storage throughout.
enum GemmEpi : int {
  EPI_STORE = 0,   // C = alpha*acc + beta*C
  EPI_SHIFT = 1,   // C = acc - B(i,j) * eps[j]            (B square operand, not transposed)
  EPI_FSUPD = 2,   // C = D(i,j) - a * (acc - B(i,j)*eps[j]), a = *alpha_dev or alpha
  EPI_RQ = 3,      // part[tile_m][j] = sum_{i in tile} acc(i,j) * D(i,j)   (C untouched); and
                   // part2[tile_m][j] = sum_{i in tile} acc(i,j)^2 when part2 is set
  EPI_G2S = 4,     // C = B(i,j) + eps[i] * (D(i,j) - acc); part[tile_m][j] = sum_i (D(i,j) - acc)^2
                   // when part is set (B square operand, not transposed; C must not alias B)
};

struct GemmArgs {
  int64_t M, N, K;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  double alpha, beta;
  const double* alpha_dev;   // optional device scalar for EPI_FSUPD
  const double* eps;         // column shifts for EPI_SHIFT / EPI_FSUPD, row scales for EPI_G2S
  const double* D; int64_t ldd;  // FSUPD base matrix / RQ partner matrix
  double* part;              // RQ partial sums [tiles_m x N]
  double* part2;             // RQ, optional: partial sums of acc^2 [tiles_m x N] (squared column norms of A X)
  const int32_t* krange;     // optional [tiles_n][2] K range per column tile
  int lower_only;            // skip tiles strictly above the diagonal
};

constexpr int GEMM_BM = 128, GEMM_BN = 128, GEMM_BK = 16;

hipError_t gemm_f64(bool ta, bool tb, int epi, const GemmArgs& a, hipStream_t s);

// ---------------------------------------------------------------- misc kernels
hipError_t mirror_lower(double* C, int64_t n, int64_t ldc, hipStream_t s);

}  // namespace pfsm
