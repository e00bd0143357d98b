// Generalized -> standard conversion (internal to libpfsm).
#pragma once
#include "common.h"
namespace pfsm {
constexpr int PFSM_INFO_B_DIAG = -5;  // a diagonal entry of B is not a positive finite number

struct G2SWork {
  double* zbuf;    // n x n (ld n): the other buffer of the iterate pair
  double* dinv;    // [n] 1 / B_ii
  double* part;    // [ceil(n/128)][n] squared-residual partial sums
  double* anorm2;  // [n] squared column norms of A
  double* blk;     // [256] block sums of part
};
size_t g2s_workspace_bytes(int64_t n);
G2SWork g2s_carve(void* base, int64_t n);
// Z = B^{-1} A by Z_{k+1} = Z_k + D^{-1}(A - B Z_k), Z_0 = A (FP64 GEMMs).
// res (optional, device, [iterations]) receives ||A - B Z_k||_F / ||A||_F.
hipError_t g2s_run(int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb, int iterations, double* Z,
                   int64_t ldz, G2SWork w, double* res, int* info, hipStream_t s);
}  // namespace pfsm
