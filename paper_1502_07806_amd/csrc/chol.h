#pragma once
#include "common.h"
#include "gemm_x3.h"
namespace pfsm {
constexpr int CHOL_NB = 64;    // diagonal block (one wavefront, registers)
constexpr int CHOL_NB2 = 512;  // panel width between trailing updates
// Cholesky: S (n x n, lower valid) -> L in place.  Tbuf holds ceil(n/64) blocks
// of 64x64: the transposed inverses of the diagonal blocks of L.
hipError_t cholesky_factor(double* S, int64_t lds, int64_t n, double* Tbuf, int* info, hipStream_t s);
// X (m x n) <- X L^{-T} with the factor and Tbuf from cholesky_factor.
hipError_t trsm_right_lt(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t n, int64_t m,
                         const double* Tbuf, hipStream_t s);
// Cholesky-QR: S = L L^T, then X <- X L^{-T}.
hipError_t cholesky_qr(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m,
                       double* Tbuf, int* info, hipStream_t s);
// Cholesky factor of an overlap matrix close to the identity (the mixed
// path): S = L L^T with L = I + K, K lower triangular.  Equating lower
// triangles gives K = Phi(S - I - K K^T), Phi keeping the strictly lower
// part and half the diagonal; the map contracts like ||K||, so two steps
// from K0 = Phi(S - I) leave an error of order ||K||^3 ||S - I||.  Each
// product K K^T is a split-BF16 GEMM on lower tiles.  S (lower valid) is
// overwritten by L.  A last-step change larger than `tol` (no convergence)
// records info = -2.  Scratch: pk (packed operand, n rows of stride ldp),
// P and L1 (n x n FP64, leading dimension ldw), colmax (n doubles); split_ws
// (nullable, split_bytes) is the K-split scratch of the products.
hipError_t cholesky_near_identity(double* S, int64_t lds, int64_t n, bf16_t* pk, int64_t ldp, double* P, double* L1,
                                  int64_t ldw, double* colmax, double tol, int x3_cfg, float* split_ws,
                                  size_t split_bytes, int* info, hipStream_t s);
}  // namespace pfsm
