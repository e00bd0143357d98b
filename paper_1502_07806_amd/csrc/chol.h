#pragma once
#include "common.h"
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
}  // namespace pfsm
