#pragma once
#include "common.h"
namespace pfsm {
constexpr int CHOL_NB = 64;
// Cholesky-QR: S (n x n, lower valid) -> L in place; X (m x n) <- X L^{-T}.
// Tbuf holds ceil(n/64) blocks of 64x64 (the transposed inverse diagonal blocks).
hipError_t cholesky_factor(double* S, int64_t lds, int64_t n, double* Tbuf, int* info, hipStream_t s);
hipError_t cholesky_qr(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m,
                       double* Tbuf, int* info, hipStream_t s);
}  // namespace pfsm
