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
// The same Cholesky-QR with one launch per 64-wide block column (the rows of X
// factored as extra rows below S, left-looking), every kernel returning at once
// when *gate == 0.  S: n x n (lower triangle read) -> L; X: m x n -> X L^{-T};
// Tbuf as above; Bcopy: n x 64 doubles of scratch.  Breakdown at column k
// records info = k (1-based, first error wins).
hipError_t cholesky_qr_gated(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m, double* Tbuf,
                             double* Bcopy, int* info, const int* gate, hipStream_t s);
// X64 = X32 (to_f64 != 0) or X32 = X64, m x n, when *gate != 0.
hipError_t convert_f32_f64_gated(const float* X32, int64_t ld32, double* X64, int64_t ld64, int64_t m, int64_t n,
                                 int to_f64, const int* gate, hipStream_t s);
}  // namespace pfsm
