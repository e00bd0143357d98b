#pragma once
// FP64-accurate products on the int8 matrix cores (error-free digit splitting).
//
// Every operand row (a row of op(A), a column of B) is scaled by a power of
// two, 2^-e with e the exponent of its largest magnitude, and written as s
// signed digits d_1..d_s in [-64, 64]:
//     x = 2^e * sum_p d_p 2^(-6 - 7 (p - 1))  (+ a remainder of at most 2^(e - 7 s)),
// each digit the nearest integer of the scaled remainder, so all steps are
// exact in FP64.  Digit products accumulate exactly in int32 on the int8
// MFMA (|d_p d_q| <= 2^12, and s K < 2^19 keeps a group of up to s pairs
// below 2^31), and the groups of equal weight p + q = g are summed in FP64:
//     C(i, j) = 2^(e_i + f_j) * sum_{g = 2}^{s + 1} 2^(-12 - 7 (g - 2)) * sum_{p + q = g} (D_p E_q^T)(i, j).
// The dropped groups (p + q > s + 1) and the digit remainders (below
// 2^(-7 s) relative to the row maximum) bound the error by about
// (s + 1) K 2^(-7 s) 2^(e_i + f_j), and by sqrt(K) in place of K for entries of
// random sign (s = 5: 6 * 2^-35 per unit of K).
#include "common.h"

namespace pfsm {

constexpr int OZ_MAX_SLICES = 8;
constexpr int OZ_BM = 256, OZ_BN = 256, OZ_BK = 128;

// Digit-row stride in bytes (K rounded up to the k tile; the padding is zero).
inline int64_t oz_row_stride(int64_t K) { return (K + OZ_BK - 1) / OZ_BK * OZ_BK; }
// Bytes of the digit planes for `rows` operand rows of length K.
inline size_t oz_plane_bytes(int64_t rows, int64_t K, int s) { return (size_t)s * rows * oz_row_stride(K); }

// Split the columns of X (K x ncols, column-major, ldx) into s digit planes:
// plane p (0-based) holds column c's digits at P + p * ncols * ldp + c * ldp,
// ldp = oz_row_stride(K); expo[c] = e.  A column with a non-finite entry
// gets zero digits and records info = -1 (first error wins).
hipError_t oz_split(const double* X, int64_t ldx, int64_t K, int64_t ncols, int s, int8_t* P, int* expo, int* info,
                    hipStream_t st);

// C (M x N, column-major, ldc) = A B from the digit planes of the rows of A
// (Ap, ea: M operand rows) and of the columns of B (Bp, eb: N operand rows),
// both split with the same s and K.  The weight groups' FP64 values are
// added smallest weights first, C(i, j) = ((v_{s+1} + v_s) + ...) + v_2, in every
// tile configuration (cfg < 0: the default), so all give the same bits.
hipError_t gemm_oz(int64_t M, int64_t N, int64_t K, int s, const int8_t* Ap, const int* ea, const int8_t* Bp,
                   const int* eb, double* C, int64_t ldc, hipStream_t st, int cfg = -1);
extern int oz_default_cfg;  // tile configuration used when cfg < 0

hipError_t oz_init();  // once per process and device, before the first launch (large dynamic LDS)

}  // namespace pfsm
