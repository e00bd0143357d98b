#pragma once
#include "common.h"
namespace pfsm {
hipError_t fill_i32(int* p, int64_t count, int value, hipStream_t s);
// y[i] = deterministic pseudo-random values in [-1, 1) (hash of i and seed).
hipError_t fill_hash_f32(float* y, int64_t count, uint32_t seed, hipStream_t s);
// Zero rows [krange[2 t], krange[2 t + 1]) (clipped to m) of every column c of
// X (m x n, column-major), t = c / tile_n: what remains is X outside the K
// range a per-column-tile product with that krange covers.
hipError_t zero_krange_rows(float* X, int64_t ldx, int64_t m, int64_t n, const int32_t* krange, int64_t tile_n,
                            hipStream_t s);
// Gershgorin interval of At (scal[1], scal[2]), the step length alpha (scal[0]),
// the largest off-diagonal absolute row sum (scal[3]) and PFSM_BAND_TOL times
// the Gershgorin bound (scal[4]); info = -1 if not finite.
hipError_t gershgorin_alpha(const double* At, int64_t n, int64_t ld, int q, double user_alpha,
                            double* part_lo, double* part_hi, double* scal, int* info, hipStream_t s);
// The same from FP32 columns (each entry widened exactly to FP64).
hipError_t gershgorin_alpha(const float* At, int64_t n, int64_t ld, int q, double user_alpha,
                            double* part_lo, double* part_hi, double* scal, int* info, hipStream_t s);
hipError_t rq_reduce(const double* part, int tiles_m, int64_t n, const double* den, double* out, hipStream_t s);
hipError_t col_norm2(const double* X, int64_t m, int64_t n, int64_t ldx, double* out, hipStream_t s);
hipError_t finalize_order(const double* lam_u, const double* X, int64_t n, int64_t ldx, double* Xp, int64_t ldxp,
                          double* lam_out, int* rank, double* sgn, int* info, hipStream_t s);
// rank[j] = stable ascending rank of num[j] (of num[j] / den[j] when den is
// given) in the NaN-last total order; a permutation of 0..n-1 for any input.
hipError_t rank_ascending(const double* num, const double* den, int64_t n, int* rank, hipStream_t s);
// Stable ascending ranks of lam_u (NaN last, info = -1 for non-finite) and lam_out[rank] = lam_u.
hipError_t finalize_order_values(const double* lam_u, int64_t n, double* lam_out, int* rank, int* info, hipStream_t s);
constexpr int PFSM_INFO_BASIS = -4;
// info = -4 when some nn[j] (squared column norm) is outside [1/4, 4] or not finite.
hipError_t norm_check(const double* nn, int64_t n, int* info, hipStream_t s);
hipError_t adjoint_middle(double* T, int64_t ldt, int64_t n, const double* lam, const double* glam, double eta,
                          bool have_t, hipStream_t s);
hipError_t symmetrize(double* C, int64_t n, int64_t ldc, hipStream_t s);
hipError_t scale_cols(const double* V, int64_t n, int64_t ldv, const double* d, double* out, int64_t ldo, hipStream_t s);
hipError_t diag_sums(const double* A, int64_t lda, const double* AV, int64_t ldav, const double* V, int64_t ldv,
                     const double* lam, const double* G, int64_t ldg, int64_t n, double* part, double* out,
                     hipStream_t s);
}  // namespace pfsm
