#pragma once
#include "common.h"
namespace pfsm {
constexpr int REFINE_KMAX = 32;         // largest cluster handled by one Rayleigh-Ritz block
constexpr double REFINE_TAU = 1e-4;     // relative gap below which neighbours are refined together
// Largest |S - I| (overlap of the folded-spectrum vectors) for which the
// mixed path keeps the first-order orthonormalisation; above it the FP64
// Cholesky-QR of the overlap runs instead.
constexpr double ORTHO_FIRST_ORDER_MAX = 1e-3;
// Digits per operand of the refinement product Z = A V_new on the int8 matrix
// cores: the fewest for which the Rayleigh quotients stay well inside 1e-8 of
// max|lambda| (s = 5, s (s + 1) / 2 = 15 digit products).  Each entry of Z
// errs by at most (s + 1) 2^-7s 2^(e_i + f_j) per term of its sum (e_i, f_j:
// exponents of the row and column maxima), about sqrt(n) times that for
// errors of random sign; the Rayleigh quotient of a unit vector inherits
// about the same size: at n = 8192 (2^e_i ~ 1, 2^f_j ~ 1/16) that is
// 6 * 2^-35 * 90.5 / 16 ~ 1e-9, against 7e-8 for s = 4 and 6e-12 for s = 6.
constexpr int REFINE_OZ_SLICES = 5;

constexpr int PFSM_INFO_RESIDUAL = -2;  // a residual above the plan's threshold

struct RefineBufs {
  double* d;       // [n] v_j^T z_j
  double* nn;      // [n] v_j^T v_j
  double* lam_s;   // [n] sorted estimates
  int* rank;       // [n] column -> sorted position
  int* inv;        // [n] sorted position -> column
  int* clus;       // [1] number of clusters
  int* cstart;     // [n] cluster starts
  int* csize;      // [n] cluster sizes
  double* zz = nullptr;     // [n] z_j^T z_j (with resid)
  double* resid = nullptr;  // [n] optional: residuals ||A v - lambda v|| of the outputs, output order
};

// FP64 refinement of the eigenpair estimates (columns of V, Z = A V):
// Rayleigh quotients, ascending order, Rayleigh-Ritz on each cluster of
// estimates closer than tau * max|lambda|, normalisation; writes lambda and
// Vout (column-major, ldvo).
hipError_t refine_rr(const double* V, int64_t ldv, const double* Z, int64_t ldz, int64_t n, double tau,
                     double* lam, double* Vout, int64_t ldvo, RefineBufs b, int* info, hipStream_t s);

// info = -2 when max_i r[i] > tol * max_i |lam[i]| (or not a number).
hipError_t residual_check(const double* r, const double* lam, int64_t n, double tol, int* info, hipStream_t s);
// FP64 path: r_out[rank[j]] = sqrt(max(zz[j] - lam[j]^2, 0)).
hipError_t residuals_from_rq(const double* zz, const double* lam, const int* rank, int64_t n, double* r_out,
                             hipStream_t s);

// Mixed-path helpers.
hipError_t f32_mirror_lower(float* At32, double* diag, int64_t n, hipStream_t s);  // lower -> both; diag in FP64
// *gate = 1 when max |L - I| over the lower triangle exceeds limit (or is not
// a number), else 0; scratch: n doubles.  cl (optional, 2 doubles): n max |L - I|
// (a bound on the absolute row sums of the first-order correction) and
// PFSM_BAND_TOL, the gate of the correction's band form.
hipError_t lower_minus_identity_check(const double* L, int64_t ldl, int64_t n, double limit, double* scratch,
                                      int* gate, double* cl, hipStream_t s);
hipError_t col_sign_f32(float* X, int64_t n, int64_t ldx, double* sgn, hipStream_t s);  // flips in place
hipError_t permute_f64_cols(const double* X, int64_t ldx, const int* rank, double* Y, int64_t ldy, int64_t m,
                            int64_t n, hipStream_t s);
}  // namespace pfsm
