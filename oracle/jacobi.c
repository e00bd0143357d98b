/*
 * Oracle (test infrastructure only; never linked into the product library).
 *
 * Cyclic two-sided Jacobi eigensolver for a dense real symmetric matrix, FP64.
 * It is the "exact" eigendecomposition the method is compared with: the paper
 * poses the reduced problem A x_i = lambda_i x_i (Eq. 3) and delegates it to
 * standard dense solvers; a Jacobi sweep is the textbook way to compute it
 * (Golub & Van Loan, Matrix Computations, cyclic Jacobi with the 2x2
 * symmetric Schur decomposition).
 *
 * Storage: column-major, a[i + j*lda].  The matrix is overwritten; on return
 * its diagonal holds the (unsorted) eigenvalues.  v (ldv) receives the
 * eigenvectors as columns.  Row-cyclic order: (0,1), (0,2), ..., (n-2,n-1).
 * A pair is rotated when |a_pq| exceeds tol * sqrt(|a_pp| |a_qq|) (relative
 * threshold) or when it is larger than tiny; a sweep without any rotation ends
 * the iteration.  Returns the number of sweeps, or -1 if max_sweeps ran out.
 */
#include <math.h>
#include <stdint.h>

int oracle_jacobi_eigh(int64_t n, double* a, int64_t lda, double* v, int64_t ldv,
                       double tol, int max_sweeps) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) v[i + j * ldv] = (i == j) ? 1.0 : 0.0;
  if (n < 2) return 0;
  const double tiny = 1e-300;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    int64_t rotations = 0;
    for (int64_t p = 0; p < n - 1; ++p) {
      for (int64_t q = p + 1; q < n; ++q) {
        double apq = a[p + q * lda];
        double app = a[p + p * lda];
        double aqq = a[q + q * lda];
        double thr = tol * sqrt(fabs(app) * fabs(aqq));
        if (fabs(apq) <= thr || fabs(apq) <= tiny) continue;
        ++rotations;
        /* 2x2 symmetric Schur decomposition: choose t = tan(theta) with
           |theta| <= pi/4 so that the rotated (p,q) entry vanishes. */
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = t * c;
        /* A <- J^T A J with J = [[c, s], [-s, c]] acting on rows/cols p, q. */
        for (int64_t k = 0; k < n; ++k) {  /* columns p, q */
          double akp = a[k + p * lda], akq = a[k + q * lda];
          a[k + p * lda] = c * akp - s * akq;
          a[k + q * lda] = s * akp + c * akq;
        }
        for (int64_t k = 0; k < n; ++k) {  /* rows p, q */
          double apk = a[p + k * lda], aqk = a[q + k * lda];
          a[p + k * lda] = c * apk - s * aqk;
          a[q + k * lda] = s * apk + c * aqk;
        }
        a[p + q * lda] = 0.0;
        a[q + p * lda] = 0.0;
        for (int64_t k = 0; k < n; ++k) {  /* eigenvectors V <- V J */
          double vkp = v[k + p * ldv], vkq = v[k + q * ldv];
          v[k + p * ldv] = c * vkp - s * vkq;
          v[k + q * ldv] = s * vkp + c * vkq;
        }
      }
    }
    if (rotations == 0) return sweep;
  }
  return -1;
}
