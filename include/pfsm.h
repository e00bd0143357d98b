/*
 * libpfsm -- partitioned folded spectrum method (PFSM) subspace
 * diagonalisation on AMD Instinct MI355X (gfx950).
 *
 * Method: Briggs, Kelley, Bernholc, "Parallel implementation of electronic
 * structure eigensolver using a partitioned folded spectrum method"
 * (arXiv:1502.07806).  Given a real symmetric A (Eq. 3) and the previous
 * eigenvectors V_prev, one call
 *   1. forms the operator in the previous basis, At = V_prev^T A V_prev
 *      (the matrix elements of Eq. 12);
 *   2. splits the eigen-index range into slices, one per partition, and
 *      diagonalises an overlapping diagonal submatrix of At around each slice
 *      (Methodology: submatrices of order M, slice inside its submatrix,
 *      Fig. 1);
 *   3. pads the selected submatrix eigenvectors with zeros to start vectors
 *      and uses the submatrix eigenvalues as shifts;
 *   4. applies folded-spectrum iterations x <- x - alpha (At - eps I)^q x
 *      (Eq. 11 for q = 2; q = 1 is the one-product variant);
 *   5. orthonormalises all vectors (Gram-Schmidt in column order, computed as
 *      Cholesky-QR: S = X^T X = L L^T, X <- X L^{-T});
 *   6. returns Rayleigh quotients as eigenvalues (ascending) and the vectors
 *      rotated back, V = V_prev X.
 *
 * Conventions (LAPACK style, as the paper's "calling interface similar to the
 * standard eigensolvers" suggests): column-major storage with leading
 * dimensions; eigenvectors are columns; eigenvalues ascending; every device
 * pointer refers to memory on the current HIP device; the caller owns every
 * buffer it passes.  The `stream` arguments are hipStream_t values (NULL =
 * the default stream).
 *
 * Errors: the return value reports synchronous argument / resource errors
 * only.  Conditions found on the device are written to *dInfo (int32, device
 * memory, cleared by the call itself):
 *      0  success
 *    k>0  the overlap matrix is not positive definite at column k (the start
 *         vectors do not span: a randomly mixed, non-diagonally-dominant input
 *         as the Methodology section warns, or duplicated previous vectors)
 *     -1  a non-finite eigenvalue (non-finite input propagates to it)
 *     -2  a returned eigenpair's residual ||A v_i - lambda_i v_i|| exceeds the
 *         plan's threshold resid_tol * max_j |lambda_j| (plans with resid_tol > 0)
 *     -3  a submatrix eigensolver did not converge within its sweep limit
 *     -4  an output vector lost its length (squared norm outside [1/4, 4] before
 *         normalisation): V_prev does not have orthonormal columns
 *     -5  generalized -> standard conversion: a diagonal entry of B is not a
 *         positive finite number
 * The first condition found wins.
 */
#ifndef PFSM_H
#define PFSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pfsm_status {
  PFSM_OK = 0,
  PFSM_INVALID_ARG = 1,
  PFSM_NOT_SUPPORTED = 2,
  PFSM_OOM = 3,
  PFSM_HIP_ERROR = 4,
  PFSM_WORKSPACE_TOO_SMALL = 5
} pfsm_status;

typedef enum pfsm_precision {
  PFSM_PREC_FP64 = 0,       /* every product in FP64 on matrix cores */
  PFSM_PREC_MIXED_BF16 = 1  /* products on BF16 matrix cores, FP32 accumulation: the basis change,
                               overlap and back-rotation with every operand split into hi + lo
                               BF16 parts (three products), the folded-spectrum products on plain
                               BF16 operands (one product; see PFSM_FLAG_FS_SPLIT); FP64 for the
                               submatrix eigensolver (its rotation floor 2^-24 of the Gershgorin
                               bound, the unit roundoff of the FP32 start vectors; its pair
                               problems stop after a sweep of rotations below 2^-14) and the final
                               Rayleigh quotients / cluster Rayleigh-Ritz against A (from an
                               FP64-accurate int8 digit product).
                               Orthonormalisation: to first order in S - I while max |S - I| <=
                               1e-3 (a correction product on the matrix cores), otherwise the FP64
                               Cholesky-QR of the overlap, chosen on the device */
} pfsm_precision;

typedef enum pfsm_shift_mode {
  PFSM_SHIFT_FIXED = 0,    /* eps = submatrix eigenvalue, held fixed (Methodology) */
  PFSM_SHIFT_RAYLEIGH = 1  /* eps = Rayleigh quotient refreshed before every iteration */
} pfsm_shift_mode;

/* Plan descriptor.  All pointers are host pointers, read during plan creation only. */
typedef struct pfsm_desc {
  int64_t n;                   /* matrix order, >= 1 */
  int32_t num_parts;           /* number of slices P, 1 <= P <= n */
  const int64_t* part_offsets; /* P+1 ascending slice boundaries, [0] = 0, [P] = n, no empty slice */
  int64_t halo;                /* rows added on each side of a slice to form its submatrix
                                  (order M_p = min(n, m_p + 2 halo)); < 0: half of the largest slice */
  int32_t iterations;          /* folded-spectrum iterations, >= 0 */
  int32_t fs_power;            /* q: 2 (Eq. 11) or 1 */
  double alpha;                /* step length; <= 0: 1 / rho^q, rho = Gershgorin width of At (Eqs. 8-11) */
  int32_t shift_mode;          /* pfsm_shift_mode */
  int32_t precision;           /* pfsm_precision */
  int32_t max_sweeps;          /* submatrix Jacobi sweep limit; <= 0: 10 */
  int32_t flags;               /* PFSM_FLAG_* bits; 0 = defaults */
  double resid_tol;            /* > 0: per-column residuals are computed and info = -2 when
                                  max_i ||A v_i - lambda_i v_i|| > resid_tol * max_j |lambda_j|;
                                  0: no check */
} pfsm_desc;

/* Mixed precision only: skip the FP64 refinement against A and return the
 * eigenvalue estimates of the reduced-precision step (Rayleigh quotients in the
 * rotated basis) -- the "FP32 result" of the mixed path. */
#define PFSM_FLAG_NO_REFINE 1
/* Mixed precision, fs_power 2: run the two products of each folded-spectrum
 * iteration, and the small correction product of the orthonormalisation
 * (X Phi(S - I)^T), on hi/lo split operands (three BF16 products, FP32
 * accumulation) instead of the default plain BF16 operands (one product, FP32
 * accumulation).
 * The FP64 refinement against A removes what the plain products leave: the
 * refined eigenvalues of the two forms agree to 1e-9 of max |lambda| and both
 * stay within 1e-8 of an FP64 computation; only the unrefined estimates
 * (PFSM_FLAG_NO_REFINE) move. */
#define PFSM_FLAG_FS_SPLIT 2
/* Compute the per-column residuals r_i = ||A v_i - lambda_i v_i||_2 of the
 * returned eigenpairs during the solve (read them with pfsm_residuals).  FP64
 * path: from the Rayleigh-quotient product, r_i^2 = ||At x_i||^2 - lambda_i^2;
 * mixed path: from the refinement product Z = A V_new (for the Ritz vectors
 * of a cluster, from y^T (Z_c^T Z_c) y - mu^2).  The difference of squares
 * loses digits for residuals below about 1e-8 |lambda|.  Implied by
 * resid_tol > 0; not available with PFSM_FLAG_NO_REFINE. */
#define PFSM_FLAG_RESIDUALS 4
/* Mixed precision: run the two n x n products of pfsm_backward with V on
 * split-BF16 operands (about 16 significant bits, gradients to about 1e-4
 * relative) instead of the default FP64 products. */
#define PFSM_FLAG_BACKWARD_SPLIT 8

typedef struct pfsm_plan pfsm_plan;

/* Validate the descriptor and build the partition/submatrix tables.
 * Allocates the plan (host) and a small device table on the current device.
 * Errors: INVALID_ARG (bad sizes/offsets/options), HIP_ERROR, OOM. */
pfsm_status pfsm_plan_create(pfsm_plan** plan, const pfsm_desc* desc);

/* Bytes of device workspace pfsm_solve / pfsm_backward need for this plan. */
pfsm_status pfsm_workspace_size(const pfsm_plan* plan, size_t* bytes);

/* One PFSM step (Methodology; Eqs. 3, 11, 12).
 *   dA      n x n symmetric (both triangles read; not symmetrised), lda >= n
 *   dVprev  n x n previous eigenvectors, columns ordered by ascending previous
 *           eigenvalue, ldv >= n
 *   dLambda n eigenvalues out (ascending)
 *   dVout   n x n eigenvectors out, ldvo >= n; must not overlap dA or dVprev
 *   dWork   device workspace of at least pfsm_workspace_size bytes, 256-byte aligned
 *   dInfo   device int32 status word (see above)
 * The call only enqueues work on `stream`: it does not allocate, synchronise
 * or read device memory on the host.  Inputs are not modified.
 * Errors: INVALID_ARG (null pointer, bad leading dimension, aliasing),
 * WORKSPACE_TOO_SMALL, HIP_ERROR (launch failure). */
pfsm_status pfsm_solve(pfsm_plan* plan, const double* dA, int64_t lda, const double* dVprev, int64_t ldv,
                       double* dLambda, double* dVout, int64_t ldvo, void* dWork, size_t work_bytes,
                       int32_t* dInfo, void* stream);

/* Bytes of the library-owned device workspace behind pfsm_solve_static
 * (64 MiB; every GPU the library runs on holds one copy until the process
 * ends). */
#define PFSM_STATIC_SCRATCH_BYTES (64u << 20)

/* pfsm_solve without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * fixed device array of PFSM_STATIC_SCRATCH_BYTES owned by the library, one
 * per device; its address is looked up once per device (at the first plan
 * creation or static solve on it).  Arguments, layout and device info codes
 * as pfsm_solve; the outputs must not overlap the inputs.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (the solve clears what it needs itself): calls that overlap
 * in time on one device -- on different streams or from different threads --
 * race and must be serialised by the caller.
 * Errors: WORKSPACE_TOO_SMALL when pfsm_workspace_size(plan) exceeds
 * PFSM_STATIC_SCRATCH_BYTES (nothing is enqueued; e.g. FP64 plans up to
 * n ~ 1400, mixed-precision plans up to n ~ 800), INVALID_ARG (batched plan,
 * as pfsm_solve), HIP_ERROR. */
pfsm_status pfsm_solve_static(pfsm_plan* plan, const double* dA, int64_t lda, const double* dVprev, int64_t ldv,
                              double* dLambda, double* dVout, int64_t ldvo, int32_t* dInfo, void* stream);

/* Reverse-mode gradient of a symmetric eigendecomposition A = V diag(lambda) V^T
 * (eigen-adjoint: dA = sym(V (diag(gLambda) + F o (V^T gV)) V^T), F_ij =
 * d/(d^2 + eta^2), d = lambda_j - lambda_i, F_ii = 0; the Lorentzian keeps an
 * exactly degenerate pair finite).
 *   dLambda, dV   forward outputs (n, n x n with ldv)
 *   dGradLambda   dL/dlambda (n) or NULL (zero)
 *   dGradV        dL/dV (n x n, ldg) or NULL (zero)
 *   dGradA        output n x n symmetric, ldga >= n; must not overlap the inputs
 * The middle factor is symmetrised in FP64 before the products
 * (M_ij = F_ij (T_ij - T_ji) / 2, T = V^T gV in FP64), so dA = V M V^T; the two
 * n x n products with V run in FP64 (also for a mixed-precision plan, unless
 * it sets PFSM_FLAG_BACKWARD_SPLIT: split-BF16 matrix-core products).
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL, HIP_ERROR. */
pfsm_status pfsm_backward(pfsm_plan* plan, const double* dLambda, const double* dV, int64_t ldv,
                          const double* dGradLambda, const double* dGradV, int64_t ldg, double eta,
                          double* dGradA, int64_t ldga, void* dWork, size_t work_bytes, int32_t* dInfo,
                          void* stream);

/* Batched plans: `count` independent instances (k-points / spins), each with
 * its own descriptor (order, slices, options).  pfsm_workspace_size reports
 * the sum of the instances' workspaces.  Errors as pfsm_plan_create, for the
 * first instance that fails. */
pfsm_status pfsm_plan_create_batched(pfsm_plan** plan, const pfsm_desc* descs, int32_t count);

/* One PFSM step for every instance of a batched plan.  The pointer and
 * leading-dimension arrays are HOST arrays of length count (device pointers
 * inside, read during the call); dInfo points to count device int32 words.
 * The instances are enqueued largest first over internal streams forked from
 * and joined back into `stream` with events, so the call is capturable: a
 * hipStreamBeginCapture / EndCapture around it yields one graph whose
 * branches run the instances concurrently.  Every instance is checked as
 * pfsm_solve checks it, and the outputs of one instance must not overlap the
 * inputs or outputs of another, the info array or the workspace; any such
 * error returns before anything is enqueued.  Errors: INVALID_ARG
 * (non-batched plan, null pointer, bad leading dimension, overlap),
 * WORKSPACE_TOO_SMALL, HIP_ERROR (a failed launch: the internal streams are
 * still joined back into `stream`). */
pfsm_status pfsm_solve_batched(pfsm_plan* plan, const double* const* dA, const int64_t* lda,
                               const double* const* dVprev, const int64_t* ldv, double* const* dLambda,
                               double* const* dVout, const int64_t* ldvo, void* dWork, size_t work_bytes,
                               int32_t* dInfo, void* stream);

/* Copy the per-column residuals of the last solve (output order, n doubles)
 * from the workspace to dR (device) on `stream`.  Errors: INVALID_ARG,
 * NOT_SUPPORTED (the plan does not compute residuals: see
 * PFSM_FLAG_RESIDUALS), WORKSPACE_TOO_SMALL, HIP_ERROR. */
pfsm_status pfsm_residuals(const pfsm_plan* plan, const void* dWork, size_t work_bytes, double* dR, void* stream);

/* Number of instances of a batched plan (0 for a single plan or NULL). */
int32_t pfsm_batch_count(const pfsm_plan* plan);

/* Mixed precision: signed 7-bit digits per operand row in the FP64-accurate
 * refinement product Z = A V_new on the int8 matrix cores (s; the product
 * sums the s (s + 1) / 2 digit products of weight up to s + 1, error about
 * (s + 1) 2^-7s sqrt(n) times the row and column maxima per entry). */
int32_t pfsm_refine_digit_count(void);

/* Tile autotuning of the split-BF16 products (mixed precision): times each
 * tile configuration on an N x N x N product of pseudo-random operands in the
 * plan's workspace (on `stream`, synchronising it) and keeps the fastest in
 * the plan (for a batched plan, per instance).  Choices are remembered per
 * process and order; when the environment variable PFSM_TUNE_CACHE names a
 * file, they are also read from and appended to it as lines
 * "<gfx arch> <HIP runtime version> x3 <n> <cfg> <ms>", and a stored choice
 * for the same architecture, runtime and order is taken without timing.
 * *chosen (nullable) receives the configuration, -1 when nothing was tuned
 * (FP64 plans, batched plans).  The folded-spectrum products on plain
 * operands have a single configuration and are not tuned.  Call it outside
 * any stream capture.  Errors: INVALID_ARG, HIP_ERROR. */
pfsm_status pfsm_autotune(pfsm_plan* plan, void* dWork, size_t work_bytes, int32_t* chosen, void* stream);

/* Fix the split-BF16 tile configuration (-1: library default, 0..5: see
 * pfsm_autotune) for a plan and its instances.  Errors: INVALID_ARG. */
pfsm_status pfsm_set_tile_config(pfsm_plan* plan, int32_t cfg);

/* Release the plan and its device table (synchronises the device first). */
void pfsm_plan_destroy(pfsm_plan* plan);

/* Static string for a status code. */
const char* pfsm_status_string(pfsm_status status);

/* Diagnostics for tests and benchmarks (not part of the method):
 * out[0] = ||A V - V diag(lambda)||_F / ||A||_F, out[1] = ||V^T V - I||_F,
 * computed in FP64 on the device; out is a device array of 2 doubles.
 * Uses the plan's workspace (the result of a previous solve must already be
 * in dLambda / dV, which must not lie inside the workspace). */
pfsm_status pfsm_diagnostics(pfsm_plan* plan, const double* dA, int64_t lda, const double* dLambda,
                             const double* dV, int64_t ldv, double* dOut, void* dWork, size_t work_bytes,
                             void* stream);

/* Stage timing for benchmarks (instrumentation, off by default).
 * pfsm_timing_begin creates max_solves x PFSM_TIMING_BOUNDS HIP events (on the
 * plan's device) and makes the next max_solves calls of pfsm_solve record an
 * event at each stage boundary on their stream.  pfsm_timing_read
 * synchronises those events and writes, for each recorded solve s and stage k,
 * the elapsed milliseconds between boundary k and k+1 to ms[s * (PFSM_TIMING_BOUNDS-1) + k]
 * (unused stages read 0).  Stage order: 0 basis change, 1 step length, 2
 * submatrix eigensolver + start vectors, 3 + 2i shifted product of iteration i,
 * 4 + 2i folded-spectrum update of iteration i (i < iterations, at most 8),
 * 19 overlap, 20 Cholesky-QR, 21 Rayleigh quotients, 22 ordering, 23
 * back-rotation (mixed precision: with the digit split of A and V_new), 24
 * refinement product Z = A V_new (mixed precision, one launch), 25
 * refinement Rayleigh quotients, cluster Rayleigh-Ritz and ordering (mixed
 * precision; the ordering of the unrefined mixed result also falls here).
 * pfsm_timing_end releases the events.
 * Errors: INVALID_ARG, HIP_ERROR. */
#define PFSM_TIMING_BOUNDS 27
/* Internal counters of the last solve (instrumentation; synchronises the
 * device).  out[2p] = sweep at which submatrix p was found converged (0: never),
 * out[2p+1] = pair problems of submatrix p that needed rotations; then, for
 * mixed precision, the number of refinement clusters, of clusters with more
 * than one estimate, the largest cluster, the number of folded-spectrum
 * products that ran in the band form, and 1 if the orthonormalisation
 * correction did (0 otherwise).  *count = 2P + 5.
 * Errors: INVALID_ARG (capacity < 2P + 5), HIP_ERROR. */
pfsm_status pfsm_debug_stats(pfsm_plan* plan, const void* dWork, size_t work_bytes, int32_t* out, int32_t capacity,
                             int32_t* count);
pfsm_status pfsm_timing_begin(pfsm_plan* plan, int32_t max_solves);
pfsm_status pfsm_timing_read(pfsm_plan* plan, float* ms, int32_t capacity, int32_t* solves_recorded);
pfsm_status pfsm_timing_end(pfsm_plan* plan);

/* Generalized -> standard conversion (Implementation section, Eqs. 13-15).
 * For A x = lambda B x with B symmetric positive definite and diagonally
 * dominant (the overlap matrix of ultrasoft pseudopotentials), writes
 * Z = B^{-1} A, reached without forming B^{-1} by `iterations` steps of
 * Z_{k+1} = (I - D^{-1} B) Z_k + D^{-1} A, D = diag(B), from Z_0 = A (the
 * identity as the initial approximation of B^{-1}).  The steps converge when
 * the spectral radius of I - D^{-1} B is below one; each costs one FP64
 * matrix-core product (2 n^3 flop) and the columns of Z are independent.
 *   dA, dB: n x n column-major (lda, ldb >= n), read only; B must be symmetric
 *     (the product is formed as B^T Z).
 *   dZ: n x n output (ldz >= n); must not overlap A, B or the workspace.
 *   dWork: >= pfsm_g2s_workspace_size(n) bytes, 256-byte aligned, caller-owned.
 *   dResidual (nullable, device, `iterations` doubles): entry k receives
 *     ||A - B Z_k||_F / ||A||_F, the residual of the iterate step k starts from.
 *   dInfo (device int32, cleared by the call): -5 when a diagonal entry of B is
 *     not a positive finite number, -1 when a residual is not finite.
 * Enqueued on `stream` with no allocation and no synchronisation.
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL, HIP_ERROR. */
pfsm_status pfsm_g2s_workspace_size(int64_t n, size_t* bytes);
pfsm_status pfsm_generalized_to_standard(int64_t n, const double* dA, int64_t lda, const double* dB, int64_t ldb,
                                         int32_t iterations, double* dZ, int64_t ldz, void* dWork,
                                         size_t work_bytes, double* dResidual, int32_t* dInfo, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PFSM_H */
