// Test hooks: C entry points to internal kernels for kernel-level parity tests
// and microbenchmarks.  Linked only into libpfsm_testhooks.so, never into the
// product library libpfsm.so.
#include "../common.h"
#include "../gemm_x3.h"
#include "../chol.h"
#include "../gemm_oz.h"
#include "../refine.h"

using namespace pfsm;

static hipError_t ensure_x3() {
  static bool init = false;
  if (!init) {
    const hipError_t e = x3_init();
    if (e != hipSuccess) return e;
    init = true;
  }
  return hipSuccess;
}

extern "C" {

int pfsm_test_gemm_f64(int ta, int tb, int epi, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                       const double* eps, const double* D, int64_t ldd, double* part, int lower_only, void* stream) {
  GemmArgs g = {};
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.eps = eps; g.D = D; g.ldd = ldd; g.part = part; g.lower_only = lower_only;
  return (int)gemm_f64(ta != 0, tb != 0, epi, g, (hipStream_t)stream);
}

int pfsm_test_pack_x3(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, void* P,
                      int64_t ldp, void* stream) {
  return (int)pack_x3(X, src_double, m, n, ldx, flags, (bf16_t*)P, ldp, (hipStream_t)stream);
}

// The band part (far = 0) or the gated far part (far = 1) of a pack (pack_x3_band, pack_x3_far_gated).
int pfsm_test_pack_x3_part(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, void* P,
                           int64_t ldp, const int32_t* krange, int band_chunks, int far, const unsigned* gate_far,
                           const double* gate_cl, void* stream) {
  if (far)
    return (int)pack_x3_far_gated(X, src_double, m, n, ldx, flags, (bf16_t*)P, ldp, krange, gate_far, gate_cl,
                                  (hipStream_t)stream);
  return (int)pack_x3_band(X, src_double, m, n, ldx, flags, (bf16_t*)P, ldp, krange, band_chunks, (hipStream_t)stream);
}

int pfsm_test_gemm_x3_ws(int epi, int cfg, int tiles, int64_t M, int64_t N, int64_t K, const void* Ap, int64_t ldap,
                         const void* Bp, int64_t ldbp, void* C, int64_t ldc, int c_double, double alpha, double beta,
                         const float* B32, int64_t ldb32, const void* D, int64_t ldd, int d_double, const double* eps,
                         double* part, void* split_ws, size_t split_bytes, void* stream) {
  X3Args g = {};
  g.M = M; g.N = N; g.K = K; g.Ap = (const bf16_t*)Ap; g.ldap = ldap; g.Bp = (const bf16_t*)Bp; g.ldbp = ldbp;
  g.C = C; g.ldc = ldc; g.c_double = c_double; g.alpha = alpha; g.beta = beta; g.B32 = B32; g.ldb32 = ldb32;
  g.D = D; g.ldd = ldd; g.d_double = d_double; g.eps = eps; g.part = part; g.tiles = tiles; g.cfg = cfg;
  g.split_ws = (float*)split_ws; g.split_bytes = split_bytes;
  const hipError_t e = ensure_x3();
  if (e != hipSuccess) return (int)e;
  return (int)gemm_x3(epi, g, (hipStream_t)stream);
}

int pfsm_test_gemm_x3(int epi, int cfg, int tiles, int64_t M, int64_t N, int64_t K, const void* Ap, int64_t ldap,
                      const void* Bp, int64_t ldbp, void* C, int64_t ldc, int c_double, double alpha, double beta,
                      const float* B32, int64_t ldb32, const void* D, int64_t ldd, int d_double, const double* eps,
                      double* part, void* stream) {
  return pfsm_test_gemm_x3_ws(epi, cfg, tiles, M, N, K, Ap, ldap, Bp, ldbp, C, ldc, c_double, alpha, beta, B32, ldb32,
                              D, ldd, d_double, eps, part, nullptr, 0, stream);
}

// SHIFT / FSUPD / ADD product (FP32 C and D) with `products` BF16 products: 3
// from split operands, 1 from plain operands (row strides ldap / ldbp in bf16
// elements); tiles as in X3Args.
int pfsm_test_gemm_x3_fs(int epi, int products, int tiles, int64_t M, int64_t N, int64_t K, const void* Ap,
                         int64_t ldap, const void* Bp, int64_t ldbp, float* C, int64_t ldc, const float* B32,
                         int64_t ldb32, const float* D, int64_t ldd, const double* eps, double alpha, void* stream) {
  X3Args g = {};
  g.tiles = tiles;
  g.M = M; g.N = N; g.K = K; g.Ap = (const bf16_t*)Ap; g.ldap = ldap; g.Bp = (const bf16_t*)Bp; g.ldbp = ldbp;
  g.C = C; g.ldc = ldc; g.c_double = 0; g.alpha = alpha; g.B32 = B32; g.ldb32 = ldb32; g.D = D; g.ldd = ldd;
  g.eps = eps; g.cfg = -1; g.products = products;
  const hipError_t e = ensure_x3();
  if (e != hipSuccess) return (int)e;
  return (int)gemm_x3(epi, g, (hipStream_t)stream);
}

int64_t pfsm_test_x3_plain_stride(int64_t K) { return x3_plain_stride(K); }

// K-split scratch bytes for an order-n lower-triangle product (0: no split).
int64_t pfsm_test_x3_split_bytes(int64_t n) {
  if (ensure_x3() != hipSuccess) return -1;
  return (int64_t)x3_split_bytes(n);
}

int64_t pfsm_test_x3_row_stride(int64_t K) { return x3_row_stride(K); }

int pfsm_test_cholesky(double* S, int64_t lds, int64_t n, double* Tbuf, int* info, void* stream) {
  return (int)cholesky_factor(S, lds, n, Tbuf, info, (hipStream_t)stream);
}

int pfsm_test_trsm(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t n, int64_t m, const double* Tbuf,
                   void* stream) {
  return (int)trsm_right_lt(L, ldl, X, ldx, n, m, Tbuf, (hipStream_t)stream);
}

int pfsm_test_cholesky_qr_gated(double* S, int64_t lds, double* X, int64_t ldx, int64_t n, int64_t m, double* Tbuf,
                                double* Bcopy, int* info, const int* gate, void* stream) {
  return (int)cholesky_qr_gated(S, lds, X, ldx, n, m, Tbuf, Bcopy, info, gate, (hipStream_t)stream);
}

int pfsm_test_convert_gated(void* X32, int64_t ld32, double* X64, int64_t ld64, int64_t m, int64_t n, int to_f64,
                            const int* gate, void* stream) {
  return (int)convert_f32_f64_gated((const float*)X32, ld32, X64, ld64, m, n, to_f64, gate, (hipStream_t)stream);
}

int pfsm_test_oz_split(const double* X, int64_t ldx, int64_t K, int64_t ncols, int s, void* P, int* expo, int* info,
                       void* stream) {
  return (int)oz_split(X, ldx, K, ncols, s, (int8_t*)P, expo, info, (hipStream_t)stream);
}

int pfsm_test_gemm_oz(int64_t M, int64_t N, int64_t K, int s, const void* Ap, const int* ea, const void* Bp,
                      const int* eb, double* C, int64_t ldc, int cfg, void* stream) {
  static bool init = false;
  if (!init) {
    const hipError_t e = oz_init();
    if (e != hipSuccess) return (int)e;
    init = true;
  }
  return (int)gemm_oz(M, N, K, s, (const int8_t*)Ap, ea, (const int8_t*)Bp, eb, C, ldc, (hipStream_t)stream, cfg);
}

int64_t pfsm_test_oz_row_stride(int64_t K) { return oz_row_stride(K); }

int64_t pfsm_test_oz_plane_bytes(int64_t n, int s) { return (int64_t)oz_plane_bytes(n, n, s); }
int pfsm_test_refine_slices() { return REFINE_OZ_SLICES; }
double pfsm_test_refine_tau() { return REFINE_TAU; }
int pfsm_test_refine_kmax() { return REFINE_KMAX; }

// The mixed path's refinement on given FP64 estimates V (n x n, ldv): digits
// of A and V, Z = A V on the int8 matrix cores, then refine_rr.  planes:
// 2 * pfsm_test_oz_plane_bytes(n, s) bytes; expo: 2n ints; Z: n x n doubles
// (ld n); rb: 7n + 8 doubles.
int pfsm_test_refine(int64_t n, const double* A, int64_t lda, const double* V, int64_t ldv, void* planes, int* expo,
                     double* Z, double* rb, double* lam, double* Vout, int64_t ldvo, int* info, void* stream) {
  static bool init = false;
  if (!init) {
    const hipError_t e = oz_init();
    if (e != hipSuccess) return (int)e;
    init = true;
  }
  hipStream_t st = (hipStream_t)stream;
  const int s = REFINE_OZ_SLICES;
  int8_t* pA = (int8_t*)planes;
  int8_t* pV = pA + oz_plane_bytes(n, n, s);
  hipError_t e = oz_split(A, lda, n, n, s, pA, expo, info, st);
  if (e == hipSuccess) e = oz_split(V, ldv, n, n, s, pV, expo + n, info, st);
  if (e == hipSuccess) e = gemm_oz(n, n, n, s, pA, expo, pV, expo + n, Z, n, st);
  if (e != hipSuccess) return (int)e;
  RefineBufs b;
  b.d = rb; b.nn = rb + n; b.lam_s = rb + 2 * n;
  b.rank = (int*)(rb + 3 * n); b.inv = (int*)(rb + 4 * n); b.cstart = (int*)(rb + 5 * n);
  b.csize = (int*)(rb + 6 * n); b.clus = (int*)(rb + 7 * n);
  return (int)refine_rr(V, ldv, Z, n, n, REFINE_TAU, lam, Vout, ldvo, b, info, st);
}

}  // extern "C"
