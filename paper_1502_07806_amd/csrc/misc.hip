// Bandwidth-bound helper kernels of the PFSM step: Gershgorin interval and
// step length, Rayleigh-quotient reduction, sign convention + stable ordering
// + column permutation, the eigen-adjoint middle factor, symmetrisation and
// diagnostic norms.  One workgroup per column wherever a column is reduced,
// so every read is a contiguous column segment.
#include "common.h"
#include "misc.h"
#include "order_key.h"
#include <cfloat>

namespace pfsm {
namespace {

constexpr int NT = 256;

__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) t += sh[w];  // fixed order: deterministic
  return t;
}

__global__ void k_fill_i32(int* p, int64_t count, int value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Column j of the symmetric At: radius sum_{i != j} |At_ij| (= row radius by symmetry).
template <typename T>
__global__ __launch_bounds__(NT) void k_gersh_col(const T* At, int64_t n, int64_t ld, double* lo, double* hi) {
  __shared__ double sh[NT / 64];
  const int64_t j = blockIdx.x;
  const T* c = At + j * ld;
  double s = 0.0;
  // unrolled: eight loads in flight per thread; the sum keeps its order
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += NT) s += fabs((double)c[i]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    double d = (double)c[j];
    double r = s - fabs(d);
    lo[j] = d - r;
    hi[j] = d + r;
  }
}

__global__ __launch_bounds__(NT) void k_gersh_final(const double* lo, const double* hi, int64_t n, int q,
                                                     double user_alpha, double* scal, int* info) {
  __shared__ double slo[NT], shi[NT], srad[NT];
  double a = DBL_MAX, b = -DBL_MAX, rad = 0.0;  // rad: largest off-diagonal absolute row sum
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    double x = lo[i], y = hi[i];
    a = (x != x) ? x : fmin(a, x);  // keep NaN visible (fmin would drop it)
    b = (y != y) ? y : fmax(b, y);
    rad = fmax(rad, 0.5 * (y - x));
    if (a != a || b != b) { a = b = rad = __builtin_nan(""); break; }
  }
  slo[threadIdx.x] = a;
  shi[threadIdx.x] = b;
  srad[threadIdx.x] = rad;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double a2 = slo[threadIdx.x + w], b2 = shi[threadIdx.x + w], r2 = srad[threadIdx.x + w];
      slo[threadIdx.x] = (a2 != a2) ? a2 : fmin(slo[threadIdx.x], a2);
      shi[threadIdx.x] = (b2 != b2) ? b2 : fmax(shi[threadIdx.x], b2);
      srad[threadIdx.x] = (r2 != r2) ? r2 : fmax(srad[threadIdx.x], r2);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double rho = shi[0] - slo[0];
    double alpha;
    if (user_alpha > 0.0) alpha = user_alpha;
    else alpha = rho > 0.0 ? 1.0 / (q == 2 ? rho * rho : rho) : 0.0;
    scal[0] = alpha;
    scal[1] = slo[0];
    scal[2] = shi[0];
    scal[3] = srad[0];
    // dropped-term limit of the folded-spectrum products' band form
    scal[4] = PFSM_BAND_TOL * fmax(fabs(slo[0]), fabs(shi[0]));
    // A non-finite entry of A or V_prev spreads over every entry of At.
    if (info && !(isfinite(slo[0]) && isfinite(shi[0]))) atomicCAS(info, 0, -1);
  }
}

__global__ void k_rq_reduce(const double* part, int tiles_m, int64_t n, const double* den, double* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int t = 0; t < tiles_m; ++t) s += part[(int64_t)t * n + j];
  if (den) s /= den[j];
  out[j] = s;
}

__global__ __launch_bounds__(NT) void k_col_norm2(const double* X, int64_t m, int64_t ldx, double* out) {
  __shared__ double sh[NT / 64];
  const int64_t j = blockIdx.x;
  const double* c = X + j * ldx;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += NT) s += c[i] * c[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// Sign convention: the largest-magnitude entry of each column is positive
// (ties: lowest row).  One workgroup per column.
__global__ __launch_bounds__(NT) void k_col_sign(const double* X, int64_t n, int64_t ldx, double* sgn) {
  __shared__ double sv[NT];
  __shared__ int64_t si[NT];
  const int64_t j = blockIdx.x;
  const double* c = X + j * ldx;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    double a = fabs(c[i]);
    if (a > best) { best = a; bi = i; }  // strided scan: first maximum per thread
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double a = sv[threadIdx.x + w];
      int64_t ai = si[threadIdx.x + w];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sgn[j] = (c[si[0]] < 0.0) ? -1.0 : 1.0;
}

// Stable ascending rank of v_j = num_j (or num_j / den_j): the number of
// values ordered before it in the NaN-safe total order (ties by index), a
// permutation of 0..n-1 for any input.  The comparison range is split over
// gridDim.y slices whose partial counts are added atomically into rank
// (cleared beforehand), so the O(n^2) comparisons spread over the chip.
__global__ __launch_bounds__(NT) void k_rank_count(const double* num, const double* den, int64_t n, int* rank) {
  __shared__ double tile[NT];
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  const double lj = j < n ? (den ? num[j] / den[j] : num[j]) : 0.0;
  const int64_t chunk = (n + gridDim.y - 1) / gridDim.y;
  const int64_t lo = (int64_t)blockIdx.y * chunk, hi = min<int64_t>(n, lo + chunk);
  int r = 0;
  for (int64_t base = lo; base < hi; base += NT) {
    __syncthreads();
    const int64_t k = base + threadIdx.x;
    if (k < hi) tile[threadIdx.x] = den ? num[k] / den[k] : num[k];
    __syncthreads();
    const int cnt = (int)min<int64_t>(NT, hi - base);
    for (int t = 0; t < cnt; ++t) r += order_before(tile[t], base + t, lj, j);
  }
  if (j < n && r) atomicAdd(&rank[j], r);
}

__global__ __launch_bounds__(NT) void k_rank_place(const double* lam, int64_t n, const int* rank, double* lam_out,
                                                   int* info) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  const double lj = lam[j];
  if (!isfinite(lj)) atomicCAS(info, 0, -1);
  lam_out[rank[j]] = lj;
}

__global__ __launch_bounds__(NT) void k_permute(const double* X, int64_t n, int64_t ldx, const int* rank,
                                                  const double* sgn, double* Xp, int64_t ldxp) {
  const int64_t j = blockIdx.x;
  const double s = sgn[j];
  const double* src = X + j * ldx;
  double* dst = Xp + (int64_t)rank[j] * ldxp;
  for (int64_t i = threadIdx.x; i < n; i += NT) dst[i] = s * src[i];
}

// M = sym(diag(glam) + F o T) with F_ij = d / (d^2 + eta^2), d = lam_j - lam_i,
// F_ii = 0: since F is antisymmetric, M_ij = F_ij (T_ij - T_ji) / 2 off the
// diagonal and M_ii = glam_i.  Symmetrising here, in FP64, removes the large
// antisymmetric part of F o T (which V (.) V^T would only cancel in exact
// arithmetic) before the products.  One 32 x 32 tile pair per workgroup.
__global__ void k_adjoint_middle(double* T, int64_t ldt, int64_t n, const double* lam, const double* glam,
                                 double eta, int have_t) {
  __shared__ double a[32][33], b[32][33];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int64_t gi = bi * 32 + tx, gj = bj * 32 + r;
    a[r][tx] = (have_t && gi < n && gj < n) ? T[gi + gj * ldt] : 0.0;   // a[c][r'] = T(bi*32 + r', bj*32 + c)
    int64_t hi = bj * 32 + tx, hj = bi * 32 + r;
    b[r][tx] = (have_t && hi < n && hj < n) ? T[hi + hj * ldt] : 0.0;   // b[c][r'] = T(bj*32 + r', bi*32 + c)
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t gi = bi * 32 + tx, gj = bj * 32 + r;  // element (gi, gj), gi row
    if (gi < n && gj < n) {
      double v;
      if (gi == gj) {
        v = glam ? glam[gi] : 0.0;
      } else {
        const double d = lam[gj] - lam[gi];
        const double f = d / (d * d + eta * eta);
        v = 0.5 * f * (a[r][tx] - b[tx][r]);  // (T_ij - T_ji) F_ij / 2
      }
      T[gi + gj * ldt] = v;
      if (bi != bj) T[gj + gi * ldt] = v;
    }
  }
}

// C <- (C + C^T) / 2, tile-pair at a time through LDS.
__global__ void k_symmetrize(double* C, int64_t n, int64_t ldc) {
  __shared__ double a[32][33], b[32][33];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int64_t gi = bi * 32 + tx, gj = bj * 32 + r;
    a[r][tx] = (gi < n && gj < n) ? C[gi + gj * ldc] : 0.0;   // a[c][r] = C(bi*32+r', bj*32+c')
    int64_t hi = bj * 32 + tx, hj = bi * 32 + r;
    b[r][tx] = (hi < n && hj < n) ? C[hi + hj * ldc] : 0.0;
  }
  __syncthreads();
  // a[c][r] holds C(bi*32 + r, bj*32 + c); b[c][r] holds C(bj*32 + r, bi*32 + c)
  for (int r = ty; r < 32; r += 8) {
    int64_t gi = bi * 32 + tx, gj = bj * 32 + r;
    double v = 0.5 * (a[r][tx] + b[tx][r]);
    if (gi < n && gj < n) C[gi + gj * ldc] = v;
  }
  if (bi != bj) {
    for (int r = ty; r < 32; r += 8) {
      int64_t hi = bj * 32 + tx, hj = bi * 32 + r;
      double v = 0.5 * (b[r][tx] + a[tx][r]);
      if (hi < n && hj < n) C[hi + hj * ldc] = v;
    }
  }
}

__global__ void k_mirror_lower(double* C, int64_t n, int64_t ldc) {
  __shared__ double a[32][33];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;  // destination tile (bi < bj: strictly upper)
  if (bi > bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // read source tile (bj, bi) (lower) coalesced
  for (int r = ty; r < 32; r += 8) {
    int64_t gi = bj * 32 + tx, gj = bi * 32 + r;
    a[r][tx] = (gi < n && gj < n) ? C[gi + gj * ldc] : 0.0;  // a[c][r] = C(bj*32 + r, bi*32 + c)
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int64_t gi = bi * 32 + tx, gj = bj * 32 + r;  // destination (row gi, col gj) = C(gj, gi)
    if (gi < n && gj < n && gi < gj) C[gi + gj * ldc] = a[tx][r];
  }
}

__global__ void k_scale_cols(const double* V, int64_t n, int64_t ldv, const double* d, double* out, int64_t ldo) {
  const int64_t j = blockIdx.y;
  const double s = d ? d[j] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i + j * ldo] = s * V[i + j * ldv];
}

// Column partial sums for the diagnostics: part[0][j] = ||AV_j - lam_j V_j||^2,
// part[1][j] = ||A_j||^2, part[2][j] = ||G_j - e_j||^2 (G = V^T V).
__global__ __launch_bounds__(NT) void k_diag_cols(const double* A, int64_t lda, const double* AV, int64_t ldav,
                                                   const double* V, int64_t ldv, const double* lam, const double* G,
                                                   int64_t ldg, int64_t n, double* part) {
  __shared__ double sh[NT / 64];
  const int64_t j = blockIdx.x;
  const double lj = lam[j];
  double r = 0.0, a = 0.0, o = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    double t = AV[i + j * ldav] - lj * V[i + j * ldv];
    r += t * t;
    double x = A[i + j * lda];
    a += x * x;
    double g = G[i + j * ldg] - (i == j ? 1.0 : 0.0);
    o += g * g;
  }
  r = block_sum(r, sh);
  a = block_sum(a, sh);
  o = block_sum(o, sh);
  if (threadIdx.x == 0) {
    part[j] = r;
    part[n + j] = a;
    part[2 * n + j] = o;
  }
}

__global__ __launch_bounds__(NT) void k_diag_final(const double* part, int64_t n, double* out) {
  __shared__ double sh[NT / 64];
  double r = 0.0, a = 0.0, o = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    r += part[i];
    a += part[n + i];
    o += part[2 * n + i];
  }
  r = block_sum(r, sh);
  a = block_sum(a, sh);
  o = block_sum(o, sh);
  if (threadIdx.x == 0) {
    out[0] = sqrt(r) / sqrt(a);
    out[1] = sqrt(o);
  }
}

__global__ void k_norm_check(const double* nn, int64_t n, int* info) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double v = nn[j];
  if (!(v >= 0.25 && v <= 4.0)) atomicCAS(info, 0, PFSM_INFO_BASIS);
}

}  // namespace

hipError_t norm_check(const double* nn, int64_t n, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nn, n, info);
  return hipGetLastError();
}

// Deterministic pseudo-random values in [-1, 1) (a 32-bit integer hash of the
// index and seed), for timing products on realistic, non-zero operands.
__global__ void k_fill_hash_f32(float* y, int64_t count, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(i >> 32) ^ seed;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    y[i] = (float)((double)h * (2.0 / 4294967296.0) - 1.0);
  }
}

hipError_t fill_hash_f32(float* y, int64_t count, uint32_t seed, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_hash_f32, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 4096)), dim3(256), 0, s, y,
                     count, seed);
  return hipGetLastError();
}

__global__ void k_zero_krange_rows(float* X, int64_t ldx, int64_t m, const int32_t* krange, int64_t tile_n) {
  const int64_t c = blockIdx.x;
  const int64_t t = c / tile_n;
  const int64_t r0 = krange[2 * t], r1 = min<int64_t>(krange[2 * t + 1], m);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) X[r + c * ldx] = 0.0f;
}

hipError_t zero_krange_rows(float* X, int64_t ldx, int64_t m, int64_t n, const int32_t* krange, int64_t tile_n,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_krange_rows, dim3((unsigned)n), dim3(256), 0, s, X, ldx, m, krange, tile_n);
  return hipGetLastError();
}

hipError_t fill_i32(int* p, int64_t count, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 1024))),
                     dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t mirror_lower(double* C, int64_t n, int64_t ldc, hipStream_t s) {
  unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_mirror_lower, dim3(t, t), dim3(256), 0, s, C, n, ldc);
  return hipGetLastError();
}

template <typename T>
static hipError_t gershgorin_alpha_t(const T* At, int64_t n, int64_t ld, int q, double user_alpha, double* part_lo,
                                     double* part_hi, double* scal, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_gersh_col<T>, dim3((unsigned)n), dim3(NT), 0, s, At, n, ld, part_lo, part_hi);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(NT), 0, s, part_lo, part_hi, n, q, user_alpha, scal, info);
  return hipGetLastError();
}
hipError_t gershgorin_alpha(const double* At, int64_t n, int64_t ld, int q, double user_alpha, double* part_lo,
                            double* part_hi, double* scal, int* info, hipStream_t s) {
  return gershgorin_alpha_t(At, n, ld, q, user_alpha, part_lo, part_hi, scal, info, s);
}
hipError_t gershgorin_alpha(const float* At, int64_t n, int64_t ld, int q, double user_alpha, double* part_lo,
                            double* part_hi, double* scal, int* info, hipStream_t s) {
  return gershgorin_alpha_t(At, n, ld, q, user_alpha, part_lo, part_hi, scal, info, s);
}

hipError_t rq_reduce(const double* part, int tiles_m, int64_t n, const double* den, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rq_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, tiles_m, n, den, out);
  return hipGetLastError();
}

hipError_t col_norm2(const double* X, int64_t m, int64_t n, int64_t ldx, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_col_norm2, dim3((unsigned)n), dim3(NT), 0, s, X, m, ldx, out);
  return hipGetLastError();
}

hipError_t finalize_order(const double* lam_u, const double* X, int64_t n, int64_t ldx, double* Xp, int64_t ldxp,
                          double* lam_out, int* rank, double* sgn, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_col_sign, dim3((unsigned)n), dim3(NT), 0, s, X, n, ldx, sgn);
  hipError_t e = finalize_order_values(lam_u, n, lam_out, rank, info, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)n), dim3(NT), 0, s, X, n, ldx, rank, sgn, Xp, ldxp);
  return hipGetLastError();
}

hipError_t rank_ascending(const double* num, const double* den, int64_t n, int* rank, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipError_t e = fill_i32(rank, n, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_count, dim3((unsigned)((n + NT - 1) / NT), 16), dim3(NT), 0, s, num, den, n, rank);
  return hipGetLastError();
}

hipError_t finalize_order_values(const double* lam_u, int64_t n, double* lam_out, int* rank, int* info, hipStream_t s) {
  hipError_t e = rank_ascending(lam_u, nullptr, n, rank, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_place, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, lam_u, n, rank, lam_out, info);
  return hipGetLastError();
}

hipError_t adjoint_middle(double* T, int64_t ldt, int64_t n, const double* lam, const double* glam, double eta,
                          bool have_t, hipStream_t s) {
  unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_adjoint_middle, dim3(t, t), dim3(256), 0, s, T, ldt, n, lam, glam, eta, have_t ? 1 : 0);
  return hipGetLastError();
}

hipError_t symmetrize(double* C, int64_t n, int64_t ldc, hipStream_t s) {
  unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_symmetrize, dim3(t, t), dim3(256), 0, s, C, n, ldc);
  return hipGetLastError();
}

hipError_t scale_cols(const double* V, int64_t n, int64_t ldv, const double* d, double* out, int64_t ldo,
                      hipStream_t s) {
  dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 64), (unsigned)n);
  hipLaunchKernelGGL(k_scale_cols, grid, dim3(256), 0, s, V, n, ldv, d, out, ldo);
  return hipGetLastError();
}

hipError_t diag_sums(const double* A, int64_t lda, const double* AV, int64_t ldav, const double* V, int64_t ldv,
                     const double* lam, const double* G, int64_t ldg, int64_t n, double* part, double* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_diag_cols, dim3((unsigned)n), dim3(NT), 0, s, A, lda, AV, ldav, V, ldv, lam, G, ldg, n, part);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(NT), 0, s, part, n, out);
  return hipGetLastError();
}

}  // namespace pfsm
