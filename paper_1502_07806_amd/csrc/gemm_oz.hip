// Int8 digit GEMM (see gemm_oz.h).  Block tile 256 x 256 x 128 (k bytes),
// 256 threads = 4 waves in 2 x 2, wave tile 128 x 128 = 4 x 4 blocks of
// v_mfma_i32_32x32x32_i8: one wave per SIMD with 256 int32 accumulators per
// lane, 8 fragment reads per 16 MFMAs (half the LDS rate).  Operand tiles go
// global -> registers -> LDS, double buffered, 144-byte rows so that the
// 16-byte fragment reads of consecutive rows fall in distinct banks.  The
// MFMA takes the B fragment first, so a lane's accumulators run along a row
// of C and one register across lanes runs down a column (contiguous
// column-major stores).  The k loop of one launch walks every digit pair
// (p, q) of one weight group back to back: the int32 sum of the group is
// exact, and the epilogue scales it by its power of two into FP64.
#include "common.h"
#include "gemm_oz.h"

namespace pfsm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BM = OZ_BM, BN = OZ_BN, BK = OZ_BK;
constexpr int NT = 256;
constexpr int ROWB = BK + 16;        // LDS bytes per operand row
constexpr int TILE = BM * ROWB;      // 36864 bytes per operand per stage
constexpr int WR = 4, WC = 4;        // 32 x 32 blocks per wave
constexpr int LQ = BM * (BK / 16) / NT;  // 16-byte chunks per thread and operand (8)

struct OzArgs {
  int64_t M, N, ldp, pa, pb;  // ldp: digit-row stride; pa / pb: plane strides (bytes)
  const int8_t* Ap;
  const int8_t* Bp;
  const int* ea;
  const int* eb;
  double* C;
  int64_t ldc;
  int g, first, s, ntk;       // weight group p + q, store or add, slices, k tiles per pair
};

__device__ inline int xcd_remap(int b, int total) {
  // consecutive tiles to one XCD (blocks are dealt to the 8 XCDs round robin)
  if (total % 8 != 0) return b;
  return (b % 8) * (total / 8) + b / 8;
}

__global__ __launch_bounds__(NT, 1) void gemm_oz_kernel(OzArgs a, int tiles_m, int tiles_n) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  unsigned char* As = lds;              // [2][BM][ROWB]
  unsigned char* Bs = lds + 2 * TILE;   // [2][BN][ROWB]
  int tm, tn;
  {
    const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int GROUP = 4;  // row tiles sharing the streamed column tiles
    const int first_m = (t / (GROUP * tiles_n)) * GROUP;
    const int gsz = min(tiles_m - first_m, GROUP);
    tm = first_m + (t % (GROUP * tiles_n)) % gsz;
    tn = (t % (GROUP * tiles_n)) / gsz;
  }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi0 = (wave & 1) * (32 * WR), wj0 = (wave >> 1) * (32 * WC);
  const int l32 = lane & 31, lh = lane >> 5;
  // digit pairs of the group: p + q = g with 1 <= p, q <= s
  const int p_lo = max(1, a.g - a.s);
  const int p_hi = min(a.s, a.g - 1);
  const int total = (p_hi - p_lo + 1) * a.ntk;

  v16i acc[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

  const int chunk = tid & 7, rbase = tid >> 3;  // rows rbase + 32 q
  v4i ra[LQ], rb[LQ];
  auto load_tile = [&](int t) {
    const int pair = t / a.ntk, kt = t - pair * a.ntk;
    const int p = p_lo + pair, q = a.g - p;
    const int8_t* A = a.Ap + (int64_t)(p - 1) * a.pa + (int64_t)kt * BK + chunk * 16;
    const int8_t* B = a.Bp + (int64_t)(q - 1) * a.pb + (int64_t)kt * BK + chunk * 16;
    const v4i z = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < LQ; ++u) {
      const int r = rbase + (NT / 8) * u;
      const int64_t gi = m0 + r, gj = n0 + r;
      ra[u] = (gi < a.M) ? *(const v4i*)(A + gi * a.ldp) : z;
      rb[u] = (gj < a.N) ? *(const v4i*)(B + gj * a.ldp) : z;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int u = 0; u < LQ; ++u) {
      const int r = rbase + (NT / 8) * u;
      *(v4i*)(As + buf * TILE + r * ROWB + chunk * 16) = ra[u];
      *(v4i*)(Bs + buf * TILE + r * ROWB + chunk * 16) = rb[u];
    }
  };

  if (total > 0) {
    load_tile(0);
    store_tile(0);
    __syncthreads();
    for (int t = 0; t < total; ++t) {
      const int cur = t & 1;
      if (t + 1 < total) load_tile(t + 1);
      const unsigned char* Ab = As + cur * TILE;
      const unsigned char* Bb = Bs + cur * TILE;
#pragma unroll
      for (int sub = 0; sub < BK / 32; ++sub) {
        const int koff = 32 * sub + 16 * lh;  // this lane's 16 k bytes
        v4i af[WR], bf[WC];
#pragma unroll
        for (int ib = 0; ib < WR; ++ib) af[ib] = *(const v4i*)(Ab + (wi0 + ib * 32 + l32) * ROWB + koff);
#pragma unroll
        for (int jb = 0; jb < WC; ++jb) bf[jb] = *(const v4i*)(Bb + (wj0 + jb * 32 + l32) * ROWB + koff);
#pragma unroll
        for (int ib = 0; ib < WR; ++ib)
#pragma unroll
          for (int jb = 0; jb < WC; ++jb)
            acc[ib][jb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[jb], af[ib], acc[ib][jb], 0, 0, 0);
      }
      if (t + 1 < total) store_tile(cur ^ 1);
      __syncthreads();
    }
  }

  // acc[ib][jb][r] is the group sum for C(i, j), i = wi0 + 32 ib + lane % 32,
  // j = wj0 + 32 jb + 8 (r / 4) + 4 (lane / 32) + r % 4.
  const int shift = -12 - 7 * (a.g - 2);
#pragma unroll
  for (int ib = 0; ib < WR; ++ib) {
    const int64_t gi = m0 + wi0 + ib * 32 + l32;
    if (gi >= a.M) continue;
    const int ei = a.ea[gi] + shift;
#pragma unroll
    for (int jb = 0; jb < WC; ++jb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gj = n0 + wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
        if (gj >= a.N) continue;
        const double v = ldexp((double)acc[ib][jb][r], ei + a.eb[gj]);
        double* cp = a.C + gi + gj * a.ldc;
        *cp = a.first ? v : *cp + v;
      }
  }
}

// One block per column: exponent of the column maximum, then the digits of
// four consecutive k per thread (one 32-bit word per plane).
__global__ __launch_bounds__(256) void k_oz_split(const double* X, int64_t ldx, int64_t K, int64_t ldp,
                                                  int64_t pstride, int s, int8_t* P, int* expo, int* info) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x;
  const double* x = X + c * ldx;
  const int tid = threadIdx.x;
  double m = 0.0;
  for (int64_t k = tid; k < K; k += 256) {
    const double v = fabs(x[k]);
    m = (v > m || v != v) ? v : m;
  }
  sh[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      const double o = sh[tid + w];
      sh[tid] = (o > sh[tid] || o != o) ? o : sh[tid];
    }
    __syncthreads();
  }
  const double mx = sh[0];
  const bool bad = !(mx <= 1.7976931348623157e308);  // NaN or infinity
  int e = 0;
  if (!bad && mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [1/2, 1): |x| 2^-e < 1
  if (tid == 0) {
    expo[c] = e;
    if (bad) atomicCAS(info, 0, -1);
  }
  int8_t* out = P + c * ldp;
  for (int64_t k4 = 4 * (int64_t)tid; k4 < ldp; k4 += 4 * 256) {
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = (!bad && k4 + u < K) ? ldexp(x[k4 + u], 6 - e) : 0.0;  // |t| < 64
    for (int p = 0; p < s; ++p) {
      uint32_t word = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double d = rint(t[u]);  // |d| <= 64, |t - d| <= 1/2
        word |= ((uint32_t)(int)d & 0xffu) << (8 * u);
        t[u] = (t[u] - d) * 128.0;
      }
      *(uint32_t*)(out + p * pstride + k4) = word;
    }
  }
}

}  // namespace

hipError_t oz_init() {
  return hipFuncSetAttribute((const void*)gemm_oz_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 4 * TILE);
}

hipError_t oz_split(const double* X, int64_t ldx, int64_t K, int64_t ncols, int s, int8_t* P, int* expo, int* info,
                    hipStream_t st) {
  if (s < 1 || s > OZ_MAX_SLICES || K < 0 || ncols < 0) return hipErrorInvalidValue;
  if (ncols == 0) return hipSuccess;
  const int64_t ldp = oz_row_stride(K);
  hipLaunchKernelGGL(k_oz_split, dim3((unsigned)ncols), dim3(256), 0, st, X, ldx, K, ldp, ncols * ldp, s, P, expo,
                     info);
  return hipGetLastError();
}

hipError_t gemm_oz(int64_t M, int64_t N, int64_t K, int s, const int8_t* Ap, const int* ea, const int8_t* Bp,
                   const int* eb, double* C, int64_t ldc, hipStream_t st) {
  if (s < 1 || s > OZ_MAX_SLICES || K < 0 || (int64_t)s * K >= (1 << 19)) return hipErrorInvalidValue;
  if (M <= 0 || N <= 0) return hipSuccess;
  OzArgs a = {};
  a.M = M; a.N = N; a.ldp = oz_row_stride(K); a.pa = M * a.ldp; a.pb = N * a.ldp;
  a.Ap = Ap; a.Bp = Bp; a.ea = ea; a.eb = eb; a.C = C; a.ldc = ldc; a.s = s;
  a.ntk = (int)(a.ldp / BK);
  const int tm = (int)((M + BM - 1) / BM), tn = (int)((N + BN - 1) / BN);
  for (int g = s + 1; g >= 2; --g) {  // smallest weights first
    a.g = g;
    a.first = (g == s + 1);
    hipLaunchKernelGGL(gemm_oz_kernel, dim3((unsigned)(tm * tn)), dim3(NT), 4 * TILE, st, a, tm, tn);
  }
  return hipGetLastError();
}

}  // namespace pfsm
