// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64) with LDS double
// buffering and fused epilogues for the PFSM contractions:
//   basis change  W = A V,  At = V^T W            (EPI_STORE, lower tiles + mirror)
//   folded-spectrum products (At - eps)X, X - a(At - eps)Y   (EPI_SHIFT / EPI_FSUPD)
//   overlap S = X^T X, Cholesky trailing updates    (EPI_STORE, alpha/beta)
//   Rayleigh quotients  x_j^T (At x_j)               (EPI_RQ column-dot partials)
//
// Block tile 128x128x16, 256 threads = 4 waves in a 2x2 grid, each wave owns a
// 64x64 sub-tile = 4x4 MFMA blocks of 16x16.  The MFMA is issued with the B
// fragment as its first operand so that each lane's accumulator entries run
// down a column of C (row = lane%16, col = lane/16 + 4*reg), which makes the
// column-major stores contiguous per column.
#include "common.h"

namespace pfsm {
namespace {

constexpr int BM = GEMM_BM, BN = GEMM_BN, BK = GEMM_BK;
constexpr int PAD = 16;                 // row stride 144 doubles: k and k+1 rows hit opposite bank halves
constexpr int LDA_S = BM + PAD, LDB_S = BN + PAD;
// A tile that is contiguous along k in memory can be kept in LDS as [row][k]
// with an odd stride (17 doubles), so the coalesced global->LDS stores
// (consecutive k) and the MFMA fragment reads (consecutive rows) both avoid
// bank conflicts; the other layout is [k][row].  op(A) = A^T uses [row][k];
// op(B) = B uses it only together with op(A) = A^T (the combination measured
// fastest at N = 8192: 61 TFLOP/s).  Products with a symmetric left operand
// are therefore issued as A^T B.
constexpr int KS = BK + 1;
constexpr int BUF = (BK * LDA_S > BM * KS ? BK * LDA_S : BM * KS);  // doubles per operand buffer
constexpr int NT = 256;
constexpr int A_PER_T = BM * BK / NT;   // 8
constexpr int B_PER_T = BN * BK / NT;   // 8

__device__ inline int xcd_tile(int b, int total) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so neighbouring tiles share its L2.
  if (total % 8 != 0) return b;
  return (b % 8) * (total / 8) + b / 8;
}

__device__ inline void tri_index(int t, int& a, int& b) {
  // t -> (a, b) with a >= b, row-major over the lower triangle
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  a = r;
  b = t - r * (r + 1) / 2;
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(NT, 2) void gemm_f64_kernel(GemmArgs g, int tiles_m, int tiles_n) {
  __shared__ double As[2][BUF];
  __shared__ double Bs[2][BUF];
  __shared__ double red[2][BN];
  // element (row, k) of the A tile / (k, col) of the B tile in buffer b
  auto a_at = [&](int b, int row, int k) -> double& { return TA ? As[b][row * KS + k] : As[b][k * LDA_S + row]; };
  // B tile: [col][k] when it is k-contiguous and A is transposed (measured faster),
  // otherwise [k][col]
  auto b_at = [&](int b, int k, int col) -> double& {
    return (!TB && TA) ? Bs[b][col * KS + k] : Bs[b][k * LDB_S + col];
  };

  int tm, tn;
  if (g.lower_only) {
    // only tiles on or below the diagonal are launched (tiles_m == tiles_n)
    const int total = tiles_m * (tiles_m + 1) / 2;
    tri_index(xcd_tile(blockIdx.x, total), tm, tn);
  } else {
    const int total = tiles_m * tiles_n;
    const int t_lin = xcd_tile(blockIdx.x, total);
    // group 8 row tiles together so consecutive tiles reuse B columns and A rows
    const int GROUP = 8;
    const int group_id = t_lin / (GROUP * tiles_n);
    const int first_m = group_id * GROUP;
    const int gsz = min(tiles_m - first_m, GROUP);
    tm = first_m + (t_lin % (GROUP * tiles_n)) % gsz;
    tn = (t_lin % (GROUP * tiles_n)) / gsz;
  }

  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi0 = (wave & 1) * 64, wj0 = (wave >> 1) * 64;
  const int l16 = lane & 15, lq = lane >> 4;

  int64_t kbeg = 0, kend = g.K;
  if (g.krange) {
    kbeg = g.krange[2 * tn];
    kend = g.krange[2 * tn + 1];
  }

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  double ra[A_PER_T], rb[B_PER_T];

  auto load_tile = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < A_PER_T; ++r) {
      int idx = tid + NT * r;
      int i, k;
      if (!TA) { i = idx % BM; k = idx / BM; } else { k = idx % BK; i = idx / BK; }
      int64_t gi = m0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < g.M && gk < kend) v = TA ? g.A[gk + gi * g.lda] : g.A[gi + gk * g.lda];
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < B_PER_T; ++r) {
      int idx = tid + NT * r;
      int j, k;
      if (!TB) { k = idx % BK; j = idx / BK; } else { j = idx % BN; k = idx / BN; }
      int64_t gj = n0 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < g.N && gk < kend) v = TB ? g.B[gj + gk * g.ldb] : g.B[gk + gj * g.ldb];
      rb[r] = v;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < A_PER_T; ++r) {
      int idx = tid + NT * r;
      int i, k;
      if (!TA) { i = idx % BM; k = idx / BM; } else { k = idx % BK; i = idx / BK; }
      a_at(buf, i, k) = ra[r];
    }
#pragma unroll
    for (int r = 0; r < B_PER_T; ++r) {
      int idx = tid + NT * r;
      int j, k;
      if (!TB) { k = idx % BK; j = idx / BK; } else { j = idx % BN; k = idx / BN; }
      b_at(buf, k, j) = rb[r];
    }
  };

  const int64_t ntk = (kend - kbeg + BK - 1) / BK;
  if (ntk > 0) {
    load_tile(kbeg);
    store_tile(0);
    __syncthreads();
    for (int64_t t = 0; t < ntk; ++t) {
      const int cur = (int)(t & 1);
      if (t + 1 < ntk) load_tile(kbeg + (t + 1) * BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double af[4], bf[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) af[ib] = a_at(cur, wi0 + ib * 16 + l16, kk + lq);
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) bf[jb] = b_at(cur, kk + lq, wj0 + jb * 16 + l16);
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
          for (int jb = 0; jb < 4; ++jb)
            acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[jb], af[ib], acc[ib][jb], 0, 0, 0);
      }
      if (t + 1 < ntk) store_tile(cur ^ 1);
      __syncthreads();
    }
  }

  // ---------------------------------------------------------------- epilogue
  if (EPI == EPI_RQ) {
    // column partial sums of acc .* D over this tile's rows
    double cs[4][4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        int64_t gj = n0 + wj0 + jb * 16 + lq + 4 * r;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          int64_t gi = m0 + wi0 + ib * 16 + l16;
          if (gi < g.M && gj < g.N) s += acc[ib][jb][r] * g.D[gi + gj * g.ldd];
        }
        // reduce over the 16 lanes that share this column (same lane>>4)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
        cs[jb][r] = s;
      }
    if (l16 == 0) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave & 1][wj0 + jb * 16 + lq + 4 * r] = cs[jb][r];
    }
    __syncthreads();
    if (tid < BN) {
      int64_t gj = n0 + tid;
      if (gj < g.N) g.part[(int64_t)tm * g.N + gj] = red[0][tid] + red[1][tid];
    }
    if (!g.part2) return;
    // the same for acc^2 (squared norms of the columns of A X over this tile's rows)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        const int64_t gj = n0 + wj0 + jb * 16 + lq + 4 * r;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          const int64_t gi = m0 + wi0 + ib * 16 + l16;
          if (gi < g.M && gj < g.N) s += acc[ib][jb][r] * acc[ib][jb][r];
        }
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
        cs[jb][r] = s;
      }
    __syncthreads();  // red is read above
    if (l16 == 0) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave & 1][wj0 + jb * 16 + lq + 4 * r] = cs[jb][r];
    }
    __syncthreads();
    if (tid < BN) {
      const int64_t gj = n0 + tid;
      if (gj < g.N) g.part2[(int64_t)tm * g.N + gj] = red[0][tid] + red[1][tid];
    }
    return;
  }

  if (EPI == EPI_G2S) {
    // C = Z + D^{-1}(A - B Z) for the generalized -> standard iteration, with
    // per-column partial sums of the squared residual.  The loads of one row
    // block are gathered before its stores.
    double cs[4][4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) cs[jb][r] = 0.0;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      const int64_t gi = m0 + wi0 + ib * 16 + l16;
      if (gi >= g.M) continue;
      const double di = g.eps[gi];
      double zv[4][4], av[4][4];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gj = min<int64_t>(n0 + wj0 + jb * 16 + lq + 4 * r, g.N - 1);
          zv[jb][r] = g.B[gi + gj * g.ldb];
          av[jb][r] = g.D[gi + gj * g.ldd];
        }
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gj = n0 + wj0 + jb * 16 + lq + 4 * r;
          if (gj >= g.N) continue;
          const double res = av[jb][r] - acc[ib][jb][r];
          g.C[gi + gj * g.ldc] = zv[jb][r] + di * res;
          cs[jb][r] += res * res;
        }
    }
    if (!g.part) return;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s = cs[jb][r];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
        cs[jb][r] = s;
      }
    if (l16 == 0) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave & 1][wj0 + jb * 16 + lq + 4 * r] = cs[jb][r];
    }
    __syncthreads();
    if (tid < BN) {
      const int64_t gj = n0 + tid;
      if (gj < g.N) g.part[(int64_t)tm * g.N + gj] = red[0][tid] + red[1][tid];
    }
    return;
  }

  double a_eff = g.alpha;
  if (EPI == EPI_FSUPD && g.alpha_dev) a_eff = *g.alpha_dev;
#pragma unroll
  for (int ib = 0; ib < 4; ++ib) {
    const int64_t gi = m0 + wi0 + ib * 16 + l16;
    if (gi >= g.M) continue;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gj = n0 + wj0 + jb * 16 + lq + 4 * r;
        if (gj >= g.N) continue;
        double v = acc[ib][jb][r];
        double* cp = g.C + gi + gj * g.ldc;
        if (EPI == EPI_STORE) {
          v = g.alpha * v;
          if (g.beta != 0.0) v += g.beta * (*cp);
        } else if (EPI == EPI_SHIFT) {
          v = v - g.B[gi + gj * g.ldb] * g.eps[gj];
        } else if (EPI == EPI_FSUPD) {
          v = g.D[gi + gj * g.ldd] - a_eff * (v - g.B[gi + gj * g.ldb] * g.eps[gj]);
        }
        *cp = v;
      }
  }
}

template <bool TA, bool TB>
hipError_t launch_epi(int epi, const GemmArgs& a, hipStream_t s) {
  int tm = (int)((a.M + BM - 1) / BM), tn = (int)((a.N + BN - 1) / BN);
  if (tm == 0 || tn == 0) return hipSuccess;
  if (a.lower_only && tm != tn) return hipErrorInvalidValue;
  dim3 grid(a.lower_only ? tm * (tm + 1) / 2 : tm * tn), block(NT);
  switch (epi) {
    case EPI_STORE: hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, EPI_STORE>), grid, block, 0, s, a, tm, tn); break;
    case EPI_SHIFT: hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, EPI_SHIFT>), grid, block, 0, s, a, tm, tn); break;
    case EPI_FSUPD: hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, EPI_FSUPD>), grid, block, 0, s, a, tm, tn); break;
    case EPI_RQ: hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, EPI_RQ>), grid, block, 0, s, a, tm, tn); break;
    case EPI_G2S: hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, EPI_G2S>), grid, block, 0, s, a, tm, tn); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_f64(bool ta, bool tb, int epi, const GemmArgs& a, hipStream_t s) {
  // SHIFT / FSUPD read B at output positions: only the non-transposed square case is valid.
  if ((epi == EPI_SHIFT || epi == EPI_FSUPD || epi == EPI_G2S) && (tb || a.K < a.M)) return hipErrorInvalidValue;
  if (!ta && !tb) return launch_epi<false, false>(epi, a, s);
  if (ta && !tb) return launch_epi<true, false>(epi, a, s);
  if (!ta && tb) return launch_epi<false, true>(epi, a, s);
  return launch_epi<true, true>(epi, a, s);
}

}  // namespace pfsm
