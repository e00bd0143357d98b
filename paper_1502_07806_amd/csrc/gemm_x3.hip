// BF16 hi/lo split GEMM (see gemm_x3.h).  Block tile 256x256x32, 512 threads =
// 8 waves in a 2 (rows) x 4 (columns) grid, each wave 128x64 = 4x2 blocks of
// v_mfma_f32_32x32x16_bf16, two waves per SIMD so one wave's LDS reads overlap
// the other's matrix-core work; per block and k16 step three products
// (hi*hi, hi*lo, lo*hi).  Operand tiles go through registers into LDS
// (double buffered, 144-byte rows so 16 consecutive rows read by a
// ds_read_b128 hit distinct banks).  The MFMA is issued with the B fragment
// first so that each lane's accumulators run down a column of C, which keeps
// the column-major stores contiguous.
#include "common.h"
#include "gemm_x3.h"

#include <algorithm>

namespace pfsm {
namespace {

constexpr int BM = X3_BM, BN = X3_BN, BK = X3_BK;
constexpr int ROWB = 144;                 // LDS bytes per packed row (128 + 16 pad)
constexpr int TILE_BYTES = BM * ROWB;     // 36864 per operand per stage

// Tile configurations: waves per workgroup and MFMA blocks (32x32) per wave.
//   CFG 0: 8 waves in 2 x 4, wave tile 128 x 64  (two waves per SIMD)
//   CFG 1: 4 waves in 2 x 2, wave tile 128 x 128 (one wave per SIMD, least LDS traffic)
//   CFG 2: 8 waves in 4 x 2, wave tile 64 x 128
//   CFG 3: CFG 0 plus an L2 warm-up load (one dword per 128-byte row chunk) of
//          the K tile two steps ahead, consumed one step later, so first-touch
//          HBM latency overlaps two tiles of matrix-core work
//   CFG 4: 8 waves in 4 x 2 fed by direct global -> LDS loads into a 4-stage
//          ring (gemm_x3_dl)
//   CFG 5: CFG 4 with the LDS fragments of the next stage read while the
//          MFMAs of the current one run
template <int CFG> struct X3Cfg;
template <> struct X3Cfg<0> { static constexpr int NT = 512, WGR = 2, WR = 4, WC = 2, PF = 0; };
template <> struct X3Cfg<1> { static constexpr int NT = 256, WGR = 2, WR = 4, WC = 4, PF = 0; };
template <> struct X3Cfg<2> { static constexpr int NT = 512, WGR = 4, WR = 2, WC = 4, PF = 0; };
template <> struct X3Cfg<3> { static constexpr int NT = 512, WGR = 2, WR = 4, WC = 2, PF = 1; };

__device__ inline int xcd_remap(int b, int total) {
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

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ inline v8bf as_bf(u32x4 v) { return __builtin_bit_cast(v8bf, v); }

// Output tile of this block: XCD-grouped, lower / upper triangle enumeration
// for the triangular modes, otherwise groups of 4 row tiles sharing column tiles.
// KPREFIX tiles differ in length (their K ranges follow the triangle), so
// they are dealt longest first with consecutive blocks on different XCDs,
// which balances the XCDs and fills the last wave with short tiles.
__device__ inline void x3_tile_coords(const X3Args& g, int tiles_m, int tiles_n, int& tm, int& tn) {
  int total;
  if (g.tiles == X3_LOWER) total = tiles_m * (tiles_m + 1) / 2;
  else total = tiles_m * tiles_n;
  if (g.split_s > 0) total = g.split_full;  // whole tiles only (the split ones follow)
  const int b = blockIdx.x;
  if (g.tiles == X3_KPREFIX) {  // K range [0, n0 + BN): longest column tiles first
    tn = tiles_n - 1 - b / tiles_m;
    tm = b % tiles_m;
    return;
  }
  const int t = xcd_remap(b, total);
  if (g.tiles == X3_LOWER) {
    tri_index(t, tm, tn);
  } else {
    const int GROUP = 4;
    const int first_m = (t / (GROUP * tiles_n)) * GROUP;
    const int gsz = min(tiles_m - first_m, GROUP);
    tm = first_m + (t % (GROUP * tiles_n)) % gsz;
    tn = (t % (GROUP * tiles_n)) / gsz;
  }
}

// k range of a tile (multiples of 32): the optional per-column-tile and
// per-row-tile ranges, clipped in the KPREFIX mode (op(B) upper triangular).
__device__ inline void x3_k_range(const X3Args& g, int tm, int tn, int64_t m0, int64_t n0, int64_t& kbeg,
                                   int64_t& kend) {
  kbeg = 0;
  kend = (g.K + 31) / 32 * 32;
  if (g.krange) {
    kbeg = g.krange[2 * tn];
    kend = g.krange[2 * tn + 1];
  }
  if (g.krange_rows) {
    kbeg = max<int64_t>(kbeg, g.krange_rows[2 * tm]);
    kend = min<int64_t>(kend, g.krange_rows[2 * tm + 1]);
  }
  if (g.tiles == X3_KPREFIX) kend = min<int64_t>(kend, n0 + BN);
}

// Gate of the band / full forms of a folded-spectrum product (see X3Args):
// true when this launch is not the one that should run.  Every workgroup reads
// the same words, written by earlier launches, so the whole grid agrees.
__device__ inline bool x3_gate_closed(const X3Args& g) {
  if (!g.gate_far) return false;
  const float m = __uint_as_float(*g.gate_far);
  const bool band_ok = g.gate_cl[0] * (double)m <= g.gate_cl[1];  // false for NaN
  return band_ok != (g.gate_band != 0);
}

__device__ inline bf16_t f2bf(float x) {
  // round to nearest even (finite inputs; NaN stays NaN)
  uint32_t b = __builtin_bit_cast(uint32_t, x);
  if ((b & 0x7f800000u) == 0x7f800000u) return (bf16_t)((b >> 16) | ((b & 0xffffu) ? 0x40u : 0u));
  b += 0x7fffu + ((b >> 16) & 1u);
  return (bf16_t)(b >> 16);
}
__device__ inline float bf2f(bf16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// Epilogue shared by the split-BF16 kernels: acc[ib][jb][r] is C(i, j) with
// i = wi0 + 32 ib + lane % 32, j = wj0 + 32 jb + 8 (r / 4) + 4 (lane / 32) + r % 4.
template <int EPI, int WGR, int WR, int WC>
__device__ inline void x3_epilogue(const X3Args& g, v16f (&acc)[WR][WC], int64_t m0, int64_t n0, int wi0, int wj0,
                                   int tid, int tm, double (*red)[BN]) {
  const int lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  if (EPI == X3_RQ) {
    const float* D = (const float*)g.D;
    double cs[WC][16];
#pragma unroll
    for (int jb = 0; jb < WC; ++jb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gj = n0 + wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
        double sum = 0.0;
#pragma unroll
        for (int ib = 0; ib < WR; ++ib) {
          const int64_t gi = m0 + wi0 + ib * 32 + l32;
          if (gi < g.M && gj < g.N) sum += (double)acc[ib][jb][r] * (double)D[gi + gj * g.ldd];
        }
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) sum += __shfl_xor(sum, off, 64);
        cs[jb][r] = sum;
      }
    if (l32 == 0) {
#pragma unroll
      for (int jb = 0; jb < WC; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) red[wave % WGR][wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4)] = cs[jb][r];
    }
    __syncthreads();
    if (tid < BN) {
      const int64_t gj = n0 + tid;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < WGR; ++w) sum += red[w][tid];
      if (gj < g.N) g.part[(int64_t)tm * g.N + gj] = sum;
    }
    return;
  }
  double a_eff = g.alpha;
  if (EPI == X3_FSUPD && g.alpha_dev) a_eff = *g.alpha_dev;
  // rows outside [fk0, fk1) are the far rows of this column tile
  int64_t fk0 = 0, fk1 = 0;
  if ((EPI == X3_SHIFT || EPI == X3_FSUPD) && g.farmax_out) {
    const int64_t tn = n0 / BN;
    fk0 = g.far_krange[2 * tn];
    fk1 = g.far_krange[2 * tn + 1];
  }
  float farmax = 0.0f;
  // C may alias D (in-place update): the inputs of GR outputs are gathered
  // before any of them is stored, so GR loads per input are in flight instead
  // of one.  The folded-spectrum epilogues (FP32 inputs, the whole tile's
  // HBM traffic) gather 16: the main loop's registers are free by now.
  constexpr int GR = (EPI == X3_SHIFT || EPI == X3_FSUPD) ? 16 : 8;
#pragma unroll
  for (int ib = 0; ib < WR; ++ib) {
    const int64_t gi = m0 + wi0 + ib * 32 + l32;
    if (gi >= g.M) continue;
    const double dg = ((EPI == X3_SHIFT || EPI == X3_FSUPD) && g.diag) ? g.diag[gi * g.diag_stride] : 0.0;
    const bool far_row = gi < fk0 || gi >= fk1;
#pragma unroll
    for (int jb = 0; jb < WC; ++jb)
#pragma unroll
      for (int r0 = 0; r0 < 16; r0 += GR) {
        // unconditional loads (columns past N read column N - 1), so that no
        // branch separates them and all of them issue before the first use
        using In = typename std::conditional<EPI == X3_SHIFT || EPI == X3_FSUPD, float, double>::type;
        In in1[GR], in2[GR];
        double ev[GR];
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int r = r0 + u;
          const int64_t gj = min<int64_t>(n0 + wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4), g.N - 1);
          in1[u] = 0.0;
          in2[u] = 0.0;
          ev[u] = 0.0;
          if (EPI == X3_STORE) {
            if (g.beta != 0.0)
              in1[u] = g.c_double ? ((const double*)g.C)[gi + gj * g.ldc] : (double)((const float*)g.C)[gi + gj * g.ldc];
          } else if (EPI == X3_SHIFT) {
            in1[u] = g.B32[gi + gj * g.ldb32];
            ev[u] = g.eps[gj];
          } else if (EPI == X3_FSUPD) {
            in1[u] = g.B32[gi + gj * g.ldb32];
            ev[u] = g.eps[gj];
            in2[u] = ((const float*)g.D)[gi + gj * g.ldd];
          } else if (EPI == X3_ADD) {
            in1[u] = g.d_double ? ((const double*)g.D)[gi + gj * g.ldd] : (double)((const float*)g.D)[gi + gj * g.ldd];
          }
        }
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int r = r0 + u;
          const int64_t gj = n0 + wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
          if (gj >= g.N) continue;
          const double v = (double)acc[ib][jb][r];
          double outv;
          if (EPI == X3_STORE) outv = g.alpha * v + g.beta * in1[u];
          else if (EPI == X3_STORE_PACK) outv = g.alpha * v;
          else if (EPI == X3_SHIFT) outv = v + (double)in1[u] * (dg - ev[u]);
          else if (EPI == X3_FSUPD) outv = (double)in2[u] - a_eff * (v + (double)in1[u] * (dg - ev[u]));
          else outv = g.alpha * v + in1[u];
          if (EPI == X3_STORE_PACK) {  // the hi / lo parts of the FP32 value, as pack_x3 makes them
            const float y = (float)outv;
            const bf16_t h = f2bf(y), l = f2bf((float)((double)y - (double)bf2f(h)));
            bf16_t* dst = g.pack_split + gj * g.ld_pack_split + (gi >> 5) * 64 + (gi & 31);
            dst[0] = h;
            dst[32] = l;
          } else if (g.c_double) {
            ((double*)g.C)[gi + gj * g.ldc] = outv;
          } else {
            ((float*)g.C)[gi + gj * g.ldc] = (float)outv;
          }
          if ((EPI == X3_SHIFT || EPI == X3_FSUPD) && far_row) {
            const float a = fabsf((float)outv);
            farmax = (a > farmax || a != a) ? a : farmax;
          }
        }
      }
  }
  if ((EPI == X3_SHIFT || EPI == X3_FSUPD) && g.farmax_out) {
    // wave maximum, then one atomic per wave (non-negative floats order like
    // their bits; a NaN's bits exceed every finite value's)
    unsigned mb = __float_as_uint(farmax);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) mb = max(mb, (unsigned)__shfl_xor((int)mb, off, 64));
    if (lane == 0 && mb != 0u) atomicMax(g.farmax_out, mb);
  }
}

template <int EPI, int CFG>
__global__ __launch_bounds__(X3Cfg<CFG>::NT, 1) void gemm_x3_kernel(X3Args g, int tiles_m, int tiles_n) {
  constexpr int NT = X3Cfg<CFG>::NT, WGR = X3Cfg<CFG>::WGR, WR = X3Cfg<CFG>::WR, WC = X3Cfg<CFG>::WC;
  constexpr int PF = X3Cfg<CFG>::PF;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  unsigned char* As = lds;                       // [2][BM][ROWB]
  unsigned char* Bs = lds + 2 * TILE_BYTES;      // [2][BN][ROWB]
  __shared__ double red[WGR][BN];
  if (x3_gate_closed(g)) return;
  if (g.band_count && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(g.band_count, 1u);

  int tm, tn;
  x3_tile_coords(g, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi0 = (wave % WGR) * (32 * WR), wj0 = (wave / WGR) * (32 * WC);
  const int l32 = lane & 31, lh = lane >> 5;
  int64_t kbeg, kend;
  x3_k_range(g, tm, tn, m0, n0, kbeg, kend);

  v16f acc[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // global -> register staging: thread t loads chunk (t % 8) of rows t/8 + 64 q, q < 4
  constexpr int LQ = BM * 8 / NT;  // 4
  const int chunk = tid & 7, rbase = tid >> 3;
  u32x4 ra[LQ], rb[LQ];
  auto load_tile = [&](int64_t k0) {
    const int64_t kc = k0 / 32;
#pragma unroll
    for (int q = 0; q < LQ; ++q) {
      const int r = rbase + (NT / 8) * q;
      const int64_t gi = m0 + r, gj = n0 + r;
      u32x4 z = {0u, 0u, 0u, 0u};
      ra[q] = (gi < g.M) ? *(const u32x4*)(g.Ap + gi * g.ldap + kc * 64 + chunk * 8) : z;
      rb[q] = (gj < g.N) ? *(const u32x4*)(g.Bp + gj * g.ldbp + kc * 64 + chunk * 8) : z;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LQ; ++q) {
      const int r = rbase + (NT / 8) * q;
      *(u32x4*)(As + buf * TILE_BYTES + r * ROWB + chunk * 16) = ra[q];
      *(u32x4*)(Bs + buf * TILE_BYTES + r * ROWB + chunk * 16) = rb[q];
    }
  };

  const int64_t ntk = kend > kbeg ? (kend - kbeg) / BK : 0;
  // L2 warm-up (PF): thread t touches row t % 256 of A (t < 256) or of B, one dword per tile
  uint32_t pf_keep = 0, pf_sink = 0;
  auto warm = [&](int64_t k0) {
    const int r = tid & 255;
    const bool isA = tid < 256;
    const int64_t row = (isA ? m0 : n0) + r;
    const int64_t lim = isA ? g.M : g.N;
    if (row < lim) {
      const bf16_t* base = isA ? g.Ap + row * g.ldap : g.Bp + row * g.ldbp;
      pf_keep = *(const uint32_t*)(base + (k0 / 32) * 64);
    }
  };
  if (ntk > 0) {
    load_tile(kbeg);
    store_tile(0);
    if (PF && ntk > 2) warm(kbeg + 2 * BK);
    __syncthreads();
    for (int64_t t = 0; t < ntk; ++t) {
      const int cur = (int)(t & 1);
      if (t + 1 < ntk) load_tile(kbeg + (t + 1) * BK);
      if (PF) {
        pf_sink ^= pf_keep;  // consumes the warm-up load issued one step earlier
        if (t + 3 < ntk) warm(kbeg + (t + 3) * BK);
      }
      const unsigned char* Ab = As + cur * TILE_BYTES;
      const unsigned char* Bb = Bs + cur * TILE_BYTES;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int koff = 32 * s + 16 * lh;  // byte offset of this lane's 8 k values in the hi plane
        v8bf ah[WR], al[WR], bh[WC], bl[WC];
#pragma unroll
        for (int ib = 0; ib < WR; ++ib) {
          const unsigned char* p = Ab + (wi0 + ib * 32 + l32) * ROWB + koff;
          ah[ib] = as_bf(*(const u32x4*)p);
          al[ib] = as_bf(*(const u32x4*)(p + 64));
        }
#pragma unroll
        for (int jb = 0; jb < WC; ++jb) {
          const unsigned char* p = Bb + (wj0 + jb * 32 + l32) * ROWB + koff;
          bh[jb] = as_bf(*(const u32x4*)p);
          bl[jb] = as_bf(*(const u32x4*)(p + 64));
        }
#pragma unroll
        for (int ib = 0; ib < WR; ++ib)
#pragma unroll
          for (int jb = 0; jb < WC; ++jb) {
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh[jb], ah[ib], acc[ib][jb], 0, 0, 0);
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bl[jb], ah[ib], acc[ib][jb], 0, 0, 0);
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh[jb], al[ib], acc[ib][jb], 0, 0, 0);
          }
      }
      if (t + 1 < ntk) store_tile(cur ^ 1);
      __syncthreads();
    }
  }

  if (PF && pf_sink == 0x7fc0ffeeu && g.part) g.part[0] = 0.0;  // keeps the warm-up loads alive
  x3_epilogue<EPI, WGR, WR, WC>(g, acc, m0, n0, wi0, wj0, tid, tm, red);
}

// Direct global -> LDS variant (CFG 4): a 4-stage ring of k16 stages filled
// by 16-byte-per-lane direct loads, so loads run three stages ahead of the
// matrix cores with no register staging.  A stage row is 64 bytes: the hi
// and lo halves of 16 k values, two 16-byte chunks each, XOR-swizzled by
// chunk ^ ((row >> 1) ^ (row >> 2)) & 3 (fragment reads of 8 and of 16
// consecutive rows hit distinct banks).  8 waves in 4 x 2, wave tile 64 x 128.
// Rows past the matrix edge read the last row (their outputs are not stored).
constexpr int DST = 4, DROW = 64, DTILE = BM * DROW;  // 16 KB per operand and stage

__device__ inline int dswz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding direct-to-LDS load); the empty asm statements
// keep the compiler from moving LDS accesses across it.
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int W> __device__ inline void wait_vm() {
  // vmcnt = W (0..63); expcnt and lgkmcnt left at their maxima
  __builtin_amdgcn_s_waitcnt((W & 15) | (7 << 4) | (15 << 8) | (((W >> 4) & 3) << 14));
}

// NP = 3: the three split products of k16 stages of the split layout.
// NP = 1: one product from operands in the plain layout; a stage then holds
// 32 k values per row (the same 64 bytes, four 16-byte chunks of 8 k), and
// the two fragment slots (hi, lo) carry the first and second 16 k of it.
template <int EPI, bool PIPE, int NP = 3>
__global__ __launch_bounds__(512, 1) void gemm_x3_dl(X3Args g, int tiles_m, int tiles_n) {
  constexpr int NW = 8, WGR = 4, WR = 2, WC = 4, CPW = 16 / NW;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ double red[WGR][BN];
  if (x3_gate_closed(g)) return;
  if (g.band_count && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(g.band_count, 1u);
  int tm, tn, unit = -1;  // unit: K-split piece of a tail tile, -1 for a whole tile
  if (g.split_s > 0 && (int)blockIdx.x >= g.split_full) {
    unit = (int)blockIdx.x - g.split_full;
    tri_index(g.split_full + unit / g.split_s, tm, tn);
  } else {
    x3_tile_coords(g, tiles_m, tiles_n, tm, tn);
  }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi0 = (wave % WGR) * (32 * WR), wj0 = (wave / WGR) * (32 * WC);
  const int l32 = lane & 31, lh = lane >> 5;
  int64_t kbeg, kend;
  x3_k_range(g, tm, tn, m0, n0, kbeg, kend);
  if (unit >= 0) {  // piece unit % S of S equal runs of k16 stages
    const int64_t st = kend > kbeg ? (kend - kbeg) / 16 : 0, sl = unit % g.split_s;
    const int64_t b0 = kbeg + 16 * (st * sl / g.split_s), b1 = kbeg + 16 * (st * (sl + 1) / g.split_s);
    kbeg = b0;
    kend = b1;
  }
  constexpr int SK = NP == 1 ? 32 : 16;  // k values per stage
  const int total = kend > kbeg ? (int)((kend - kbeg) / SK) : 0;

  // byte offsets of this lane's 16-byte chunk in each 1 KB row group it loads
  int64_t offA[CPW], offB[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int row = 16 * (wave * CPW + j) + (lane >> 2);
    // logical chunk: split layout hi k0-7, hi k8-15, lo k0-7, lo k8-15;
    // plain layout k0-7, k8-15, k16-23, k24-31
    const int c = (lane & 3) ^ dswz(row);
    const int coff = NP == 1 ? 16 * c : (c >> 1) * 64 + (c & 1) * 16;
    offA[j] = min<int64_t>(m0 + row, g.M - 1) * g.ldap * 2 + coff;
    offB[j] = min<int64_t>(n0 + row, g.N - 1) * g.ldbp * 2 + coff;
  }
  auto issue = [&](int t) {
    const int64_t k0 = kbeg + SK * (int64_t)t;
    const int64_t koff = NP == 1 ? 2 * k0 : (k0 >> 5) * 128 + ((k0 >> 4) & 1) * 32;
    const unsigned char* A = (const unsigned char*)g.Ap + koff;
    const unsigned char* B = (const unsigned char*)g.Bp + koff;
    unsigned char* sA = lds + (t % DST) * 2 * DTILE;
    unsigned char* sB = sA + DTILE;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(A + offA[j]),
                                       (void __attribute__((address_space(3)))*)(sA + (wave * CPW + j) * 1024), 16, 0,
                                       0);
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(B + offB[j]),
                                       (void __attribute__((address_space(3)))*)(sB + (wave * CPW + j) * 1024), 16, 0,
                                       0);
    }
  };

  v16f acc[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  struct Frags {
    v8bf ah[WR], al[WR], bh[WC], bl[WC];
  };
  auto read_frags = [&](int t, Frags& f) {
    const unsigned char* Ab = lds + (t % DST) * 2 * DTILE;
    const unsigned char* Bb = Ab + DTILE;
#pragma unroll
    for (int ib = 0; ib < WR; ++ib) {
      const int row = wi0 + ib * 32 + l32, sw = dswz(row);
      f.ah[ib] = as_bf(*(const u32x4*)(Ab + row * DROW + 16 * (lh ^ sw)));
      f.al[ib] = as_bf(*(const u32x4*)(Ab + row * DROW + 16 * ((2 + lh) ^ sw)));
    }
#pragma unroll
    for (int jb = 0; jb < WC; ++jb) {
      const int row = wj0 + jb * 32 + l32, sw = dswz(row);
      f.bh[jb] = as_bf(*(const u32x4*)(Bb + row * DROW + 16 * (lh ^ sw)));
      f.bl[jb] = as_bf(*(const u32x4*)(Bb + row * DROW + 16 * ((2 + lh) ^ sw)));
    }
  };
  auto mma = [&](const Frags& f) {
    // product-major order: consecutive MFMAs update different accumulators
    if (NP == 3) {
#pragma unroll
      for (int pr = 0; pr < 3; ++pr)
#pragma unroll
        for (int ib = 0; ib < WR; ++ib)
#pragma unroll
          for (int jb = 0; jb < WC; ++jb)
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pr == 1 ? f.bl[jb] : f.bh[jb],
                                                                  pr == 2 ? f.al[ib] : f.ah[ib], acc[ib][jb], 0, 0, 0);
    } else {  // first 16 k of the stage, then the second 16
#pragma unroll
      for (int pr = 0; pr < 2; ++pr)
#pragma unroll
        for (int ib = 0; ib < WR; ++ib)
#pragma unroll
          for (int jb = 0; jb < WC; ++jb)
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pr == 1 ? f.bl[jb] : f.bh[jb],
                                                                  pr == 1 ? f.al[ib] : f.ah[ib], acc[ib][jb], 0, 0, 0);
    }
  };

  for (int t = 0; t < DST - 1 && t < total; ++t) issue(t);
  if (!PIPE) {
    for (int t = 0; t < total; ++t) {
      const int later = min(DST - 2, total - 1 - t);  // stages issued after t that may still be in flight
      if (later >= 2) wait_vm<2 * 2 * CPW>();
      else if (later == 1) wait_vm<2 * CPW>();
      else wait_vm<0>();
      // Bare barrier (a fenced one would wait for every outstanding load):
      // every wave's part of stage t has landed, and stage t - 1 was consumed.
      lds_barrier();
      if (t + DST - 1 < total) issue(t + DST - 1);
      Frags f;
      read_frags(t, f);
      mma(f);
    }
  } else if (total > 0) {
    // Fragments one stage ahead: stage t + 1 is read from LDS while the
    // MFMAs of stage t run.  Stage t + 1 must have landed before that read
    // (barrier at the top of iteration t); the slot refilled in iteration t,
    // (t + 3) % 4, held stage t - 1, whose fragments were read in iteration
    // t - 2 and consumed in iteration t - 1, before this barrier.
    {
      const int later0 = min(DST - 2, total - 1);
      if (later0 >= 2) wait_vm<2 * 2 * CPW>();
      else if (later0 == 1) wait_vm<2 * CPW>();
      else wait_vm<0>();
      lds_barrier();
    }
    Frags F0, F1;
    read_frags(0, F0);
    // The fragment read is unconditional (past the last stage it reads a
    // stale slot whose values are never used): with the same number of LDS
    // reads on every path, the wait before the MFMAs covers only the
    // previous step's reads instead of draining all of them.
    auto step = [&](int t, Frags& cur, Frags& nxt) {
      if (t + 1 < total) {
        if (t + 2 <= total - 1) wait_vm<2 * CPW>();  // stage t + 2 may still be in flight
        else wait_vm<0>();
        lds_barrier();
        if (t + DST - 1 < total) issue(t + DST - 1);
      }
      __builtin_amdgcn_sched_barrier(0);
      read_frags(t + 1, nxt);
      mma(cur);
      // interleave: two MFMAs of stage t, then one fragment read of stage
      // t + 1, so the reads complete under this step's MFMAs and the wait at
      // the next step finds them done
      if (NP == 3) {
#pragma unroll
        for (int u = 0; u < 2 * (WR + WC); ++u) {
          __builtin_amdgcn_sched_group_barrier(0x008, 3 * WR * WC / (2 * (WR + WC)), 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
      } else {  // 2 WR WC MFMAs and 2 (WR + WC) fragment reads
#pragma unroll
        for (int u = 0; u < 2 * (WR + WC); ++u) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    };
    for (int t = 0; t < total; t += 2) {
      step(t, F0, F1);
      if (t + 1 < total) step(t + 1, F1, F0);
    }
  }
  __syncthreads();  // the RQ epilogue reuses shared memory; no wave may still be reading stages
  if (unit >= 0) {
    // partial sums of a K piece, tile-local column-major: ws[unit][j][i]
    float* P = g.split_ws + (size_t)unit * BM * BN;
#pragma unroll
    for (int ib = 0; ib < WR; ++ib)
#pragma unroll
      for (int jb = 0; jb < WC; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          P[(wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4)) * BM + wi0 + ib * 32 + l32] = acc[ib][jb][r];
    return;
  }
  x3_epilogue<EPI, WGR, WR, WC>(g, acc, m0, n0, wi0, wj0, tid, tm, red);
}

// Sum of the S K pieces of each split tail tile (fixed order) and the STORE
// epilogue C = alpha * sum + beta * C.  Block (tile, column), thread = row.
__global__ __launch_bounds__(256) void k_x3_split_sum(X3Args g) {
  const int tile = blockIdx.x;
  int tm, tn;
  tri_index(g.split_full + tile, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int i = threadIdx.x;
  const int64_t gi = m0 + i;
  const int j = blockIdx.y;
  const int64_t gj = n0 + j;
  if (gi >= g.M || gj >= g.N) return;
  {
    const float* P = g.split_ws + ((size_t)tile * g.split_s * BN + j) * BM + i;
    float sum = 0.f;
    for (int u = 0; u < g.split_s; ++u) sum += P[(size_t)u * BM * BN];
    double outv = g.alpha * (double)sum;
    if (g.beta != 0.0)
      outv += g.beta * (g.c_double ? ((const double*)g.C)[gi + gj * g.ldc] : (double)((const float*)g.C)[gi + gj * g.ldc]);
    if (g.c_double) ((double*)g.C)[gi + gj * g.ldc] = outv;
    else ((float*)g.C)[gi + gj * g.ldc] = (float)outv;
  }
}

// ---------------------------------------------------------------- packing

// One workgroup packs a 32 (k) x 64 (r) block: reads through LDS so that
// both the column-major source and the packed destination are contiguous.
// One 64 (r) x 32 (k) block of the packed operand (rows r0 .., chunk kc).
__device__ void pack_block(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P,
                           int64_t ldp, int64_t r0, int64_t kc, double (*tile)[33], bf16_t* P2 = nullptr,
                           int64_t ldp2 = 0);

// krange (optional): only the chunks inside [krange[2 t], krange[2 t + 1]) for
// the rows of P in tile t = r / 256 (band part, the grid's x covering the
// widest range), or with FAR only the chunks outside it, striding over a
// fixed grid, and only when the gate {gate_far, gate_cl} of X3Args is closed
// for the band form.
template <bool FAR>
__global__ __launch_bounds__(256) void k_pack(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx,
                                              int flags, bf16_t* P, int64_t ldp, const int32_t* krange,
                                              const unsigned* gate_far, const double* gate_cl) {
  __shared__ double tile[64][33];
  const int by_rows = flags & PACK_BY_ROWS;
  const int64_t R = by_rows ? m : n;
  const int64_t K = by_rows ? n : m;
  if (!FAR) {
    const int64_t r0 = (int64_t)blockIdx.y * 64;
    int64_t kc = blockIdx.x;
    if (krange) {
      kc += krange[2 * (r0 / BN)] / 32;
      if (32 * kc >= krange[2 * (r0 / BN) + 1]) return;
    }
    pack_block(X, src_double, m, n, ldx, flags, P, ldp, r0, kc, tile);
    return;
  }
  const float gm = __uint_as_float(*gate_far);
  if (gate_cl[0] * (double)gm <= gate_cl[1]) return;  // the band form runs (false for NaN)
  const int64_t nkc = (K + 31) / 32, nrb = (R + 63) / 64;
  for (int64_t b = blockIdx.x; b < nkc * nrb; b += gridDim.x) {  // uniform per workgroup
    const int64_t r0 = (b / nkc) * 64, kc = b % nkc;
    if (32 * kc >= krange[2 * (r0 / BN)] && 32 * kc < krange[2 * (r0 / BN) + 1]) continue;
    pack_block(X, src_double, m, n, ldx, flags, P, ldp, r0, kc, tile);
    __syncthreads();  // the tile is reused by the next block
  }
}

// Both layouts from one read: P split (flags without PACK_PLAIN), P2 plain.
__global__ __launch_bounds__(256) void k_pack_dual(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx,
                                                   int flags, bf16_t* P, int64_t ldp, bf16_t* P2, int64_t ldp2) {
  __shared__ double tile[64][33];
  pack_block(X, src_double, m, n, ldx, flags, P, ldp, (int64_t)blockIdx.y * 64, blockIdx.x, tile, P2, ldp2);
}

__device__ void pack_block(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P,
                           int64_t ldp, int64_t r0, int64_t kc, double (*tile)[33], bf16_t* P2, int64_t ldp2) {
  const int by_rows = flags & PACK_BY_ROWS;
  // packed operand: rows r in [0, R), k in [0, K); R = by_rows ? m : n, K = by_rows ? n : m
  const int64_t R = by_rows ? m : n;
  const int64_t K = by_rows ? n : m;
  const int tid = threadIdx.x;
  // load X values for (r, k) r in [r0, r0+64), k in [32 kc, 32 kc + 32)
  for (int idx = tid; idx < 64 * 32; idx += 256) {
    int rr, kk;
    int64_t row, col;  // position in X (column-major)
    if (by_rows) {  // X(r, k): contiguous in r for fixed k
      rr = idx % 64; kk = idx / 64;
      row = r0 + rr; col = 32 * kc + kk;
    } else {        // X(k, r): contiguous in k for fixed r
      kk = idx % 32; rr = idx / 32;
      row = 32 * kc + kk; col = r0 + rr;
    }
    double v = 0.0;
    const bool keep = !((flags & PACK_LOWER) && row < col) && !((flags & PACK_UPPER) && row > col);
    if ((by_rows ? (row < R && col < K) : (row < K && col < R)) && keep) {
      v = src_double ? ((const double*)X)[row + col * ldx] : (double)((const float*)X)[row + col * ldx];
      if ((flags & PACK_SUB_I) && row == col) v -= 1.0;
      if ((flags & PACK_HALF_DIAG) && row == col) v *= 0.5;
      if ((flags & PACK_OFFDIAG) && row == col) v = 0.0;
    }
    tile[rr][kk] = v;
  }
  __syncthreads();
  // write: 64 rows x 64 bf16 (hi 32 | lo 32); thread (row, c) makes k = 8c .. 8c+7
  // and stores one 16-byte chunk of each plane
  const int rr = tid >> 2, c = tid & 3;
  const int64_t r = r0 + rr;
  if (r < R) {
    u32x4 hw, lw;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double v0 = tile[rr][8 * c + 2 * u], v1 = tile[rr][8 * c + 2 * u + 1];
      const bf16_t h0 = f2bf((float)v0), h1 = f2bf((float)v1);
      const bf16_t l0 = f2bf((float)(v0 - (double)bf2f(h0))), l1 = f2bf((float)(v1 - (double)bf2f(h1)));
      hw[u] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      lw[u] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    if (P2) *(u32x4*)(P2 + r * ldp2 + kc * 32 + 8 * c) = hw;  // the plain layout holds the hi parts
    if (flags & PACK_PLAIN) {  // 64-byte aligned: ldp is a multiple of 32
      *(u32x4*)(P + r * ldp + kc * 32 + 8 * c) = hw;
      return;
    }
    bf16_t* dst = P + r * ldp + kc * 64;  // 128-byte aligned: ldp is a multiple of 64
    *(u32x4*)(dst + 8 * c) = hw;
    *(u32x4*)(dst + 32 + 8 * c) = lw;
  }
}

// Packing without transpose (row r of the packed operand is column r of X, k
// contiguous in memory): no staging is needed.  A thread turns 8 consecutive k
// of one column into a 16-byte chunk of each plane; 16 threads cover 128 k of
// a column (contiguous loads, 128-byte packed chunks).  VEC: X and ldx allow
// 16-byte loads.
// krange (optional): only the k in [krange[2 t], krange[2 t + 1]) for the rows
// r of P in tile t = r / 256, the grid's x covering the widest range.
template <bool DBL, bool VEC>
__global__ __launch_bounds__(256) void k_pack_cols(const void* X, int64_t K, int64_t R, int64_t ldx, int flags,
                                                   bf16_t* P, int64_t ldp, const int32_t* krange) {
  const int q = threadIdx.x & 15;
  const int64_t r = (int64_t)blockIdx.y * 16 + (threadIdx.x >> 4);
  if (r >= R) return;
  int64_t k0 = (int64_t)blockIdx.x * 128 + 8 * q, kend = (K + 31) / 32 * 32;  // chunks past K are zero-filled
  if (krange) {
    k0 += krange[2 * (r / BN)];
    kend = krange[2 * (r / BN) + 1];
  }
  if (k0 >= kend) return;
  double v[8];
  if (VEC && k0 + 8 <= K) {
    if (DBL) {
      const double2* src = (const double2*)((const double*)X + k0 + r * ldx);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 w = src[u];
        v[2 * u] = w.x;
        v[2 * u + 1] = w.y;
      }
    } else {
      const float4* src = (const float4*)((const float*)X + k0 + r * ldx);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float4 w = src[u];
        v[4 * u] = w.x;
        v[4 * u + 1] = w.y;
        v[4 * u + 2] = w.z;
        v[4 * u + 3] = w.w;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t k = k0 + u;
      v[u] = k < K ? (DBL ? ((const double*)X)[k + r * ldx] : (double)((const float*)X)[k + r * ldx]) : 0.0;
    }
  }
  if (flags & (PACK_LOWER | PACK_UPPER | PACK_SUB_I | PACK_HALF_DIAG | PACK_OFFDIAG)) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t k = k0 + u;  // X(row = k, col = r)
      if (((flags & PACK_LOWER) && k < r) || ((flags & PACK_UPPER) && k > r)) v[u] = 0.0;
      if (k == r && k < K) {
        if (flags & PACK_SUB_I) v[u] -= 1.0;
        if (flags & PACK_HALF_DIAG) v[u] *= 0.5;
        if (flags & PACK_OFFDIAG) v[u] = 0.0;
      }
    }
  }
  u32x4 hw, lw;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const bf16_t h0 = f2bf((float)v[2 * u]), h1 = f2bf((float)v[2 * u + 1]);
    const bf16_t l0 = f2bf((float)(v[2 * u] - (double)bf2f(h0))), l1 = f2bf((float)(v[2 * u + 1] - (double)bf2f(h1)));
    hw[u] = (uint32_t)h0 | ((uint32_t)h1 << 16);
    lw[u] = (uint32_t)l0 | ((uint32_t)l1 << 16);
  }
  if (flags & PACK_PLAIN) {
    *(u32x4*)(P + r * ldp + k0) = hw;
    return;
  }
  bf16_t* dst = P + r * ldp + (k0 >> 5) * 64 + (k0 & 31);
  *(u32x4*)dst = hw;
  *(u32x4*)(dst + 32) = lw;
}

// Eight consecutive k (a multiple of 8) of FP32 column r as plain BF16, zero
// past K.
template <bool VEC>
__device__ inline void pack_plain_chunk(const float* X, int64_t K, int64_t ldx, int64_t r, int64_t k0, bf16_t* P,
                                        int64_t ldp) {
  float v[8];
  if (VEC && k0 + 8 <= K) {
    const float4* src = (const float4*)(X + k0 + r * ldx);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float4 w = src[u];
      v[4 * u] = w.x;
      v[4 * u + 1] = w.y;
      v[4 * u + 2] = w.z;
      v[4 * u + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k0 + u < K ? X[k0 + u + r * ldx] : 0.0f;
  }
  u32x4 hw;
#pragma unroll
  for (int u = 0; u < 4; ++u) hw[u] = (uint32_t)f2bf(v[2 * u]) | ((uint32_t)f2bf(v[2 * u + 1]) << 16);
  *(u32x4*)(P + r * ldp + k0) = hw;
}

// Far part: a fixed grid striding over every (column, chunk of 8 k) outside
// the band, after the gate test of x3_gate_closed for the band launch.
template <bool VEC>
__global__ __launch_bounds__(256) void k_pack_plain_far(const float* X, int64_t K, int64_t R, int64_t ldx,
                                                        const int32_t* krange, bf16_t* P, int64_t ldp,
                                                        const unsigned* gate_far, const double* gate_cl) {
  const float m = __uint_as_float(*gate_far);
  if (gate_cl[0] * (double)m <= gate_cl[1]) return;  // the band form runs (false for NaN)
  const int64_t nch = (K + 31) / 32 * 4;  // chunks of 8 per column, padding included
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < R * nch; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = c / nch, k = (c % nch) * 8, t = r / BN;
    if (k >= krange[2 * t] && k < krange[2 * t + 1]) continue;
    pack_plain_chunk<VEC>(X, K, ldx, r, k, P, ldp);
  }
}

template <int CFG>
hipError_t launch_cfg(int epi, const X3Args& a, int tm, int tn, hipStream_t s) {
  int total = a.tiles == X3_LOWER ? tm * (tm + 1) / 2 : tm * tn;
  const size_t lds = 4 * (size_t)TILE_BYTES;
  dim3 grid(total), block(X3Cfg<CFG>::NT);
  switch (epi) {
#define X3_CASE(E)                                                                \
  case E:                                                                         \
    hipLaunchKernelGGL((gemm_x3_kernel<E, CFG>), grid, block, lds, s, a, tm, tn); \
    break;
    X3_CASE(X3_STORE)
    X3_CASE(X3_SHIFT)
    X3_CASE(X3_FSUPD)
    X3_CASE(X3_ADD)
    X3_CASE(X3_RQ)
#undef X3_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int CFG>
hipError_t set_attrs() {
  const int lds = 4 * TILE_BYTES;
  hipError_t e = hipSuccess;
#define X3_ATTR(E)                                                                                        \
  if (e == hipSuccess)                                                                                    \
    e = hipFuncSetAttribute((const void*)gemm_x3_kernel<E, CFG>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            lds);
  X3_ATTR(X3_STORE)
  X3_ATTR(X3_SHIFT)
  X3_ATTR(X3_FSUPD)
  X3_ATTR(X3_ADD)
  X3_ATTR(X3_RQ)
#undef X3_ATTR
  return e;
}

}  // namespace

int x3_default_cfg = 5;  // fastest measured at N = 8192 (direct-to-LDS ring, fragments one stage ahead)
static int x3_num_cu = 0;  // compute units of the device (workgroups of one wave)

size_t x3_split_bytes(int64_t n) {
  const int64_t t = (n + BM - 1) / BM, tiles = t * (t + 1) / 2;
  if (x3_num_cu <= 0 || tiles <= x3_num_cu) return 0;
  return (size_t)x3_num_cu * BM * BN * sizeof(float);
}

hipError_t x3_init() {
  {
    int dev = 0, cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    x3_num_cu = cu;
  }
  // Dynamic LDS above 64 KiB must be enabled per kernel before the first
  // launch; done once at plan creation so that solves stay capturable.
  hipError_t e = set_attrs<0>();
  if (e == hipSuccess) e = set_attrs<1>();
  if (e == hipSuccess) e = set_attrs<2>();
  if (e == hipSuccess) e = set_attrs<3>();
  const int dl = DST * 2 * DTILE;
#define X3_DL_ATTR(E)                                                                                         \
  if (e == hipSuccess)                                                                                        \
    e = hipFuncSetAttribute((const void*)gemm_x3_dl<E, false>, hipFuncAttributeMaxDynamicSharedMemorySize, dl); \
  if (e == hipSuccess)                                                                                        \
    e = hipFuncSetAttribute((const void*)gemm_x3_dl<E, true>, hipFuncAttributeMaxDynamicSharedMemorySize, dl);
  X3_DL_ATTR(X3_STORE)
  X3_DL_ATTR(X3_SHIFT)
  X3_DL_ATTR(X3_FSUPD)
  X3_DL_ATTR(X3_ADD)
  X3_DL_ATTR(X3_RQ)
  X3_DL_ATTR(X3_STORE_PACK)
#undef X3_DL_ATTR
#define X3_DL1_ATTR(E)                                                                                            \
  if (e == hipSuccess)                                                                                            \
    e = hipFuncSetAttribute((const void*)gemm_x3_dl<E, true, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, dl);
  X3_DL1_ATTR(X3_SHIFT)
  X3_DL1_ATTR(X3_FSUPD)
  X3_DL1_ATTR(X3_ADD)
#undef X3_DL1_ATTR
  return e;
}

template <int E>
void launch_dl(bool one, bool pipe, int total, size_t dl, hipStream_t s, const X3Args& b, int tm, int tn) {
  if constexpr (E == X3_SHIFT || E == X3_FSUPD || E == X3_ADD) {
    if (one) {
      hipLaunchKernelGGL((gemm_x3_dl<E, true, 1>), dim3(total), dim3(512), dl, s, b, tm, tn);
      return;
    }
  }
  if (pipe) hipLaunchKernelGGL((gemm_x3_dl<E, true>), dim3(total), dim3(512), dl, s, b, tm, tn);
  else hipLaunchKernelGGL((gemm_x3_dl<E, false>), dim3(total), dim3(512), dl, s, b, tm, tn);
}

hipError_t gemm_x3(int epi, const X3Args& a, hipStream_t s) {
  const int tm = (int)((a.M + BM - 1) / BM), tn = (int)((a.N + BN - 1) / BN);
  if (tm == 0 || tn == 0) return hipSuccess;
  if (a.tiles == X3_LOWER && tm != tn) return hipErrorInvalidValue;
  if (a.products != 0 && a.products != 1 && a.products != 3) return hipErrorInvalidValue;
  if (epi == X3_STORE_PACK &&
      (!a.pack_split || a.tiles == X3_LOWER || a.M % 32 != 0 || a.ld_pack_split < x3_row_stride(a.M) || a.products == 1))
    return hipErrorInvalidValue;
  const bool one = a.products == 1;
  if (one && ((epi != X3_SHIFT && epi != X3_FSUPD && epi != X3_ADD) || a.tiles == X3_LOWER)) return hipErrorInvalidValue;
  // products on plain operands and the packing epilogue run in the direct-to-LDS configuration
  const int cfg = (one || epi == X3_STORE_PACK) ? 5 : (a.cfg >= 0 ? a.cfg : x3_default_cfg);
  switch (cfg) {
    case 0: return launch_cfg<0>(epi, a, tm, tn, s);
    case 1: return launch_cfg<1>(epi, a, tm, tn, s);
    case 2: return launch_cfg<2>(epi, a, tm, tn, s);
    case 3: return launch_cfg<3>(epi, a, tm, tn, s);
    case 4:
    case 5: {
      int total = a.tiles == X3_LOWER ? tm * (tm + 1) / 2 : tm * tn;
      const size_t dl = DST * 2 * DTILE;
      const bool pipe = cfg == 5;
      X3Args b = a;
      b.split_full = 0;
      b.split_s = 0;
      if (epi == X3_STORE && a.tiles == X3_LOWER && a.split_ws && !a.krange && x3_num_cu > 0) {
        // The tiles past the last whole wave of workgroups (rem of them, at
        // most half a wave) are each cut into S pieces along K, so that the
        // tail wave holds rem * S <= CUs short pieces instead of rem tiles.
        const int cu = x3_num_cu, rem = total % cu;
        const int64_t stages = (a.K + 31) / 32 * 2;
        if (total > cu && rem > 0 && 2 * rem <= cu) {
          const int S = (int)std::min<int64_t>(cu / rem, stages / 8);
          if (S >= 2 && (size_t)rem * S * BM * BN * sizeof(float) <= a.split_bytes) {
            b.split_full = total - rem;
            b.split_s = S;
            total = b.split_full + rem * S;
          }
        }
      }
      switch (epi) {
#define X3_DL_CASE(E)                            \
  case E:                                        \
    launch_dl<E>(one, pipe, total, dl, s, b, tm, tn); \
    break;
        X3_DL_CASE(X3_STORE)
        X3_DL_CASE(X3_SHIFT)
        X3_DL_CASE(X3_FSUPD)
        X3_DL_CASE(X3_ADD)
        X3_DL_CASE(X3_RQ)
        X3_DL_CASE(X3_STORE_PACK)
#undef X3_DL_CASE
        default: return hipErrorInvalidValue;
      }
      if (b.split_s > 0) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int rem = (total - b.split_full) / b.split_s;
        hipLaunchKernelGGL(k_x3_split_sum, dim3(rem, BN), dim3(256), 0, s, b);
      }
      return hipGetLastError();
    }
    default: return hipErrorInvalidValue;
  }
}

hipError_t pack_x3_band(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P,
                        int64_t ldp, const int32_t* krange, int band_chunks, hipStream_t s) {
  const bool by_rows = flags & PACK_BY_ROWS;
  const int64_t R = by_rows ? m : n;
  const int64_t K = by_rows ? n : m;
  if (R <= 0 || K <= 0) return hipSuccess;
  if (!by_rows) {
    const size_t es = src_double ? 8 : 4;
    const bool vec = ((uintptr_t)X % 16 == 0) && ((size_t)ldx * es) % 16 == 0;
    if (krange && band_chunks <= 0) return hipSuccess;
    dim3 grid((unsigned)(krange ? (band_chunks * 32 + 127) / 128 : (K + 127) / 128), (unsigned)((R + 15) / 16));
    const int32_t* kr = krange;
    if (src_double) {
      if (vec) hipLaunchKernelGGL((k_pack_cols<true, true>), grid, dim3(256), 0, s, X, K, R, ldx, flags, P, ldp, kr);
      else hipLaunchKernelGGL((k_pack_cols<true, false>), grid, dim3(256), 0, s, X, K, R, ldx, flags, P, ldp, kr);
    } else {
      if (vec) hipLaunchKernelGGL((k_pack_cols<false, true>), grid, dim3(256), 0, s, X, K, R, ldx, flags, P, ldp, kr);
      else hipLaunchKernelGGL((k_pack_cols<false, false>), grid, dim3(256), 0, s, X, K, R, ldx, flags, P, ldp, kr);
    }
    return hipGetLastError();
  }
  dim3 grid((unsigned)(krange ? band_chunks : (K + 31) / 32), (unsigned)((R + 63) / 64));
  hipLaunchKernelGGL(k_pack<false>, grid, dim3(256), 0, s, X, src_double, m, n, ldx, flags, P, ldp, krange, nullptr,
                     nullptr);
  return hipGetLastError();
}

hipError_t pack_x3(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P, int64_t ldp,
                   hipStream_t s) {
  return pack_x3_band(X, src_double, m, n, ldx, flags, P, ldp, nullptr, 0, s);
}

hipError_t pack_x3_split_and_plain(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags,
                                   bf16_t* P, int64_t ldp, bf16_t* P2, int64_t ldp2, hipStream_t s) {
  const bool by_rows = flags & PACK_BY_ROWS;
  const int64_t R = by_rows ? m : n, K = by_rows ? n : m;
  if (R <= 0 || K <= 0) return hipSuccess;
  if ((flags & PACK_PLAIN) || ldp < x3_row_stride(K) || ldp2 < x3_plain_stride(K) || ldp2 % 32 != 0)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((K + 31) / 32), (unsigned)((R + 63) / 64));
  hipLaunchKernelGGL(k_pack_dual, grid, dim3(256), 0, s, X, src_double, m, n, ldx, flags, P, ldp, P2, ldp2);
  return hipGetLastError();
}

hipError_t pack_x3_far_gated(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P,
                             int64_t ldp, const int32_t* krange, const unsigned* gate_far, const double* gate_cl,
                             hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (!krange || !gate_far || !gate_cl) return hipErrorInvalidValue;
  if (!(flags & PACK_BY_ROWS)) {
    if (src_double || flags != PACK_PLAIN || ldp < x3_plain_stride(m) || ldp % 8 != 0) return hipErrorInvalidValue;
    const bool vec = ((uintptr_t)X % 16 == 0) && (ldx * 4) % 16 == 0;
    const float* Xf = (const float*)X;
    // a modest grid: when the gate is open (the usual case) every workgroup only reads it
    if (vec)
      hipLaunchKernelGGL(k_pack_plain_far<true>, dim3(1024), dim3(256), 0, s, Xf, m, n, ldx, krange, P, ldp, gate_far,
                         gate_cl);
    else
      hipLaunchKernelGGL(k_pack_plain_far<false>, dim3(1024), dim3(256), 0, s, Xf, m, n, ldx, krange, P, ldp,
                         gate_far, gate_cl);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_pack<true>, dim3(1024), dim3(256), 0, s, X, src_double, m, n, ldx, flags, P, ldp, krange,
                     gate_far, gate_cl);
  return hipGetLastError();
}

}  // namespace pfsm
