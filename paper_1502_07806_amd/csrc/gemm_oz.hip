// Int8 digit GEMM (see gemm_oz.h).  Block tile 256 x 256, 512 threads = 8
// waves (two per SIMD), blocks of v_mfma_i32_32x32x32_i8.  The MFMA takes the
// B fragment first, so a lane's accumulators run along a row of C and one
// register across lanes runs down a column (contiguous column-major
// stores).  The k loop walks every digit pair (p, q) of a weight group back
// to back: the int32 sum of the group is exact, and the epilogue scales it
// by its power of two into FP64.
#include "common.h"
#include "gemm_oz.h"

namespace pfsm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BM = OZ_BM, BN = OZ_BN, BK = OZ_BK;
constexpr int ROWB = BK + 16;        // LDS bytes per operand row
constexpr int TILE = BM * ROWB;      // 36864 bytes per operand per stage

// Tile configurations (all 256 x 256 block tiles, 8 waves, two per SIMD):
//   CFG 0: one launch for all weight groups, direct-to-LDS 4-stage ring,
//          waves in 2 x 4 of 128 x 64 (gemm_oz_fused)
//   CFG 1: CFG 0 with waves in 4 x 2 of 64 x 128
//   CFG 2: one launch per weight group, direct-to-LDS ring (gemm_oz_dl), 4 x 2
//   CFG 3: one launch per weight group, tiles staged through registers into
//          double-buffered LDS (gemm_oz_kernel), 4 x 2
//   CFG 4: CFG 0 with the fragments of the next k32 step read between the
//          MFMAs of the current one
//   CFG 5: all weight groups at once from one staging of every plane
//          (gemm_oz_multi; 128 x 128 block tiles, 8 waves of 64 x 32, a
//          four-slot ring of 32-byte k stages), s = 3 .. 5
//   CFG 6: CFG 5 with a two-slot ring of 64-byte k stages (the default)
// The per-group kernels keep the running sum in C (read-modify-write per
// launch); the fused kernel pays that launch and epilogue cost once per tile.
template <int CFG> struct OzCfg;
template <> struct OzCfg<3> { static constexpr int NT = 512, WGR = 4, WR = 2, WC = 4; };

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

template <int CFG>
__global__ __launch_bounds__(OzCfg<CFG>::NT, 1) void gemm_oz_kernel(OzArgs a, int tiles_m, int tiles_n) {
  constexpr int NT = OzCfg<CFG>::NT, WGR = OzCfg<CFG>::WGR, WR = OzCfg<CFG>::WR, WC = OzCfg<CFG>::WC;
  constexpr int LQ = BM * (BK / 16) / NT;  // 16-byte chunks per thread and operand
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
  const int wi0 = (wave % WGR) * (32 * WR), wj0 = (wave / WGR) * (32 * WC);
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

  const int chunk = tid & 7, rbase = tid >> 3;  // rows rbase + (NT / 8) u
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

// Direct global -> LDS loads (16 bytes per lane, no register
// staging) into a 4-stage ring of 64-byte k tiles, so loads run three tiles
// ahead of the matrix cores.  A wave-wide load fills 1 KB of LDS in lane
// order, i.e. 16 rows of 64 bytes; the lane -> global mapping applies the XOR
// swizzle chunk ^ ((row >> 1) ^ (row >> 2)) & 3, which keeps the fragment
// reads of 8 and of 16 consecutive rows in distinct banks.  Rows past the
// matrix edge read the last row (their outputs are not stored).
constexpr int DBK = 64, DST = 4, DTILE = BM * DBK;  // 16 KB per operand and stage

__device__ inline int dswz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding direct-to-LDS load); the empty asm statements
// keep the compiler from moving LDS accesses across it.
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int WAITS> __device__ inline void wait_vm() {
  // vmcnt = WAITS (0..63); expcnt and lgkmcnt left at their maxima
  __builtin_amdgcn_s_waitcnt((WAITS & 15) | (7 << 4) | (15 << 8) | (((WAITS >> 4) & 3) << 14));
}

template <int NT, int WGR, int WR, int WC>
__global__ __launch_bounds__(NT, 1) void gemm_oz_dl(OzArgs a, int tiles_m, int tiles_n) {
  constexpr int NW = NT / 64;
  constexpr int CPW = 16 / NW;  // 1 KB row groups per wave, operand and stage
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  int tm, tn;
  {
    const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int GROUP = 4;
    const int first_m = (t / (GROUP * tiles_n)) * GROUP;
    const int gsz = min(tiles_m - first_m, GROUP);
    tm = first_m + (t % (GROUP * tiles_n)) % gsz;
    tn = (t % (GROUP * tiles_n)) / gsz;
  }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi0 = (wave % WGR) * (32 * WR), wj0 = (wave / WGR) * (32 * WC);
  const int l32 = lane & 31, lh = lane >> 5;
  const int p_lo = max(1, a.g - a.s);
  const int p_hi = min(a.s, a.g - 1);
  const int ntk = (int)(a.ldp / DBK);
  const int total = (p_hi - p_lo + 1) * ntk;

  int64_t offA[CPW], offB[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int row = 16 * (wave * CPW + j) + (lane >> 2);
    const int c = (lane & 3) ^ dswz(row);
    offA[j] = min<int64_t>(m0 + row, a.M - 1) * a.ldp + 16 * c;
    offB[j] = min<int64_t>(n0 + row, a.N - 1) * a.ldp + 16 * c;
  }
  auto issue = [&](int t) {
    const int pair = t / ntk, kt = t - pair * ntk;
    const int p = p_lo + pair, q = a.g - p;
    const int8_t* A = a.Ap + (int64_t)(p - 1) * a.pa + (int64_t)kt * DBK;
    const int8_t* B = a.Bp + (int64_t)(q - 1) * a.pb + (int64_t)kt * DBK;
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

  v16i acc[WR][WC];
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WC; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

  for (int t = 0; t < DST - 1 && t < total; ++t) issue(t);
  for (int t = 0; t < total; ++t) {
    // tile t has landed once at most min(DST - 2, total - 1 - t) later tiles are outstanding
    const int later = min(DST - 2, total - 1 - t);
    if (later >= 2) wait_vm<2 * 2 * CPW>();
    else if (later == 1) wait_vm<2 * CPW>();
    else wait_vm<0>();
    // Bare barrier: a fenced one would wait for every outstanding load.  After
    // it, every wave's part of tile t is in LDS (each waited for its own
    // loads above) and stage (t - 1) % DST is free (its fragments were
    // consumed by MFMAs before the barrier).
    lds_barrier();
    if (t + DST - 1 < total) issue(t + DST - 1);
    const unsigned char* Ab = lds + (t % DST) * 2 * DTILE;
    const unsigned char* Bb = Ab + DTILE;
#pragma unroll
    for (int sub = 0; sub < DBK / 32; ++sub) {
      const int c = 2 * sub + lh;  // logical 16-byte chunk of this lane's k values
      v4i af[WR], bf[WC];
#pragma unroll
      for (int ib = 0; ib < WR; ++ib) {
        const int row = wi0 + ib * 32 + l32;
        af[ib] = *(const v4i*)(Ab + row * DBK + 16 * (c ^ dswz(row)));
      }
#pragma unroll
      for (int jb = 0; jb < WC; ++jb) {
        const int row = wj0 + jb * 32 + l32;
        bf[jb] = *(const v4i*)(Bb + row * DBK + 16 * (c ^ dswz(row)));
      }
#pragma unroll
      for (int ib = 0; ib < WR; ++ib)
#pragma unroll
        for (int jb = 0; jb < WC; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[jb], af[ib], acc[ib][jb], 0, 0, 0);
    }
  }

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

// One launch for all weight groups.  Each workgroup walks the
// k tiles of every digit pair of every group of its own output tile as one
// sequence through the direct-to-LDS ring (so loads keep running ahead across
// pair and group boundaries), and at the end of each group adds the scaled
// int32 group sum into C (read-modify-write of its own tile only: no other
// workgroup touches it).  Groups run from the smallest weights up.
struct OzCursor {
  int g, p, kt;  // weight group, first digit index of the pair, k tile
};

template <int NT, int WGR, int WR, int WC, bool PIPE>
__global__ __launch_bounds__(NT, 1) void gemm_oz_fused(OzArgs a, int tiles_m, int tiles_n) {
  constexpr int NW = NT / 64;
  constexpr int CPW = 16 / NW;
  constexpr int SUBS = DBK / 32;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  int tm, tn;
  {
    const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int GROUP = 4;
    const int first_m = (t / (GROUP * tiles_n)) * GROUP;
    const int gsz = min(tiles_m - first_m, GROUP);
    tm = first_m + (t % (GROUP * tiles_n)) % gsz;
    tn = (t % (GROUP * tiles_n)) / gsz;
  }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi0 = (wave % WGR) * (32 * WR), wj0 = (wave / WGR) * (32 * WC);
  const int l32 = lane & 31, lh = lane >> 5;
  const int ntk = (int)(a.ldp / DBK);
  const int S = a.s;
  // total k tiles over all groups: s (s + 1) / 2 pairs
  const int total = S * (S + 1) / 2 * ntk;
  auto plo = [&](int g) { return max(1, g - S); };
  auto phi = [&](int g) { return min(S, g - 1); };
  auto advance = [&](OzCursor& c) {
    if (++c.kt == ntk) {
      c.kt = 0;
      if (++c.p > phi(c.g)) {
        --c.g;
        c.p = plo(c.g);
      }
    }
  };

  // Lane offsets inside the tile's rows (32-bit: rows past the edge read the
  // last row), added to a uniform 64-bit base per load: two registers per
  // load instead of four, so nothing in the k loop is spilled (a reload from
  // scratch would wait on the vector-memory counter, i.e. on every load of
  // the ring still in flight).
  uint32_t offA[CPW], offB[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int row = 16 * (wave * CPW + j) + (lane >> 2);
    const int c = (lane & 3) ^ dswz(row);
    offA[j] = (uint32_t)((min<int64_t>(m0 + row, a.M - 1) - m0) * a.ldp + 16 * c);
    offB[j] = (uint32_t)((min<int64_t>(n0 + row, a.N - 1) - n0) * a.ldp + 16 * c);
  }
  auto issue = [&](const OzCursor& c, int t) {
    const int q = c.g - c.p;
    const int8_t* A = a.Ap + (int64_t)(c.p - 1) * a.pa + (int64_t)c.kt * DBK + m0 * a.ldp;
    const int8_t* B = a.Bp + (int64_t)(q - 1) * a.pb + (int64_t)c.kt * DBK + n0 * a.ldp;
    unsigned char* sA = lds + (t % DST) * 2 * DTILE;
    unsigned char* sB = sA + DTILE;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      // opaque 32-bit copies: the address stays (uniform base) + (32-bit lane
      // offset), the scalar-base form of the load, instead of a 64-bit
      // per-lane address kept live across the loop
      uint32_t oa = offA[j], ob = offB[j];
      asm volatile("" : "+v"(oa), "+v"(ob));
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(A + oa),
                                       (void __attribute__((address_space(3)))*)(sA + (wave * CPW + j) * 1024), 16, 0,
                                       0);
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(B + ob),
                                       (void __attribute__((address_space(3)))*)(sB + (wave * CPW + j) * 1024), 16, 0,
                                       0);
    }
  };

  v16i acc[WR][WC];
  auto zero = [&]() {
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
  };
  // Scaled group sum into C: stored by the first group, then added by
  // no-return FP64 atomics, which need no registers or round trip for the
  // old value (a read-modify-write would wait for every load, as C elements
  // could alias as far as the compiler knows).  Each element is updated by
  // one thread only, in program order, so the sums are the same as with
  // plain loads and stores.
  // The exponents of the tile's rows and columns sit in LDS: a global load
  // there would wait for every atomic issued before it (one vmcnt counter).
  __shared__ int s_ea[BM], s_eb[BN];
  for (int i = tid; i < BM; i += NT) s_ea[i] = a.ea[min<int64_t>(m0 + i, a.M - 1)];
  for (int j = tid; j < BN; j += NT) s_eb[j] = a.eb[min<int64_t>(n0 + j, a.N - 1)];
  __syncthreads();
  auto flush = [&](int g, bool first) {
    const int shift = -12 - 7 * (g - 2);
    // opaque copy of ldc: keeps the compiler from hoisting every output
    // address out of the k loop into registers
    int64_t ldc = a.ldc;
    asm volatile("" : "+s"(ldc));
#pragma unroll
    for (int ib = 0; ib < WR; ++ib) {
      const int64_t gi = m0 + wi0 + ib * 32 + l32;
      if (gi >= a.M) continue;
      const int ei = s_ea[wi0 + ib * 32 + l32] + shift;
#pragma unroll
      for (int jb = 0; jb < WC; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int jl = wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
          const int64_t gj = n0 + jl;
          if (gj >= a.N) continue;
          const double v = ldexp((double)acc[ib][jb][r], ei + s_eb[jl]);
          double* cp = a.C + gi + gj * ldc;
          if (first) *cp = v;
          else unsafeAtomicAdd(cp, v);
          if (r % 8 == 7) __builtin_amdgcn_sched_barrier(0);  // bounds the registers the scheduler may hoist into
        }
    }
  };
  zero();

  struct Frags {
    v4i af[SUBS][WR], bf[SUBS][WC];
  };
  auto read_frags = [&](int t, Frags& f) {
    const unsigned char* Ab = lds + (t % DST) * 2 * DTILE;
    const unsigned char* Bb = Ab + DTILE;
#pragma unroll
    for (int sub = 0; sub < SUBS; ++sub) {
      const int c = 2 * sub + lh;
#pragma unroll
      for (int ib = 0; ib < WR; ++ib) {
        const int row = wi0 + ib * 32 + l32;
        f.af[sub][ib] = *(const v4i*)(Ab + row * DBK + 16 * (c ^ dswz(row)));
      }
#pragma unroll
      for (int jb = 0; jb < WC; ++jb) {
        const int row = wj0 + jb * 32 + l32;
        f.bf[sub][jb] = *(const v4i*)(Bb + row * DBK + 16 * (c ^ dswz(row)));
      }
    }
  };
  auto mma = [&](const Frags& f) {
#pragma unroll
    for (int sub = 0; sub < SUBS; ++sub)
#pragma unroll
      for (int ib = 0; ib < WR; ++ib)
#pragma unroll
        for (int jb = 0; jb < WC; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.bf[sub][jb], f.af[sub][ib], acc[ib][jb], 0, 0, 0);
  };

  OzCursor cc = {S + 1, plo(S + 1), 0};  // compute cursor
  OzCursor ic = cc;                       // issue cursor
  for (int t = 0; t < DST - 1 && t < total; ++t) {
    issue(ic, t);
    advance(ic);
  }
  auto group_end = [&]() {  // after the MFMAs of the current k tile
    const int g = cc.g;
    advance(cc);
    if (cc.g != g || cc.g < 2) {  // group g complete
      flush(g, g == S + 1);
      zero();
    }
  };
  if (!PIPE) {
    for (int t = 0; t < total; ++t) {
      const int later = min(DST - 2, total - 1 - t);
      if (later >= 2) wait_vm<2 * 2 * CPW>();
      else if (later == 1) wait_vm<2 * CPW>();
      else wait_vm<0>();
      lds_barrier();  // as in gemm_oz_dl
      if (t + DST - 1 < total) {
        issue(ic, t + DST - 1);
        advance(ic);
      }
      Frags f;
      read_frags(t, f);
      mma(f);
      group_end();
    }
  } else if (total > 0) {
    // Fragments one k32 step ahead, read between the MFMAs of the current
    // one (see the split-BF16 kernel).  Sub-step 0 of tile t prefetches
    // sub-step 1 of the same tile; before sub-step 1 the barrier makes tile
    // t + 1 visible, and its first fragments are read during sub-step 1.
    // The slot refilled at that barrier, (t + 3) % 4, held tile t - 1, whose
    // last fragments were read before it.  Flush atomics also count in
    // vmcnt; issued after the loads being waited for, they only make the
    // waits more conservative.
    static_assert(SUBS == 2, "two k32 steps per k tile");
    {
      const int later0 = min(DST - 2, total - 1);
      if (later0 >= 2) wait_vm<2 * 2 * CPW>();
      else if (later0 == 1) wait_vm<2 * CPW>();
      else wait_vm<0>();
      lds_barrier();
    }
    struct Sub {
      v4i af[WR], bf[WC];
    };
    auto read_sub = [&](int t, int sub, Sub& f) {
      const unsigned char* Ab = lds + (t % DST) * 2 * DTILE;
      const unsigned char* Bb = Ab + DTILE;
      const int c = 2 * sub + lh;
#pragma unroll
      for (int ib = 0; ib < WR; ++ib) {
        const int row = wi0 + ib * 32 + l32;
        f.af[ib] = *(const v4i*)(Ab + row * DBK + 16 * (c ^ dswz(row)));
      }
#pragma unroll
      for (int jb = 0; jb < WC; ++jb) {
        const int row = wj0 + jb * 32 + l32;
        f.bf[jb] = *(const v4i*)(Bb + row * DBK + 16 * (c ^ dswz(row)));
      }
    };
    auto mma_sub = [&](const Sub& f) {
#pragma unroll
      for (int ib = 0; ib < WR; ++ib)
#pragma unroll
        for (int jb = 0; jb < WC; ++jb)
          acc[ib][jb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.bf[jb], f.af[ib], acc[ib][jb], 0, 0, 0);
    };
    auto interleave = [&]() {
#pragma unroll
      for (int u = 0; u < WR + WC; ++u) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, WR * WC - (WR + WC), 0);
    };
    Sub F0, F1;
    read_sub(0, 0, F0);
    for (int t = 0; t < total; ++t) {
      __builtin_amdgcn_sched_barrier(0);
      read_sub(t, 1, F1);
      mma_sub(F0);
      interleave();
      __builtin_amdgcn_sched_barrier(0);
      if (t + 1 < total) {
        if (t + 2 <= total - 1) wait_vm<2 * CPW>();
        else wait_vm<0>();
        lds_barrier();
        if (t + DST - 1 < total) {
          issue(ic, t + DST - 1);
          advance(ic);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      read_sub(t + 1, 0, F0);  // past the last tile: a stale slot, never used
      mma_sub(F1);
      interleave();
      __builtin_amdgcn_sched_barrier(0);
      group_end();
    }
  }
}

// All weight groups at once.  The fused kernel above walks the digit pairs one
// after the other: every plane is staged and read from LDS once per pair it
// takes part in (s times for the first planes).  Here a workgroup of eight
// waves (128 x 128 block tile, 64 x 32 per wave) stages the k32 slice of all s
// planes of both operands once, reads each plane's fragments once and issues
// every pair (p, q), p + q <= s + 1, from them into the int32 accumulator of
// its weight group.  The s group sums (s x 32 registers a lane) are scaled and
// added in FP64 at the end, smallest weights first: the same additions in the
// same order as the fused kernel's store and atomic adds, so C is the same bit
// for bit, and it is written once.
constexpr int MT = 128;

// Stage of MBK k bytes per row (32 or 64), MST = 128 KB / ... stages in the ring.
// 32-byte rows: the two 16-byte chunks of rows 8..15 (mod 16) swap places; 64-byte
// rows: chunk c of row r sits at c ^ dswz(r).  Either way the fragment reads of
// 16 consecutive rows cover all 64 banks once.
template <int MBK> __device__ inline int mswz(int r) { return MBK == 32 ? (r >> 3) & 1 : dswz(r); }
template <int MBK> constexpr int multi_stages(int S) { return (MBK == 32 ? 4 : 2) + 0 * S; }

template <int S, int MBK>
__global__ __launch_bounds__(512, 1) void gemm_oz_multi(OzArgs a, int tiles_m, int tiles_n) {
  constexpr int WR = 2, WC = 1;          // 32 x 32 blocks per wave: 64 x 32
  constexpr int MPLANE = MT * MBK;       // the k slice of one plane of one operand
  constexpr int MST = multi_stages<MBK>(S);
  constexpr int STAGE = 2 * S * MPLANE;  // A planes, then B planes
  constexpr int RG = MT * MBK / 1024;    // 1 KB row groups per plane
  constexpr int LPW = 2 * S * RG / 8;    // 1 KB loads per wave and stage
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  int64_t m0, n0;
  {
    const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int GROUP = 4;
    const int first_m = (t / (GROUP * tiles_n)) * GROUP;
    const int gsz = min(tiles_m - first_m, GROUP);
    m0 = (int64_t)(first_m + (t % (GROUP * tiles_n)) % gsz) * MT;
    n0 = (int64_t)((t % (GROUP * tiles_n)) / gsz) * MT;
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi0 = (wave & 1) * 64, wj0 = (wave >> 1) * 32;
  const int l32 = lane & 31, lh = lane >> 5;
  const int ntk = (int)(a.ldp / MBK);
  // Wave w stages row group w % 4 (rows 32 (w % 4) .. + 31) of the planes
  // w / 4, w / 4 + 2, ... of the list A_1 .. A_s, B_1 .. B_s: lane L holds row
  // 32 (w % 4) + L / 2, stored chunk L % 2.  Rows past the edge read the last
  // row (their outputs are not stored).
  // (32-byte rows: wave w stages row group w % 4 of the planes w / 4, w / 4 + 2, ...;
  // 64-byte rows: row group w of every plane, lane L holding row 16 w + L / 4)
  const int rg = wave % RG, po0 = wave / RG, pstep = 8 / RG;
  uint32_t offA, offB;
  {
    constexpr int LPR = MBK / 16;  // lanes per row
    const int row = (1024 / MBK) * rg + lane / LPR;
    const int c = (lane % LPR) ^ mswz<MBK>(row);
    offA = (uint32_t)((min<int64_t>(m0 + row, a.M - 1) - m0) * a.ldp + 16 * c);
    offB = (uint32_t)((min<int64_t>(n0 + row, a.N - 1) - n0) * a.ldp + 16 * c);
  }
  auto issue = [&](int kt) {
    unsigned char* st = lds + (kt % MST) * STAGE + rg * 1024;
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const int po = po0 + pstep * i;  // wave-uniform
      const bool isA = po < S;
      const int8_t* base = isA ? a.Ap + (int64_t)po * a.pa + m0 * a.ldp : a.Bp + (int64_t)(po - S) * a.pb + n0 * a.ldp;
      uint32_t o = isA ? offA : offB;
      asm volatile("" : "+v"(o));  // keep the scalar-base load form (see gemm_oz_fused)
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(base + (int64_t)kt * MBK + o),
                                       (void __attribute__((address_space(3)))*)(st + po * MPLANE), 16, 0, 0);
    }
  };

  v16i acc[S][WR][WC];  // acc[g - 2]: weight group g
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[g][i][j][r] = 0;

  for (int t = 0; t < MST - 1 && t < ntk; ++t) issue(t);
  for (int t = 0; t < ntk; ++t) {
    // this wave's part of stage t has landed once at most the loads of the
    // later stages already issued are outstanding
    const int later = min(MST - 2, ntk - 1 - t);
    static_assert(MST <= 4, "wait counts below");
    if (later >= 2) wait_vm<2 * LPW>();
    else if (later == 1) wait_vm<LPW>();
    else wait_vm<0>();
    // After the barrier every wave's part of stage t is in LDS, and the slot of
    // stage t - 1 is free (its fragments fed MFMAs before the barrier).
    lds_barrier();
    if (t + MST - 1 < ntk) issue(t + MST - 1);
    const unsigned char* st = lds + (t % MST) * STAGE;
#pragma unroll
    for (int sub = 0; sub < MBK / 32; ++sub) {
    v4i af[S][WR], bf[S][WC];
    const int c = 2 * sub + lh;
#pragma unroll
    for (int p = 0; p < S; ++p) {
#pragma unroll
      for (int ib = 0; ib < WR; ++ib) {
        const int row = wi0 + ib * 32 + l32;
        af[p][ib] = *(const v4i*)(st + p * MPLANE + row * MBK + 16 * (c ^ mswz<MBK>(row)));
      }
#pragma unroll
      for (int jb = 0; jb < WC; ++jb) {
        const int row = wj0 + jb * 32 + l32;
        bf[p][jb] = *(const v4i*)(st + (S + p) * MPLANE + row * MBK + 16 * (c ^ mswz<MBK>(row)));
      }
    }
    // pairs in order of their larger digit index, so the first MFMAs need only
    // the first fragments read
#pragma unroll
    for (int mx = 1; mx <= S; ++mx)
#pragma unroll
      for (int p = 1; p <= S; ++p)
#pragma unroll
        for (int q = 1; q <= S; ++q) {
          if (p + q > S + 1 || (p > q ? p : q) != mx) continue;
#pragma unroll
          for (int ib = 0; ib < WR; ++ib)
#pragma unroll
            for (int jb = 0; jb < WC; ++jb)
              acc[p + q - 2][ib][jb] =
                  __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[q - 1][jb], af[p - 1][ib], acc[p + q - 2][ib][jb], 0, 0, 0);
        }
    }
  }

  // acc[g - 2][ib][jb][r] is group g's sum for C(i, j), i = wi0 + 32 ib + lane % 32,
  // j = wj0 + 32 jb + 8 (r / 4) + 4 (lane / 32) + r % 4.
#pragma unroll
  for (int ib = 0; ib < WR; ++ib) {
    const int64_t gi = m0 + wi0 + ib * 32 + l32;
    if (gi >= a.M) continue;
    const int ei = a.ea[gi];
#pragma unroll
    for (int jb = 0; jb < WC; ++jb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gj = n0 + wj0 + jb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
        if (gj >= a.N) continue;
        const int e = ei + a.eb[gj];
        double v = ldexp((double)acc[S - 1][ib][jb][r], e - 12 - 7 * (S - 1));  // group S + 1
#pragma unroll
        for (int g = S; g >= 2; --g) v += ldexp((double)acc[g - 2][ib][jb][r], e - 12 - 7 * (g - 2));
        a.C[gi + gj * a.ldc] = v;
      }
  }
}

// One block per column: exponent of the column maximum, then the digits of
// four consecutive k per thread (one 32-bit word per plane).  Columns of up
// to 256 * 4 * SPLIT_REG entries are read once, into registers, with 16-byte
// loads all in flight together; longer ones are read twice.
constexpr int SPLIT_REG = 8;

__device__ inline void oz_digits_store(double (&t)[4], int s, int8_t* out, int64_t pstride) {
  for (int p = 0; p < s; ++p) {
    uint32_t word = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double d = rint(t[u]);  // |d| <= 64, |t - d| <= 1/2
      word |= ((uint32_t)(int)d & 0xffu) << (8 * u);
      t[u] = (t[u] - d) * 128.0;
    }
    *(uint32_t*)(out + p * pstride) = word;
  }
}

__global__ __launch_bounds__(256) void k_oz_split(const double* X, int64_t ldx, int64_t K, int64_t ldp,
                                                  int64_t pstride, int s, int8_t* P, int* expo, int* info) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x;
  const double* x = X + c * ldx;
  const int tid = threadIdx.x;
  const int64_t nch = (ldp + 1023) / 1024;  // chunks of 4 entries per thread
  const bool in_regs = nch <= SPLIT_REG;
  // 16-byte loads need an even leading dimension and a 16-byte aligned base
  const bool vec = ((ldx & 1) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  double r[SPLIT_REG][4];
  double m = 0.0;
  if (in_regs) {
#pragma unroll
    for (int j = 0; j < SPLIT_REG; ++j) {
      const int64_t k4 = 4 * (int64_t)tid + 1024 * (int64_t)j;
      if (vec && k4 + 4 <= K) {
        const double2 a = *(const double2*)(x + k4), b = *(const double2*)(x + k4 + 2);
        r[j][0] = a.x; r[j][1] = a.y; r[j][2] = b.x; r[j][3] = b.y;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) r[j][u] = (k4 + u < K) ? x[k4 + u] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < SPLIT_REG; ++j)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double v = fabs(r[j][u]);
        m = (v > m || v != v) ? v : m;
      }
  } else {
    for (int64_t k = tid; k < K; k += 256) {
      const double v = fabs(x[k]);
      m = (v > m || v != v) ? v : m;
    }
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
  if (in_regs) {
#pragma unroll
    for (int j = 0; j < SPLIT_REG; ++j) {
      const int64_t k4 = 4 * (int64_t)tid + 1024 * (int64_t)j;
      if (k4 >= ldp) break;
      double t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] = (!bad && k4 + u < K) ? ldexp(r[j][u], 6 - e) : 0.0;  // |t| < 64
      oz_digits_store(t, s, out + k4, pstride);
    }
    return;
  }
  for (int64_t k4 = 4 * (int64_t)tid; k4 < ldp; k4 += 4 * 256) {
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = (!bad && k4 + u < K) ? ldexp(x[k4 + u], 6 - e) : 0.0;  // |t| < 64
    oz_digits_store(t, s, out + k4, pstride);
  }
}


template <int S, int MBK> constexpr int multi_lds() { return multi_stages<MBK>(S) * 2 * S * MT * MBK; }
template <int S, int MBK> hipError_t oz_multi_init() {
  return hipFuncSetAttribute((const void*)gemm_oz_multi<S, MBK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             multi_lds<S, MBK>());
}
template <int S, int MBK> void oz_multi_launch(const OzArgs& a, hipStream_t st) {
  const int tm = (int)((a.M + MT - 1) / MT), tn = (int)((a.N + MT - 1) / MT);
  constexpr int lds = multi_lds<S, MBK>();
  hipLaunchKernelGGL((gemm_oz_multi<S, MBK>), dim3((unsigned)(tm * tn)), dim3(512), lds, st, a, tm, tn);
}

}  // namespace

int oz_default_cfg = 6;  // fastest measured at N = 8192 (configuration 4 where s is outside 3 .. 5)

hipError_t oz_init() {
  hipError_t e = hipFuncSetAttribute((const void*)gemm_oz_kernel<3>, hipFuncAttributeMaxDynamicSharedMemorySize, 4 * TILE);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)gemm_oz_dl<512, 4, 2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            DST * 2 * DTILE);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)gemm_oz_fused<512, 2, 4, 2, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            DST * 2 * DTILE);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)gemm_oz_fused<512, 4, 2, 4, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            DST * 2 * DTILE);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)gemm_oz_fused<512, 2, 4, 2, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            DST * 2 * DTILE);
  if (e == hipSuccess) e = oz_multi_init<3, 32>();
  if (e == hipSuccess) e = oz_multi_init<4, 32>();
  if (e == hipSuccess) e = oz_multi_init<5, 32>();
  if (e == hipSuccess) e = oz_multi_init<3, 64>();
  if (e == hipSuccess) e = oz_multi_init<4, 64>();
  if (e == hipSuccess) e = oz_multi_init<5, 64>();

  return e;
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
                   const int* eb, double* C, int64_t ldc, hipStream_t st, int cfg) {
  if (cfg < 0) cfg = oz_default_cfg;
  if (cfg > 6) return hipErrorInvalidValue;
  if (cfg >= 5 && (s < 3 || s > 5)) cfg = 4;  // the all-groups kernels are built for 3 to 5 digits
  if (s < 1 || s > OZ_MAX_SLICES || K < 0 || (int64_t)s * K >= (1 << 19)) return hipErrorInvalidValue;
  if (M <= 0 || N <= 0) return hipSuccess;
  OzArgs a = {};
  a.M = M; a.N = N; a.ldp = oz_row_stride(K); a.pa = M * a.ldp; a.pb = N * a.ldp;
  a.Ap = Ap; a.Bp = Bp; a.ea = ea; a.eb = eb; a.C = C; a.ldc = ldc; a.s = s;
  a.ntk = (int)(a.ldp / BK);
  const int tm = (int)((M + BM - 1) / BM), tn = (int)((N + BN - 1) / BN);
  const dim3 grid((unsigned)(tm * tn));
  if (cfg == 0) {
    hipLaunchKernelGGL((gemm_oz_fused<512, 2, 4, 2, false>), grid, dim3(512), DST * 2 * DTILE, st, a, tm, tn);
    return hipGetLastError();
  }
  if (cfg == 1) {
    hipLaunchKernelGGL((gemm_oz_fused<512, 4, 2, 4, false>), grid, dim3(512), DST * 2 * DTILE, st, a, tm, tn);
    return hipGetLastError();
  }
  if (cfg == 4) {
    hipLaunchKernelGGL((gemm_oz_fused<512, 2, 4, 2, true>), grid, dim3(512), DST * 2 * DTILE, st, a, tm, tn);
    return hipGetLastError();
  }
  if (cfg == 5) {
    if (s == 3) oz_multi_launch<3, 32>(a, st);
    else if (s == 4) oz_multi_launch<4, 32>(a, st);
    else oz_multi_launch<5, 32>(a, st);
    return hipGetLastError();
  }
  if (cfg == 6) {
    if (s == 3) oz_multi_launch<3, 64>(a, st);
    else if (s == 4) oz_multi_launch<4, 64>(a, st);
    else oz_multi_launch<5, 64>(a, st);
    return hipGetLastError();
  }

  for (int g = s + 1; g >= 2; --g) {  // smallest weights first
    a.g = g;
    a.first = (g == s + 1);
    if (cfg == 2)
      hipLaunchKernelGGL((gemm_oz_dl<512, 4, 2, 4>), grid, dim3(512), DST * 2 * DTILE, st, a, tm, tn);
    else
      hipLaunchKernelGGL(gemm_oz_kernel<3>, grid, dim3(512), 4 * TILE, st, a, tm, tn);
  }
  return hipGetLastError();
}

}  // namespace pfsm
