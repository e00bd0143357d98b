// BF16 hi/lo split ("x3") GEMM on CDNA4 matrix cores and its operand packing.
//
// A real matrix x is carried as two bfloat16 planes, hi = bf16(x) and
// lo = bf16(x - hi); a product uses hi*hi + hi*lo + lo*hi with FP32
// accumulation (v_mfma_f32_32x32x16_bf16), about 16 significant bits per
// product term instead of BF16's 8.
//
// Packed operand layout: for an operand with rows r (output index) and
// reduction index k, row r holds ceil(K/32) chunks of 64 bf16 values:
// [32 hi values | 32 lo values] for k = 32c .. 32c+31 (zero-filled past K).
// Row stride = 64 * ceil(K/32) bf16 (128 bytes per chunk).  Both GEMM operands
// use this layout: op(A) by its rows i, op(B) by its columns j.
#pragma once
#include "common.h"

namespace pfsm {

typedef unsigned short bf16_t;

constexpr int X3_BM = 256, X3_BN = 256, X3_BK = 32;

inline int64_t x3_row_stride(int64_t K) { return 64 * ((K + 31) / 32); }

enum X3Epi : int {
  X3_STORE = 0,  // C = alpha*acc + beta*C
  X3_SHIFT = 1,  // C = acc - B32(i,j) * eps[j]                (FP32 out)
  X3_FSUPD = 2,  // C = D32(i,j) - a*(acc - B32(i,j)*eps[j])    (FP32 out)
  X3_ADD = 3,    // C = alpha*acc + D(i,j)   (D float or double)
  X3_RQ = 4,     // part[tile_m][j] = sum_i acc(i,j) * D32(i,j)
  X3_STORE_PACK = 5,  // alpha*acc written only as its split BF16 packed copy (pack_split)
};

// LOWER: only tiles with tile row >= tile column (square C); KPREFIX: the k
// range of column tile j ends at its last column (op(B) upper triangular).
enum X3Tiles : int { X3_FULL = 0, X3_LOWER = 1, X3_KPREFIX = 3 };

struct X3Args {
  int64_t M, N, K;
  const bf16_t* Ap; int64_t ldap;   // packed rows of op(A)
  const bf16_t* Bp; int64_t ldbp;   // packed columns of op(B)
  void* C; int64_t ldc; int c_double;
  double alpha, beta;
  const float* B32; int64_t ldb32;  // unpacked op(B) for SHIFT / FSUPD (FP32, column-major)
  const void* D; int64_t ldd; int d_double;  // FSUPD / ADD / RQ partner
  const double* eps;
  const double* alpha_dev;
  double* part;
  const int32_t* krange;            // optional [tiles_n][2] (multiples of 32)
  int tiles;                        // X3Tiles
  int kprefix_skip;                 // unused
  int cfg;                          // tile configuration (see gemm_x3.hip); -1 = library default
  // Optional scratch (x3_split_bytes(M) bytes, device) for X3_LOWER STORE
  // products: the tiles of a last, mostly empty wave of workgroups are split
  // along K over the whole chip and summed by a second kernel.
  float* split_ws; size_t split_bytes;
  int split_full, split_s;          // set inside gemm_x3
  // 0 or 3: hi*hi + hi*lo + lo*hi from the split layout; 1 (SHIFT, FSUPD and
  // ADD, not LOWER tiles): one BF16 product from operands in the plain layout (PACK_PLAIN,
  // ldap / ldbp = their row strides), FP32 accumulation, in the direct-to-LDS
  // configuration whatever cfg says
  int products;
  // Band form of the folded-spectrum products (SHIFT / FSUPD).  diag: the
  // diagonal d of the left operand's matrix (FP64, d_i = diag[i * diag_stride]);
  // the product itself then runs on the off-diagonal part, and the epilogue
  // adds (d_i - eps_j) b_ij.
  const double* diag; int64_t diag_stride;
  // far_krange / farmax_out: the largest |output| over the rows outside the
  // K range far_krange gives the output's column tile, folded into
  // *farmax_out (the bits of a non-negative float, atomic max).
  const int32_t* far_krange; unsigned* farmax_out;
  // Gate (optional): with m = *gate_far (a float's bits) and gate_cl = {c,
  // limit} (device), the terms a K-range-restricted product drops, bounded by
  // c m, are negligible when c m <= limit; the kernel runs only when that
  // test equals gate_band (NaN: the test fails).  band_count (optional)
  // counts the launches of the band form that ran.
  const unsigned* gate_far; const double* gate_cl; int gate_band; unsigned* band_count;
  // Optional [tiles_m][2] K range per row tile of C (multiples of 32),
  // intersected with the column tiles' range.
  const int32_t* krange_rows;
  // STORE_PACK (all tiles, M a multiple of 32): the output of pack_x3
  // (without PACK_PLAIN) for the FP32-rounded product, row j = column j of the
  // product, row stride ld_pack_split; C is not written.
  bf16_t* pack_split; int64_t ld_pack_split;
};

constexpr int X3_NUM_CFG = 6;
extern int x3_default_cfg;
hipError_t x3_init();  // once per process and device, before the first split-BF16 launch

hipError_t gemm_x3(int epi, const X3Args& a, hipStream_t s);
// Scratch bytes that let an order-n X3_LOWER product split its last wave (0:
// no split at this order).  Valid after x3_init.
size_t x3_split_bytes(int64_t n);

// Packing.  Without PACK_BY_ROWS, row r of the packed operand is column r of X
// (k runs down the column); with it, row r is row r of X (a transpose).  X is
// column-major with ld; src_double selects FP64 or FP32 storage.
// PACK_SUB_I packs X - I; PACK_LOWER / PACK_UPPER keep only the lower / upper
// triangle of X (row >= col / row <= col), zeros elsewhere; PACK_HALF_DIAG
// halves the diagonal (after PACK_SUB_I); PACK_OFFDIAG zeroes it.
// PACK_PLAIN writes the plain layout: row r holds bf16(x) for k = 0 .. K-1
// contiguously (no lo values), zero-filled to a multiple of 32, row stride at
// least x3_plain_stride(K).
enum PackFlags : int { PACK_BY_ROWS = 1, PACK_SUB_I = 2, PACK_LOWER = 4, PACK_UPPER = 8, PACK_HALF_DIAG = 16,
                       PACK_PLAIN = 32, PACK_OFFDIAG = 64 };

inline int64_t x3_plain_stride(int64_t K) { return 32 * ((K + 31) / 32); }
hipError_t pack_x3(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P, int64_t ldp,
                   hipStream_t s);

// The split layout into P and the plain one (PACK_PLAIN) into P2 from one
// read of X (transposing packs: the plain values are the split hi parts).
hipError_t pack_x3_split_and_plain(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags,
                                   bf16_t* P, int64_t ldp, bf16_t* P2, int64_t ldp2, hipStream_t s);
// The same as pack_x3, restricted to the K range krange[2 t], krange[2 t + 1] (multiples
// of 32) of each 256-row tile t of the packed operand (its rows r, t = r / 256):
// the band part, all that a product with that K range per tile reads
// (X3Args::krange for a column operand, krange_rows for a row operand).
// band_chunks: at least the widest range / 32.
hipError_t pack_x3_band(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P,
                        int64_t ldp, const int32_t* krange, int band_chunks, hipStream_t s);
// The far part: every k outside those ranges (zero padding included), written
// only when the gate {gate_far, gate_cl} of X3Args is closed for the band
// form, i.e. when the full form of the product will run.  Column operands:
// plain layout from FP32 only.
hipError_t pack_x3_far_gated(const void* X, int src_double, int64_t m, int64_t n, int64_t ldx, int flags, bf16_t* P,
                             int64_t ldp, const int32_t* krange, const unsigned* gate_far, const double* gate_cl,
                             hipStream_t s);

}  // namespace pfsm
