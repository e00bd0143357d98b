// Batched FP64 eigensolver for the PFSM submatrices (block Jacobi).
//
// Each submatrix B_p (order M_p <= Mp) is padded to Mp = multiple of 2b with
// decoupled diagonal entries PAD_DIAG (which sort above every true
// eigenvalue), and diagonalised by a two-sided block-cyclic Jacobi method:
//
//   for each sweep, for each round of a round-robin tournament over the
//   nb = Mp/b column blocks:
//     solve   (one workgroup per block pair (I,J)): the 2b x 2b matrix
//             [B_II B_IJ; B_JI B_JJ] is diagonalised in LDS by a scalar
//             parallel-order cyclic Jacobi, giving an orthogonal R_IJ;
//     apply   (one workgroup per 2b x 2b tile): B <- J^T B J and U <- U J
//             with J = diag of the R's, as small MFMA products in LDS; the
//             U tiles of a round run in the same launch as the next round's
//             pair problems (nothing reads U in between).
//
// (The pair problem is solved by a one-sided Jacobi, see solve_pair.)
// A sweep in which no pair needed a rotation marks the submatrix converged;
// later kernels of that submatrix return immediately.  A pair (p, q) is
// rotated when |b_pq| > 2^-53 sqrt(|b_pp b_qq|) (relative accuracy) and
// |b_pq| > 256 * 2^-53 * ||B|| (rounding floor of the block products, with
// ||B|| bounded by the Gershgorin interval of the full matrix).  Without the
// floor, the rounding error of the MFMA block updates would keep rotating
// exactly degenerate pairs forever.  A caller that rounds the eigenvectors
// to a shorter format raises the floor (EighBatch::floor_rel).
#include "common.h"
#include "eigh.h"
#include "order_key.h"

namespace pfsm {
namespace {

constexpr int NT = 256;
constexpr int B2 = 2 * EIGH_B;   // 64: order of a pair problem / apply tile
constexpr int LS = B2 + 1;       // LDS row stride
constexpr double TOL = 1.1102230246251565e-16;  // 2^-53
constexpr double TINY = 1e-300;
constexpr double NOISE = 256.0 * TOL;
// A pair-solver sweep whose rotations all had |sin| <= ANGLE ends the
// iteration: Jacobi converges quadratically, so the inner products left after
// such a sweep are of order ANGLE^2 relative (1e-16, below the 8u test), and
// the sweep that would only confirm it is skipped.  The column norms of
// W = S + sigma I differ by a factor of at most about 3, so small angles do
// mean small relative inner products.
constexpr double ANGLE = 1e-8;

// Gershgorin scalars and info word of submatrix p (its own instance's when
// several instances are solved together).
__device__ inline const double* scal_of(const EighBatch& e, int p) {
  return e.scal_off ? (const double*)(e.wbase + e.scal_off[p]) : e.scal;
}
__device__ inline int* info_of(const EighBatch& e, int p) {
  return e.info_idx ? e.info_base + e.info_idx[p] : e.info;
}
__device__ inline double noise_floor(const EighBatch& e, int p) {
  const double* sc = scal_of(e, p);
  return fmax(NOISE, e.floor_rel) * fmax(fmax(fabs(sc[1]), fabs(sc[2])), TINY);
}
__device__ inline bool must_rotate(double apq, double app, double aqq, double floor_abs) {
  double a = fabs(apq);
  return a > floor_abs && a > TOL * sqrt(fabs(app) * fabs(aqq));
}

// Pair rotations and their flags of a round: two buffers, by round parity, so
// that the eigenvector update of round r can run beside the pair problems of
// round r + 1.
__device__ inline double* rot_buf(const EighBatch& e, int round) {
  return e.Rw + (int64_t)(round & 1) * e.P * (e.nb / 2) * B2 * B2;
}
__device__ inline int* flag_buf(const EighBatch& e, int round) {
  return e.rflag + (int64_t)(round & 1) * e.P * (e.nb / 2);
}

// Circle-method tournament: position -> block index in round r (n even).
__device__ __host__ inline int rr_index(int pos, int r, int n) {
  if (pos == 0) return 0;
  return ((pos - 1 + r) % (n - 1)) + 1;
}
__device__ inline void pair_blocks(int k, int r, int nb, int& I, int& J) {
  int a = rr_index(k, r, nb), b = rr_index(nb - 1 - k, r, nb);
  I = min(a, b);
  J = max(a, b);
}
// global index (within the padded submatrix) of local index t in [0, 2b) of pair (I, J)
__device__ inline int pair_idx(int t, int I, int J) { return t < EIGH_B ? I * EIGH_B + t : J * EIGH_B + (t - EIGH_B); }

// ------------------------------------------------------------------ gather
template <typename T>
__global__ void gather_windows(EighBatch e, const T* __restrict__ At, int64_t ldat) {
  const int p = blockIdx.y;
  if (e.src_off) {  // this submatrix's own instance
    At = (const T*)(e.wbase + e.src_off[p]);
    ldat = e.src_ld[p];
  }
  const int Mp = e.Mp;
  const int64_t w0 = e.wstart[p];
  const int M = e.wsize[p];
  double* B = e.Bw + (int64_t)p * Mp * Mp;
  double* U = e.Uw + (int64_t)p * Mp * Mp;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)Mp * Mp;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(idx % Mp), c = (int)(idx / Mp);
    double v;
    if (r < M && c < M) v = (double)At[(w0 + r) + (w0 + c) * ldat];
    else v = (r == c) ? EIGH_PAD_DIAG : 0.0;
    B[idx] = v;
    U[idx] = (r == c) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    e.state[2 * p] = 0;      // done flag
    e.state[2 * p + 1] = 0;  // rotations in current sweep
    e.stats[2 * p] = 0;      // sweep at which the submatrix was found converged
    e.stats[2 * p + 1] = 0;  // pair problems that needed rotations, all sweeps
  }
}

// Start of a sweep: a submatrix whose previous sweep needed no rotation is done.
__global__ void sweep_begin(EighBatch e, int sweep) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= e.P) return;
  if (sweep > 0 && e.state[2 * p + 1] == 0 && !e.state[2 * p]) {
    e.state[2 * p] = 1;
    e.stats[2 * p] = sweep;
  }
  e.state[2 * p + 1] = 0;
}

// ------------------------------------------------------------------ pair solve
// Sum over the 8 lanes of an aligned lane group with DPP moves (no LDS
// round trip): quad_perm [1,0,3,2], quad_perm [2,3,0,1], then the half-row
// mirror (lane i <-> 7 - i) pairs the two quads.  Every lane of the group
// ends with the bitwise same sum (IEEE addition is commutative), so lanes
// that decide on a rotation independently always agree.
template <int CTRL> __device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double sum8(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  return v;
}
// Sum over an aligned group of 16 lanes: the 8-lane sums, then the row mirror
// (lane i <-> 15 - i) adds the other half (bitwise the same in every lane).
__device__ inline double sum16(double v) {
  v = sum8(v);
  v += dpp_d<0x140>(v);
  return v;
}
// The pair solver gives each column pair PL lanes of B2 / PL rows each;
// a workgroup has PS_NT = 32 PL threads.
constexpr int PL = 16;
constexpr int PS_NT = 32 * PL;
__device__ inline double sum_pl(double v) { return PL == 16 ? sum16(v) : sum8(v); }
// Reciprocal and reciprocal square root: the hardware estimates (relative
// error about 5e-8) refined by two Newton steps, which converge
// quadratically to one or two ulps (measured: 1.9e-16 and 2.3e-16).
__device__ inline double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) r = r * (2.0 - x * r);
  return r;
}
__device__ inline double rsq_d(double x) {
  double r = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) r = r * (1.5 - 0.5 * x * r * r);
  return r;
}

// The 2b x 2b pair problem S = [B_II B_IJ; B_JI B_JJ] is diagonalised by a
// one-sided (Hestenes) Jacobi on W = S + sigma I, sigma = 2 max|Gershgorin
// bound| so that W is positive definite: column pairs of W are rotated until
// all columns are orthogonal.  Then W = W0 R = R diag(lambda + sigma) for
// the accumulated rotation R, so the eigenvectors are the normalised final
// columns of W and R is never accumulated.  PL = 16 lanes own a column pair
// (4 rows each, two waves per SIMD) and reduce its inner product with DPP, so
// a round needs one barrier; the squared column norms are summed exactly in the first round of
// each sweep and carried through the rotations in the others.  Padding
// indices (beyond the submatrix order) never rotate.
struct SolveLds {
  double W[B2][LS];  // column-major: W[col][row]
  double nrm[B2];
  double cn[B2];     // running squared column norms of W
  int any_rot;
  int sweep_rot;
};
// Pair problem k of submatrix p in the given round (PS_NT threads).
__device__ void solve_pair(const EighBatch& e, int round, int p, int k, SolveLds& L) {
  const int npairs = e.nb / 2;
  int* flagR = flag_buf(e, round) + (int64_t)p * npairs + k;
  if (e.state[2 * p]) { if (threadIdx.x == 0) *flagR = 0; return; }
  double (*W)[LS] = L.W;
  double* nrm = L.nrm;
  double* cn = L.cn;
  int& any_rot = L.any_rot;
  int& sweep_rot = L.sweep_rot;
  const int Mp = e.Mp;
  const int msize = e.wsize[p];
  int I, J;
  pair_blocks(k, round, e.nb, I, J);
  const double* B = e.Bw + (int64_t)p * Mp * Mp;
  const int tid = threadIdx.x;
  const double fl = noise_floor(e, p);
  // pass 1: copy S (as columns) and decide whether any rotation is needed
  if (tid == 0) any_rot = 0;
  __syncthreads();
  int need = 0;
  {  // every load in flight before the first store (a loop would wait for each in turn)
    constexpr int PER = B2 * B2 / PS_NT;
    double v[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + PS_NT * m, r = idx % B2, c = idx / B2;
      v[m] = B[pair_idx(r, I, J) + (int64_t)pair_idx(c, I, J) * Mp];
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + PS_NT * m, r = idx % B2, c = idx / B2;
      W[c][r] = v[m];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < B2 * B2; idx += PS_NT) {
    int r = idx % B2, c = idx / B2;
    if (r < c && must_rotate(W[c][r], W[r][r], W[c][c], fl)) need = 1;
  }
  if (need) any_rot = 1;
  __syncthreads();
  if (!any_rot) { if (tid == 0) *flagR = 0; return; }
  const double* sc = scal_of(e, p);
  const double sigma = 2.0 * fmax(fabs(sc[1]), fabs(sc[2])) + TINY;
  for (int t = tid; t < B2; t += PS_NT) {
    const bool pad = pair_idx(t, I, J) >= msize;
    if (pad) {  // a padding column becomes a unit vector (no overflow, never rotated)
      for (int r = 0; r < B2; ++r) W[t][r] = (r == t) ? 1.0 : 0.0;
    } else {
      W[t][t] += sigma;
    }
  }
  __syncthreads();
  const int slot = tid / PL, sub = tid % PL;  // 32 column pairs x PL lanes
  const double angle = e.angle > 0.0 ? e.angle : ANGLE;
  bool converged = false;
  for (int sweep = 0; sweep < e.inner_max_sweeps; ++sweep) {
    if (tid == 0) sweep_rot = 0;
    __syncthreads();
    for (int r = 0; r < B2 - 1; ++r) {
      const int a = rr_index(slot, r, B2), b = rr_index(B2 - 1 - slot, r, B2);
      const int pc = min(a, b), qc = max(a, b);
      double x[B2 / PL], y[B2 / PL];
      double ab = 0.0, aa, bb;
      if (r == 0) {
        // exact squared column norms at the start of each sweep (every
        // column is in exactly one pair of a round); later rounds use the
        // running values in cn, updated with each rotation
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int m = 0; m < B2 / PL; ++m) {
          const int row = sub + PL * m;
          x[m] = W[pc][row];
          y[m] = W[qc][row];
          sa += x[m] * x[m];
          sb += y[m] * y[m];
          ab += x[m] * y[m];
        }
        aa = sum_pl(sa);
        bb = sum_pl(sb);
      } else {
#pragma unroll
        for (int m = 0; m < B2 / PL; ++m) {
          const int row = sub + PL * m;
          x[m] = W[pc][row];
          y[m] = W[qc][row];
          ab += x[m] * y[m];
        }
        aa = cn[pc];
        bb = cn[qc];
      }
      ab = sum_pl(ab);
      const bool padpair = pair_idx(pc, I, J) >= msize || pair_idx(qc, I, J) >= msize;
      double na = aa, nb = bb;
      // columns count as orthogonal below 8 u relative (|ab| <= 8u sqrt(aa bb),
      // compared squared): the rounding noise of the dot products stays under
      // it, so converged pairs stop rotating
      if (!padpair && fabs(ab) > TINY && ab * ab > (64.0 * TOL * TOL) * (aa * bb)) {
        // tan 2t = 2 ab / (bb - aa), |t| <= pi/4, from r = sqrt(d^2 + 4 ab^2):
        // cos 2t = |d| / r, cos^2 t = (1 + cos 2t) / 2, sin t = sin 2t / (2 cos t)
        const double d = bb - aa;
        const double ir = rsq_d(fma(d, d, 4.0 * ab * ab));
        const double h = fma(0.5 * fabs(d), ir, 0.5);
        const double ic = rsq_d(h);
        const double c = h * ic;
        const double sn = (d >= 0.0 ? ab : -ab) * ir * ic;
#pragma unroll
        for (int m = 0; m < B2 / PL; ++m) {
          const int row = sub + PL * m;
          W[pc][row] = c * x[m] - sn * y[m];
          W[qc][row] = sn * x[m] + c * y[m];
        }
        const double cs2 = 2.0 * c * sn * ab;
        na = c * c * aa - cs2 + sn * sn * bb;
        nb = sn * sn * aa + cs2 + c * c * bb;
        // only rotations by more than the stopping angle keep the sweep going (see above)
        if (sub == 0 && fabs(sn) > angle) sweep_rot = 1;
      }
      if (sub == 0) {
        cn[pc] = na;
        cn[qc] = nb;
      }
      __syncthreads();
    }
    // every thread reads the flag before thread 0 may clear it for the next sweep
    const bool again = sweep_rot != 0;
    __syncthreads();
    if (!again) {
      converged = true;
      break;
    }
  }
  // The normalised columns are orthonormal eigenvectors only once every
  // column pair is orthogonal; a pair problem that did not get there is a
  // convergence failure of the eigensolver.
  int* inf = info_of(e, p);
  if (!converged && tid == 0 && inf) atomicCAS(inf, 0, PFSM_INFO_EIGH_NOCONV);
  // eigenvectors: normalised columns of W
  if (tid < B2) {
    double s2 = 0.0;
    for (int r = 0; r < B2; ++r) s2 += W[tid][r] * W[tid][r];
    nrm[tid] = rsq_d(s2);
  }
  __syncthreads();
  double* Rg = rot_buf(e, round) + ((int64_t)p * npairs + k) * B2 * B2;
  for (int idx = tid; idx < B2 * B2; idx += PS_NT) {  // row-major: Rg[r * 2b + c] = R(r, c)
    int r = idx / B2, c = idx % B2;
    Rg[idx] = W[c][r] * nrm[c];
  }
  if (tid == 0) {
    *flagR = 1;
    atomicOr(&e.state[2 * p + 1], 1);
    atomicAdd(&e.stats[2 * p + 1], 1);
  }
}

__global__ __launch_bounds__(PS_NT) void pair_solve(EighBatch e, int round) {
  __shared__ SolveLds L;
  const int npairs = e.nb / 2;
  solve_pair(e, round, blockIdx.x / npairs, blockIdx.x % npairs, L);
}

// 64x64x64 products with FP64 MFMA by NTH / 64 waves: wave w owns rows
// [32 (w & 1), +32) and JW = 128 * 64 / NTH columns from JW (w >> 1) of Z
// (32 with four waves, 16 with eight).  The rotation operand R (row-major in
// global memory, L2-resident) is read straight into registers, all 16
// k-steps' worth before the loop; only the tile operand sits in LDS, so a
// workgroup needs one LDS tile.
template <int NTH> struct Mm64 {
  static constexpr int JW = 2 * B2 * 64 / NTH;  // columns per wave
  static constexpr int JB = JW / 16;            // 16-wide MFMA column blocks per wave
  static_assert(JB >= 1, "at most eight waves");
};
// Z = R^T Y: fragment (i, k) of R^T is R(k, i), contiguous over i.
template <int NTH>
__device__ inline void mm64_rt_y(const double* __restrict__ R, const double (*Y)[LS], v4d acc[2][Mm64<NTH>::JB]) {
  constexpr int JB = Mm64<NTH>::JB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int i0 = (wave & 1) * 32, j0 = (wave >> 1) * Mm64<NTH>::JW;
  double af[B2 / 4][2];
#pragma unroll
  for (int kk = 0; kk < B2 / 4; ++kk)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) af[kk][ib] = R[(4 * kk + lq) * B2 + i0 + ib * 16 + l16];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < B2 / 4; ++kk) {
    double bf[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) bf[jb] = Y[4 * kk + lq][j0 + jb * 16 + l16];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[jb], af[kk][ib], acc[ib][jb], 0, 0, 0);
  }
}
// Z = X R: fragment (k, j) of R is contiguous over j.
template <int NTH>
__device__ inline void mm64_x_r(const double (*X)[LS], const double* __restrict__ R, v4d acc[2][Mm64<NTH>::JB]) {
  constexpr int JB = Mm64<NTH>::JB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int i0 = (wave & 1) * 32, j0 = (wave >> 1) * Mm64<NTH>::JW;
  double bf[B2 / 4][JB];
#pragma unroll
  for (int kk = 0; kk < B2 / 4; ++kk)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) bf[kk][jb] = R[(4 * kk + lq) * B2 + j0 + jb * 16 + l16];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < B2 / 4; ++kk) {
    double af[2];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) af[ib] = X[i0 + ib * 16 + l16][4 * kk + lq];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[kk][jb], af[ib], acc[ib][jb], 0, 0, 0);
  }
}

template <int NTH> __device__ inline void store_acc(double (*Z)[LS], v4d acc[2][Mm64<NTH>::JB]) {
  constexpr int JB = Mm64<NTH>::JB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int i0 = (wave & 1) * 32, j0 = (wave >> 1) * Mm64<NTH>::JW;
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) Z[i0 + ib * 16 + l16][j0 + jb * 16 + lq + 4 * r] = acc[ib][jb][r];
}

// ------------------------------------------------------------------ apply
// B <- J^T B J: per submatrix npairs(npairs+1)/2 tiles (pairs k1 <= k2),
// each also written transposed into (k2, k1) so B stays exactly symmetric.
// U <- U J: per submatrix (Mp/2b) * npairs tiles (row tile, pair).  One
// 64 x 64 LDS tile per workgroup; a product with an unrotated pair (identity
// R) is skipped.  The B tiles of round r are what the pair problems of round
// r + 1 read; the U tiles are read by nothing until the next round's U
// update, so they run in the same launch as the next round's pair problems.
template <int NTH> __device__ void apply_b_tile(const EighBatch& e, int round, int p, int w, double (*T)[LS]) {
  if (e.state[2 * p]) return;
  const int npairs = e.nb / 2;
  const int Mp = e.Mp;
  const int* fl = flag_buf(e, round) + (int64_t)p * npairs;
  const double* Rbase = rot_buf(e, round) + (int64_t)p * npairs * B2 * B2;
  const int tid = threadIdx.x;
  v4d acc[2][Mm64<NTH>::JB];
  int k2 = 0;
  while ((k2 + 1) * (k2 + 2) / 2 <= w) ++k2;
  const int k1 = w - k2 * (k2 + 1) / 2;
  const int f1 = fl[k1], f2 = fl[k2];
  if (!f1 && !f2) return;
  int I1, J1, I2, J2;
  pair_blocks(k1, round, e.nb, I1, J1);
  pair_blocks(k2, round, e.nb, I2, J2);
  double* B = e.Bw + (int64_t)p * Mp * Mp;
  const double* R1 = Rbase + (int64_t)k1 * B2 * B2;
  const double* R2 = Rbase + (int64_t)k2 * B2 * B2;
  {  // every load in flight before the first store
    constexpr int PER = B2 * B2 / NTH;
    double v[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + NTH * m, r = idx % B2, c = idx / B2;
      v[m] = B[pair_idx(r, I1, J1) + (int64_t)pair_idx(c, I2, J2) * Mp];
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + NTH * m, r = idx % B2, c = idx / B2;
      T[r][c] = v[m];
    }
  }
  __syncthreads();
  if (f1) {
    mm64_rt_y<NTH>(R1, T, acc);  // R1^T T
    __syncthreads();
    store_acc<NTH>(T, acc);
    __syncthreads();
  }
  if (f2) {
    mm64_x_r<NTH>(T, R2, acc);  // (R1^T T) R2
    __syncthreads();
    store_acc<NTH>(T, acc);
    __syncthreads();
  }
  for (int idx = tid; idx < B2 * B2; idx += NTH) {
    const int r = idx % B2, c = idx / B2;
    B[pair_idx(r, I1, J1) + (int64_t)pair_idx(c, I2, J2) * Mp] = T[r][c];
  }
  if (k1 != k2) {  // mirror tile, written with consecutive threads along its columns
    for (int idx = tid; idx < B2 * B2; idx += NTH) {
      const int c = idx % B2, r = idx / B2;
      B[pair_idx(c, I2, J2) + (int64_t)pair_idx(r, I1, J1) * Mp] = T[r][c];
    }
  }
}

template <int NTH> __device__ void apply_u_tile(const EighBatch& e, int round, int p, int ww, double (*T)[LS]) {
  if (e.state[2 * p]) return;
  const int npairs = e.nb / 2;
  const int nrc = e.Mp / B2;
  const int Mp = e.Mp;
  const int rc = ww % nrc, k2 = ww / nrc;
  if (!flag_buf(e, round)[(int64_t)p * npairs + k2]) return;
  int I2, J2;
  pair_blocks(k2, round, e.nb, I2, J2);
  double* U = e.Uw + (int64_t)p * Mp * Mp;
  const double* R2 = rot_buf(e, round) + ((int64_t)p * npairs + k2) * B2 * B2;
  const int tid = threadIdx.x;
  v4d acc[2][Mm64<NTH>::JB];
  {  // every load in flight before the first store
    constexpr int PER = B2 * B2 / NTH;
    double v[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + NTH * m, r = idx % B2, c = idx / B2;
      v[m] = U[(rc * B2 + r) + (int64_t)pair_idx(c, I2, J2) * Mp];
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + NTH * m, r = idx % B2, c = idx / B2;
      T[r][c] = v[m];
    }
  }
  __syncthreads();
  mm64_x_r<NTH>(T, R2, acc);
  __syncthreads();
  store_acc<NTH>(T, acc);
  __syncthreads();
  for (int idx = tid; idx < B2 * B2; idx += NTH) {
    int r = idx % B2, c = idx / B2;
    U[(rc * B2 + r) + (int64_t)pair_idx(c, I2, J2) * Mp] = T[r][c];
  }
}

// B tiles of a round: one eight-wave workgroup per tile (four fit a CU).
__global__ __launch_bounds__(PS_NT) void pair_apply_b(EighBatch e, int round) {
  __shared__ double T[B2][LS];
  const int npairs = e.nb / 2, ntri = npairs * (npairs + 1) / 2;
  apply_b_tile<PS_NT>(e, round, blockIdx.x / ntri, blockIdx.x % ntri, T);
}

// The pair problems of round solve_round (the first P * npairs workgroups;
// none when solve_round < 0) beside the U tiles of round u_round (the rest).
__global__ __launch_bounds__(PS_NT) void pair_solve_apply_u(EighBatch e, int solve_round, int u_round) {
  __shared__ SolveLds L;
  const int npairs = e.nb / 2;
  const int ns = solve_round >= 0 ? e.P * npairs : 0;
  const int b = blockIdx.x;
  if (b < ns) {
    solve_pair(e, solve_round, b / npairs, b % npairs, L);
  } else {
    const int per = (e.Mp / B2) * npairs;
    apply_u_tile<PS_NT>(e, u_round, (b - ns) / per, (b - ns) % per, L.W);
  }
}

// ------------------------------------------------------------------ select + embed
// Ascending rank of each diagonal entry (stable), then the slice's ranks
// [offset, offset + size) become start vectors X0 (zero outside the
// submatrix rows) and shifts eps.  Ranking: one workgroup per 64 entries of a submatrix.
constexpr int RS_NT = 64;  // entries ranked per workgroup (one per thread)
__global__ __launch_bounds__(RS_NT) void rank_select(EighBatch e) {
  const int p = blockIdx.x;
  const int Mp = e.Mp;
  const double* B = e.Bw + (int64_t)p * Mp * Mp;
  int* sel = e.sel + (int64_t)p * Mp;
  extern __shared__ double dsh[];
#pragma unroll 8
  for (int i = threadIdx.x; i < Mp; i += RS_NT) dsh[i] = B[i + (int64_t)i * Mp];
  __syncthreads();
  const int i = blockIdx.y * RS_NT + threadIdx.x;  // Mp is a multiple of RS_NT
  const double di = dsh[i];
  int rank = 0;
  for (int j = 0; j < Mp; ++j) rank += order_before(dsh[j], j, di, i);
  sel[rank] = i;  // rank -> local index; ranks are a permutation even with NaN
  // not converged: the last sweep still rotated and no sweep was rotation-free
  int* inf = info_of(e, p);
  if (blockIdx.y == 0 && threadIdx.x == 0 && e.state[2 * p] == 0 && e.state[2 * p + 1] != 0 && inf)
    atomicCAS(inf, 0, PFSM_INFO_EIGH_NOCONV);
}

template <typename T>
__global__ void embed_x0(EighBatch e, T* __restrict__ X, int64_t ldx, double* __restrict__ eps, int64_t n) {
  // one workgroup per column c of X0
  const int64_t c = blockIdx.x;
  // find partition of column c (part offsets are ascending, P small)
  int p = 0;
  while (p + 1 < e.P && e.part_start[p + 1] <= c) ++p;
  const int64_t s = e.part_start[p];
  const int64_t w0 = e.wstart[p];
  const int M = e.wsize[p];
  const int Mp = e.Mp;
  int li = e.sel[(int64_t)p * Mp + e.offset[p] + (int)(c - s)];
  li = min(max(li, 0), Mp - 1);
  const double* U = e.Uw + (int64_t)p * Mp * Mp + (int64_t)li * Mp;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    double v = 0.0;
    if (r >= w0 && r < w0 + M) v = U[r - w0];
    X[r + c * ldx] = (T)v;
  }
  if (threadIdx.x == 0) {
    const double* B = e.Bw + (int64_t)p * Mp * Mp;
    eps[c] = B[li + (int64_t)li * Mp];
  }
}

}  // namespace

template <typename T>
static hipError_t eigh_run(const EighBatch& e, const T* At, int64_t ldat, int max_sweeps, hipStream_t s) {
  const int npairs = e.nb / 2;
  const int nrc = e.Mp / B2;
  {
    dim3 grid((unsigned)std::min<int64_t>(((int64_t)e.Mp * e.Mp + 255) / 256, 1024), e.P);
    hipLaunchKernelGGL(gather_windows<T>, grid, dim3(256), 0, s, e, At, ldat);
  }
  for (int sw = 0; sw < max_sweeps; ++sw) {
    hipLaunchKernelGGL(sweep_begin, dim3((e.P + 63) / 64), dim3(64), 0, s, e, sw);
    // round r: B tiles, then the next round's pair problems beside the U tiles
    const int rounds = e.nb - 1;
    hipLaunchKernelGGL(pair_solve, dim3(e.P * npairs), dim3(PS_NT), 0, s, e, 0);
    for (int r = 0; r < rounds; ++r) {
      hipLaunchKernelGGL(pair_apply_b, dim3(e.P * (npairs * (npairs + 1) / 2)), dim3(PS_NT), 0, s, e, r);
      const int next = r + 1 < rounds ? r + 1 : -1;
      const unsigned grid = (unsigned)((next >= 0 ? e.P * npairs : 0) + e.P * nrc * npairs);
      hipLaunchKernelGGL(pair_solve_apply_u, dim3(grid), dim3(PS_NT), 0, s, e, next, r);
    }
  }
  hipLaunchKernelGGL(rank_select, dim3(e.P, e.Mp / RS_NT), dim3(RS_NT), e.Mp * sizeof(double), s, e);
  return hipGetLastError();
}

hipError_t eigh_batched_run(const EighBatch& e, const double* At, int64_t ldat, int max_sweeps, hipStream_t s) {
  if (e.src_f32) return eigh_run(e, (const float*)At, ldat, max_sweeps, s);
  return eigh_run(e, At, ldat, max_sweeps, s);
}
hipError_t eigh_batched_run(const EighBatch& e, const float* At, int64_t ldat, int max_sweeps, hipStream_t s) {
  return eigh_run(e, At, ldat, max_sweeps, s);
}

hipError_t embed_start_vectors(const EighBatch& e, float* X, int64_t ldx, double* eps, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(embed_x0<float>, dim3((unsigned)n), dim3(256), 0, s, e, X, ldx, eps, n);
  return hipGetLastError();
}

hipError_t embed_start_vectors(const EighBatch& e, double* X, int64_t ldx, double* eps, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(embed_x0<double>, dim3((unsigned)n), dim3(256), 0, s, e, X, ldx, eps, n);
  return hipGetLastError();
}

}  // namespace pfsm
