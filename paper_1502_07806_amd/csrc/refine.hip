// FP64 refinement of the mixed-precision eigenpair estimates against the
// original matrix, plus small conversion helpers of the mixed path.
//
// With Z = A V (FP64 GEMM), each estimate gets its Rayleigh quotient
// lambda_j = v_j^T z_j / v_j^T v_j.  Estimates are ordered; runs of neighbours
// whose gaps are below tau * max|lambda| form clusters, and each cluster is
// replaced by the Ritz pairs of the pencil (V_c^T Z_c, V_c^T V_c) (Cholesky of
// the small Gram matrix + cyclic Jacobi), which removes the mixing that the
// reduced-precision products cause between close eigenvalues.  Isolated
// estimates are only normalised.
#include "common.h"
#include "refine.h"
#include "order_key.h"
#include "misc.h"

namespace pfsm {
namespace {

constexpr int NT = 256;
constexpr int KM = REFINE_KMAX;
constexpr int KS = 4;  // clusters up to this size take the one-pass Gram and output paths
constexpr int GU = 1;  // rows per thread per step of the one-pass Gram
constexpr int RU = 4;  // rows per thread in flight in the output copies

__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

__global__ __launch_bounds__(NT) void k_dots(const double* V, int64_t ldv, const double* Z, int64_t ldz, int64_t n,
                                             double* d, double* nn, double* zz) {
  __shared__ double sh[NT / 64];
  const int64_t j = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll 8  // eight loads of each operand in flight per thread; the sums keep their order
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    const double v = V[i + j * ldv], z = Z[i + j * ldz];
    a += v * z;
    b += v * v;
    c += z * z;
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (zz) c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    d[j] = a;
    nn[j] = b;
    if (zz) zz[j] = c;
  }
}

// Sorted estimates: inv[rank] = column, lam_s[rank] = d_j / nn_j (ranks from rank_ascending).
__global__ __launch_bounds__(NT) void k_rank_finish(const double* d, const double* nn, int64_t n, const int* rank,
                                                    int* inv, double* lam_s, int* info) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  const double lj = d[j] / nn[j];
  if (!isfinite(lj)) atomicCAS(info, 0, -1);
  const int r = rank[j];  // a permutation of 0..n-1 (total order)
  inv[r] = (int)j;
  lam_s[r] = lj;
}

// Single workgroup: cluster boundaries over the sorted estimates.
__global__ __launch_bounds__(1024) void k_clusters(const double* lam_s, int64_t n, double tau, int* count, int* cstart,
                                                   int* csize) {
  __shared__ double smax[1024];
  __shared__ int scan[1024];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    double a = fabs(lam_s[i]);
    m = (a > m || a != a) ? a : m;
  }
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    __syncthreads();
  }
  const double thr = tau * smax[0];
  // sequential scan in chunks: thread t owns a contiguous range
  const int64_t per = (n + 1023) / 1024;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min<int64_t>(n, b0 + per);
  // count cluster starts in my range (a start: i == 0 or gap > thr); clusters longer than KM are cut
  int cnt = 0;
  for (int64_t i = b0; i < b1; ++i) {
    bool start = (i == 0) || !(lam_s[i] - lam_s[i - 1] <= thr);
    cnt += start;
  }
  // inclusive prefix sum of the counts over the 1024 threads (log-step scan)
  scan[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  if (threadIdx.x == 1023) *count = scan[1023];  // number of natural clusters (before cutting at KM)
  int idx = scan[threadIdx.x] - cnt;  // first cluster index of my range
  for (int64_t i = b0; i < b1; ++i) {
    bool start = (i == 0) || !(lam_s[i] - lam_s[i - 1] <= thr);
    if (start) {
      int64_t e = i + 1;
      while (e < n && lam_s[e] - lam_s[e - 1] <= thr) ++e;
      cstart[idx] = (int)i;
      csize[idx] = (int)(e - i);
      ++idx;
    }
  }
}

// One workgroup per (natural) cluster; clusters longer than KM are processed
// as consecutive pieces of at most KM estimates.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_cluster_rr(const double* V, int64_t ldv, const double* Z, int64_t ldz, int64_t n,
                                                   const int* count, const int* cstart, const int* csize, const int* inv,
                                                   const double* lam_s, const double* nn, double* lam, double* Vout,
                                                   int64_t ldvo, const double* zz, double* resid) {
  const int c = blockIdx.x;
  if (c >= *count) return;
  __shared__ double G[KM][KM + 1], Mm[KM][KM + 1], Y[KM][KM + 1];
  __shared__ int col[KM];
  __shared__ double cs_c[KM / 2], cs_s[KM / 2];
  __shared__ int pp[KM / 2], qq[KM / 2];
  __shared__ int rk[KM];
  __shared__ int rot;
  __shared__ double red[NT / 64][2 * KS * KS];
  const int tid = threadIdx.x;
  const int s_all = cstart[c], k_all = csize[c];
  for (int piece = 0; piece < k_all; piece += KM) {
    const int s = s_all + piece;
    const int k = min(KM, k_all - piece);
    if (k == 1) {
      if (tid == 0) lam[s] = lam_s[s];
      const int j = inv[s];
      // residual of the normalised vector: ||z||^2 / v^T v - lambda^2
      if (resid && tid == 0) resid[s] = sqrt(fmax(zz[j] / nn[j] - lam_s[s] * lam_s[s], 0.0));
      const double inv_norm = 1.0 / sqrt(nn[j]);
      const double* vj = V + (int64_t)j * ldv;
      double* out = Vout + (int64_t)s * ldvo;
      for (int64_t i0 = tid; i0 < n; i0 += NT * RU) {  // RU rows per thread in flight
        double x[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) x[u] = vj[min<int64_t>(i0 + NT * u, n - 1)];
#pragma unroll
        for (int u = 0; u < RU; ++u)
          if (i0 + NT * u < n) out[i0 + NT * u] = x[u] * inv_norm;
      }
      __syncthreads();
      continue;
    }
    if (tid < KM) col[tid] = inv[s + min(tid, k - 1)];  // entries past k repeat a valid column
    __syncthreads();
    // G = (V_c^T Z_c + Z_c^T V_c) / 2 and Mm = V_c^T V_c, by blocks of KS x KS
    // entries: for each block pair the whole workgroup makes one pass over
    // the rows with every product of the pair accumulated at once (columns
    // past k repeat column k - 1; their sums are not stored).  V_c^T Z_c is
    // gathered in Y, which is free until the Jacobi iteration.
    const int lane = tid & 63, wave = tid >> 6;
    const int nblk = (k + KS - 1) / KS;
    for (int bp = 0; bp < nblk * nblk; ++bp) {
      const int ca = bp % nblk, cb = bp / nblk;
      int64_t oa[KS], ob[KS], oz[KS];
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        oa[t] = (int64_t)__builtin_amdgcn_readfirstlane(col[ca * KS + t]) * ldv;
        const int cbt = __builtin_amdgcn_readfirstlane(col[cb * KS + t]);
        ob[t] = (int64_t)cbt * ldv;
        oz[t] = (int64_t)cbt * ldz;
      }
      double pz[KS][KS], mv[KS][KS];
#pragma unroll
      for (int x = 0; x < KS; ++x)
#pragma unroll
        for (int y = 0; y < KS; ++y) pz[x][y] = mv[x][y] = 0.0;
      for (int64_t i0 = tid; i0 < n; i0 += NT * GU) {
        double xa[GU][KS], xb[GU][KS], yb[GU][KS];
#pragma unroll
        for (int u = 0; u < GU; ++u)
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const int64_t i = min<int64_t>(i0 + NT * u, n - 1);
            xa[u][t] = V[i + oa[t]];
            xb[u][t] = (ca == cb) ? 0.0 : V[i + ob[t]];
            yb[u][t] = Z[i + oz[t]];
          }
#pragma unroll
        for (int u = 0; u < GU; ++u) {
          if (i0 + NT * u >= n) continue;
#pragma unroll
          for (int x = 0; x < KS; ++x)
#pragma unroll
            for (int y = 0; y < KS; ++y) {
              pz[x][y] += xa[u][x] * yb[u][y];
              mv[x][y] += xa[u][x] * ((ca == cb) ? xa[u][y] : xb[u][y]);
            }
        }
      }
#pragma unroll
      for (int x = 0; x < KS; ++x)
#pragma unroll
        for (int y = 0; y < KS; ++y) {
          double p = pz[x][y], m = mv[x][y];
          for (int off = 32; off > 0; off >>= 1) {
            p += __shfl_xor(p, off, 64);
            m += __shfl_xor(m, off, 64);
          }
          if (lane == 0) {
            red[wave][x * KS + y] = p;
            red[wave][KS * KS + x * KS + y] = m;
          }
        }
      __syncthreads();
      if (tid < KS * KS) {
        const int x = tid / KS, y = tid % KS;
        const int ga = ca * KS + x, gb = cb * KS + y;
        double p = 0.0, m = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
          p += red[w][x * KS + y];
          m += red[w][KS * KS + x * KS + y];
        }
        if (ga < k && gb < k) {
          Y[ga][gb] = p;  // v_ga^T z_gb
          Mm[ga][gb] = m;
        }
      }
      __syncthreads();
    }
    for (int idx = tid; idx < k * k; idx += NT) {
      const int x = idx % k, y = idx / k;
      G[x][y] = 0.5 * (Y[x][y] + Y[y][x]);
      if (x > y) Mm[x][y] = Mm[y][x];  // the same sum in both triangles
    }
    __syncthreads();
    // Cholesky Mm = R R^T (lower R, in Mm; right-looking, rows in parallel),
    // then G <- R^{-1} G R^{-T} (independent triangular solves per column /
    // row of G, one thread each).
    for (int j = 0; j < k; ++j) {
      if (tid == 0) Mm[j][j] = sqrt(fmax(Mm[j][j], 1e-300));
      __syncthreads();
      if (tid > j && tid < k) Mm[tid][j] /= Mm[j][j];
      __syncthreads();
      for (int idx = tid; idx < k * k; idx += NT) {
        const int i = idx % k, l = idx / k;
        if (l > j && i >= l) Mm[i][l] -= Mm[i][j] * Mm[l][j];
      }
      __syncthreads();
    }
    if (tid < k) {  // W = R^{-1} G, column b = tid
      const int b = tid;
      for (int i = 0; i < k; ++i) {
        double v = G[i][b];
        for (int t = 0; t < i; ++t) v -= Mm[i][t] * G[t][b];
        G[i][b] = v / Mm[i][i];
      }
    }
    __syncthreads();
    if (tid < k) {  // C = W R^{-T}, row a = tid
      const int a = tid;
      for (int i = 0; i < k; ++i) {
        double v = G[a][i];
        for (int t = 0; t < i; ++t) v -= G[a][t] * Mm[i][t];
        G[a][i] = v / Mm[i][i];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < k * k; idx += NT) {
      const int a = idx % k, b = idx / k;
      if (a < b) {
        const double v = 0.5 * (G[a][b] + G[b][a]);
        G[a][b] = v;
        G[b][a] = v;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < KM * KM; idx += NT) Y[idx % KM][idx / KM] = (idx % KM == idx / KM) ? 1.0 : 0.0;
    __syncthreads();
    // cyclic Jacobi on the k x k matrix G (k <= 32): parallel order over a padded even size
    const int k2 = (k + 1) & ~1;
    for (int sweep = 0; sweep < 30; ++sweep) {
      if (tid == 0) rot = 0;
      __syncthreads();
      for (int r = 0; r < k2 - 1; ++r) {
        if (tid < k2 / 2) {
          int a = (tid == 0) ? 0 : ((tid - 1 + r) % (k2 - 1)) + 1;
          int bpos = k2 - 1 - tid;
          int b = (bpos == 0) ? 0 : ((bpos - 1 + r) % (k2 - 1)) + 1;
          int p = min(a, b), q = max(a, b);
          double cc = 1.0, ss = 0.0;
          if (q < k) {
            double apq = G[p][q], app = G[p][p], aqq = G[q][q];
            if (fabs(apq) > 1e-300 && fabs(apq) > 1.1102230246251565e-16 * sqrt(fabs(app) * fabs(aqq))) {
              double tau = (aqq - app) / (2.0 * apq);
              double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              cc = 1.0 / sqrt(1.0 + t * t);
              ss = t * cc;
              rot = 1;
            }
          }
          cs_c[tid] = cc; cs_s[tid] = ss; pp[tid] = p; qq[tid] = q;
        }
        __syncthreads();
        // rotate rows then columns: thread handles one index column for each pair
        for (int idx = tid; idx < (k2 / 2) * KM; idx += NT) {
          int kk = idx % (k2 / 2), i = idx / (k2 / 2);
          int p = pp[kk], q = qq[kk];
          if (q >= k || i >= k) continue;
          double cc = cs_c[kk], ss = cs_s[kk];
          double gp = G[p][i], gq = G[q][i];
          G[p][i] = cc * gp - ss * gq;
          G[q][i] = ss * gp + cc * gq;
        }
        __syncthreads();
        for (int idx = tid; idx < (k2 / 2) * KM; idx += NT) {
          int kk = idx % (k2 / 2), i = idx / (k2 / 2);
          int p = pp[kk], q = qq[kk];
          if (q >= k || i >= k) continue;
          double cc = cs_c[kk], ss = cs_s[kk];
          double gp = G[i][p], gq = G[i][q];
          G[i][p] = cc * gp - ss * gq;
          G[i][q] = ss * gp + cc * gq;
          double yp = Y[i][p], yq = Y[i][q];
          Y[i][p] = cc * yp - ss * yq;
          Y[i][q] = ss * yp + cc * yq;
        }
        __syncthreads();
        if (tid < k2 / 2) {
          int p = pp[tid], q = qq[tid];
          if (q < k && cs_s[tid] != 0.0) { G[p][q] = 0.0; G[q][p] = 0.0; }
        }
        __syncthreads();
      }
      // every thread reads the flag before thread 0 may clear it for the next sweep
      const bool again = rot != 0;
      __syncthreads();
      if (!again) break;
    }
    // Y <- R^{-T} Y (back substitution, column b = tid)
    if (tid < k) {
      const int b = tid;
      for (int i = k - 1; i >= 0; --i) {
        double v = Y[i][b];
        for (int t = i + 1; t < k; ++t) v -= Mm[t][i] * Y[t][b];
        Y[i][b] = v / Mm[i][i];
      }
      // sign of the Ritz vector: its largest-magnitude coefficient on the
      // cluster's input vectors (lowest index on ties) is positive
      double big = -1.0, sg = 1.0;
      for (int i = 0; i < k; ++i) {
        const double a = fabs(Y[i][b]);
        if (a > big) {
          big = a;
          sg = Y[i][b] < 0.0 ? -1.0 : 1.0;
        }
      }
      for (int i = 0; i < k; ++i) Y[i][b] *= sg;
    }
    __syncthreads();
    // Ritz values ascending: the rank of each diagonal entry of G (distinct
    // ranks under the total order), Y's columns placed at their ranks
    if (tid < k) {
      const double x = G[tid][tid];
      int r = 0;
      for (int b = 0; b < k; ++b) r += order_before(G[b][b], b, x, tid) ? 1 : 0;
      rk[tid] = r;
    }
    __syncthreads();
    if (tid < k) lam[s + rk[tid]] = G[tid][tid];
    for (int idx = tid; idx < k * k; idx += NT) {
      const int i = idx % k, a = idx / k;
      Mm[i][rk[a]] = Y[i][a];  // R is no longer needed
    }
    __syncthreads();
    // Vout[:, s + t] = sum_a V[:, col[a]] Mm[a][t], by blocks of KS output
    // columns: RU rows per thread, the row's entries of one block of KS
    // input columns in registers at a time.
    for (int tb = 0; tb < nblk; ++tb) {
      for (int64_t i0 = tid; i0 < n; i0 += NT * RU) {
        double acc[RU][KS];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
          for (int t = 0; t < KS; ++t) acc[u][t] = 0.0;
        for (int ab = 0; ab < nblk; ++ab) {
          double v[RU][KS];
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const int64_t oc = (int64_t)__builtin_amdgcn_readfirstlane(col[ab * KS + t]) * ldv;
#pragma unroll
            for (int u = 0; u < RU; ++u) v[u][t] = V[min<int64_t>(i0 + NT * u, n - 1) + oc];
          }
#pragma unroll
          for (int x = 0; x < KS; ++x) {
            if (ab * KS + x >= k) continue;
#pragma unroll
            for (int t = 0; t < KS; ++t) {
              const double c = Mm[ab * KS + x][tb * KS + t];
#pragma unroll
              for (int u = 0; u < RU; ++u) acc[u][t] += v[u][x] * c;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          if (i0 + NT * u >= n) continue;
#pragma unroll
          for (int t = 0; t < KS; ++t)
            if (tb * KS + t < k) Vout[i0 + NT * u + (int64_t)(s + tb * KS + t) * ldvo] = acc[u][t];
        }
      }
    }
    __syncthreads();
    if (resid) {
      // Residuals of the Ritz pairs: A u_t = Z_c y_t, so ||A u_t - mu_t u_t||^2 =
      // y_t^T (Z_c^T Z_c) y_t - mu_t^2 (u_t has unit length and Rayleigh quotient
      // mu_t).  H = Z_c^T Z_c by KS x KS blocks (one pass over the rows per block
      // pair), into G, which is free now.
      for (int bp = 0; bp < nblk * nblk; ++bp) {
        const int ca = bp % nblk, cb = bp / nblk;
        int64_t oza[KS], ozb[KS];
#pragma unroll
        for (int t = 0; t < KS; ++t) {
          oza[t] = (int64_t)__builtin_amdgcn_readfirstlane(col[ca * KS + t]) * ldz;
          ozb[t] = (int64_t)__builtin_amdgcn_readfirstlane(col[cb * KS + t]) * ldz;
        }
        double hz[KS][KS];
#pragma unroll
        for (int x = 0; x < KS; ++x)
#pragma unroll
          for (int y = 0; y < KS; ++y) hz[x][y] = 0.0;
        for (int64_t i = tid; i < n; i += NT) {
          double za[KS], zb[KS];
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            za[t] = Z[i + oza[t]];
            zb[t] = Z[i + ozb[t]];
          }
#pragma unroll
          for (int x = 0; x < KS; ++x)
#pragma unroll
            for (int y = 0; y < KS; ++y) hz[x][y] += za[x] * zb[y];
        }
#pragma unroll
        for (int x = 0; x < KS; ++x)
#pragma unroll
          for (int y = 0; y < KS; ++y) {
            double h = hz[x][y];
            for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
            if (lane == 0) red[wave][x * KS + y] = h;
          }
        __syncthreads();
        if (tid < KS * KS) {
          const int x = tid / KS, y = tid % KS;
          const int ga = ca * KS + x, gb = cb * KS + y;
          double h = 0.0;
          for (int w = 0; w < NT / 64; ++w) h += red[w][x * KS + y];
          if (ga < k && gb < k) G[ga][gb] = h;
        }
        __syncthreads();
      }
      if (tid < k) {
        double q = 0.0;
        for (int a = 0; a < k; ++a) {
          double ha = 0.0;
          for (int b = 0; b < k; ++b) ha += G[a][b] * Mm[b][tid];
          q += Mm[a][tid] * ha;
        }
        const double mu = lam[s + tid];
        resid[s + tid] = sqrt(fmax(q - mu * mu, 0.0));
      }
      __syncthreads();
    }
  }
}

// info = -2 when some residual exceeds tol * max|lambda| (one workgroup).
__global__ __launch_bounds__(1024) void k_resid_check(const double* r, const double* lam, int64_t n, double tol,
                                                      int* info) {
  __shared__ double sr[1024], sl[1024];
  double mr = 0.0, ml = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double a = r[i], b = fabs(lam[i]);
    mr = (a > mr || a != a) ? a : mr;
    ml = (b > ml || b != b) ? b : ml;
  }
  sr[threadIdx.x] = mr;
  sl[threadIdx.x] = ml;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sr[threadIdx.x + w], b = sl[threadIdx.x + w];
      sr[threadIdx.x] = (a > sr[threadIdx.x] || a != a) ? a : sr[threadIdx.x];
      sl[threadIdx.x] = (b > sl[threadIdx.x] || b != b) ? b : sl[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(sr[0] <= tol * sl[0])) atomicCAS(info, 0, PFSM_INFO_RESIDUAL);
}

// FP64 path: r_out[rank[j]] = sqrt(max(zz[j] - lam[j]^2, 0)) for unit vectors
// x_j with Rayleigh quotients lam[j] and squared norms zz[j] of At x_j.
__global__ __launch_bounds__(256) void k_resid_rq(const double* zz, const double* lam, const int* rank, int64_t n,
                                                  double* r_out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  r_out[rank[j]] = sqrt(fmax(zz[j] - lam[j] * lam[j], 0.0));
}

// Symmetric completion from the lower triangle (i >= j) of A32: A64 = the
// full symmetric matrix in FP64 and the upper triangle of A32 overwritten by
// the mirrored lower one.  One block per 64 x 64 tile pair (I >= J), staged
// through LDS so that both the direct and the mirrored accesses are
// coalesced.
constexpr int TT = 64;
__device__ inline void tile_pair(int t, int& I, int& J) {  // t -> (I, J), I >= J, row-major lower triangle
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  I = r;
  J = t - r * (r + 1) / 2;
}
__global__ __launch_bounds__(256) void k_sym_from_lower(float* A32, double* dg, int64_t n) {
  __shared__ float T[TT][TT + 1];
  int I, J;
  tile_pair(blockIdx.x, I, J);
  const int64_t i0 = (int64_t)I * TT, j0 = (int64_t)J * TT;
  const int a = threadIdx.x & 63, b0 = threadIdx.x >> 6;
  // T[r][c] = A32(i0 + r, j0 + c) where that is in the lower triangle (all
  // sixteen loads of a thread in flight before the first store)
  {
    float v[TT / 4];
#pragma unroll
    for (int m = 0; m < TT / 4; ++m) {
      const int64_t i = i0 + a, j = j0 + b0 + 4 * m;
      v[m] = (i < n && j < n && i >= j) ? A32[i + j * n] : 0.f;
    }
#pragma unroll
    for (int m = 0; m < TT / 4; ++m) T[a][b0 + 4 * m] = v[m];
  }
  __syncthreads();
  for (int c = b0; c < TT; c += 4) {
    // tile (I, J): element (i0 + a, j0 + c)
    {
      const int64_t i = i0 + a, j = j0 + c;
      if (i < n && j < n) {
        const float v = (i >= j) ? T[a][c] : T[c][a];  // the latter only on the diagonal tile
        if (I == J && i < j) A32[i + j * n] = v;
        if (i == j) dg[i] = (double)v;
      }
    }
    // mirrored tile (J, I): element (j0 + a, i0 + c) = A(i0 + c, j0 + a)
    if (I != J) {
      const int64_t i = j0 + a, j = i0 + c;
      if (i < n && j < n) {
        const float v = T[c][a];
        A32[i + j * n] = v;
      }
    }
  }
}

// max |L - I| over the lower triangle (one workgroup per column, then a max).
__global__ __launch_bounds__(NT) void k_lmi_col(const double* L, int64_t ldl, int64_t n, double* out) {
  __shared__ double sh[NT];
  const int64_t j = blockIdx.x;
  double m = 0.0;
#pragma unroll 8  // eight loads in flight per thread
  for (int64_t i = j + threadIdx.x; i < n; i += NT) {
    double v = fabs(L[i + j * ldl] - (i == j ? 1.0 : 0.0));
    m = (v > m || v != v) ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double o = sh[threadIdx.x + w];
      sh[threadIdx.x] = (o > sh[threadIdx.x] || o != o) ? o : sh[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sh[0];
}
__global__ __launch_bounds__(NT) void k_lmi_final(const double* col, int64_t n, double limit, int* gate, double* cl) {
  __shared__ double sh[NT];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    double v = col[i];
    m = (v > m || v != v) ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double o = sh[threadIdx.x + w];
      sh[threadIdx.x] = (o > sh[threadIdx.x] || o != o) ? o : sh[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *gate = (sh[0] <= limit) ? 0 : 1;  // NaN: 1
    if (cl) {
      cl[0] = (double)n * sh[0];
      cl[1] = PFSM_BAND_TOL;
    }
  }
}

__global__ __launch_bounds__(NT) void k_col_sign_f32(float* X, int64_t n, int64_t ldx, double* sgn) {
  __shared__ float sv[NT];
  __shared__ int64_t si[NT];
  const int64_t j = blockIdx.x;
  float* c = X + j * ldx;
  float best = -1.f;
  int64_t bi = 0;
#pragma unroll 8  // eight loads in flight per thread
  for (int64_t i = threadIdx.x; i < n; i += NT) {
    float a = fabsf(c[i]);
    if (a > best) { best = a; bi = i; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      float a = sv[threadIdx.x + w];
      int64_t ai = si[threadIdx.x + w];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  const float sg = (c[si[0]] < 0.f) ? -1.f : 1.f;
  __syncthreads();
  if (sg < 0.f)
    for (int64_t i = threadIdx.x; i < n; i += NT) c[i] = -c[i];
  if (threadIdx.x == 0 && sgn) sgn[j] = sg;
}

__global__ void k_permute_f64(const double* X, int64_t ldx, const int* rank, double* Y, int64_t ldy, int64_t m) {
  const int64_t j = blockIdx.y;
  double* dst = Y + (int64_t)rank[j] * ldy;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = X[i + j * ldx];
}

}  // namespace

hipError_t refine_rr(const double* V, int64_t ldv, const double* Z, int64_t ldz, int64_t n, double tau, double* lam,
                     double* Vout, int64_t ldvo, RefineBufs b, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3((unsigned)n), dim3(NT), 0, s, V, ldv, Z, ldz, n, b.d, b.nn, b.resid ? b.zz : nullptr);
  hipError_t e = norm_check(b.nn, n, info, s);
  if (e != hipSuccess) return e;
  e = rank_ascending(b.d, b.nn, n, b.rank, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_finish, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, b.d, b.nn, n, b.rank, b.inv,
                     b.lam_s, info);
  hipLaunchKernelGGL(k_clusters, dim3(1), dim3(1024), 0, s, b.lam_s, n, tau, b.clus, b.cstart, b.csize);
  hipLaunchKernelGGL(k_cluster_rr, dim3((unsigned)n), dim3(NT), 0, s, V, ldv, Z, ldz, n, b.clus, b.cstart, b.csize,
                     b.inv, b.lam_s, b.nn, lam, Vout, ldvo, b.zz, b.resid);
  return hipGetLastError();
}

hipError_t residual_check(const double* r, const double* lam, int64_t n, double tol, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_check, dim3(1), dim3(1024), 0, s, r, lam, n, tol, info);
  return hipGetLastError();
}

hipError_t residuals_from_rq(const double* zz, const double* lam, const int* rank, int64_t n, double* r_out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_resid_rq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, zz, lam, rank, n, r_out);
  return hipGetLastError();
}

hipError_t f32_mirror_lower(float* At32, double* diag, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t t = (n + TT - 1) / TT;
  hipLaunchKernelGGL(k_sym_from_lower, dim3((unsigned)(t * (t + 1) / 2)), dim3(256), 0, s, At32, diag, n);
  return hipGetLastError();
}

hipError_t lower_minus_identity_check(const double* L, int64_t ldl, int64_t n, double limit, double* scratch,
                                      int* gate, double* cl, hipStream_t s) {
  hipLaunchKernelGGL(k_lmi_col, dim3((unsigned)n), dim3(NT), 0, s, L, ldl, n, scratch);
  hipLaunchKernelGGL(k_lmi_final, dim3(1), dim3(NT), 0, s, scratch, n, limit, gate, cl);
  return hipGetLastError();
}

hipError_t col_sign_f32(float* X, int64_t n, int64_t ldx, double* sgn, hipStream_t s) {
  hipLaunchKernelGGL(k_col_sign_f32, dim3((unsigned)n), dim3(NT), 0, s, X, n, ldx, sgn);
  return hipGetLastError();
}

hipError_t permute_f64_cols(const double* X, int64_t ldx, const int* rank, double* Y, int64_t ldy, int64_t m, int64_t n,
                            hipStream_t s) {
  dim3 grid((unsigned)std::min<int64_t>((m + 255) / 256, 32), (unsigned)n);
  hipLaunchKernelGGL(k_permute_f64, grid, dim3(256), 0, s, X, ldx, rank, Y, ldy, m);
  return hipGetLastError();
}

}  // namespace pfsm
