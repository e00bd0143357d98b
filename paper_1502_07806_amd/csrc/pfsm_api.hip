// C ABI of libpfsm: plan construction (partition / submatrix tables, step
// layout, workspace carving) and the enqueue sequence of one PFSM step.
#include "../../include/pfsm.h"
#include "common.h"
#include "eigh.h"
#include "chol.h"
#include "misc.h"
#include "gemm_x3.h"
#include "refine.h"
#include "gemm_oz.h"
#include "g2s.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <new>
#include <vector>

using namespace pfsm;

// Workspace of pfsm_solve_static: one copy per device, held until the process
// ends.  Host code never passes this name to a kernel (on the host it is only
// a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PFSM_STATIC_SCRATCH_BYTES];

struct pfsm_plan {
  int64_t n = 0;
  int P = 0;
  int64_t halo = 0;
  int iterations = 0, q = 2, shift_mode = 0, precision = 0, max_sweeps = 10, flags = 0;
  double alpha = 0.0;
  bool residuals = false;  // per-column residuals computed (PFSM_FLAG_RESIDUALS or resid_tol > 0)
  double resid_tol = 0.0;  // > 0: info -2 when a residual exceeds resid_tol * max|lambda|
  std::vector<int64_t> part_start, wstart;
  std::vector<int32_t> part_size, wsize, offset;
  std::vector<int32_t> krange;  // [tiles_n][2] K range of the first folded-spectrum product (128-column tiles)
  std::vector<int32_t> krange_x3;  // same for the 256-column tiles of the split-BF16 GEMM
  std::vector<int32_t> krange_rows;  // [tiles][2] K range of the correction's band form per 256-row tile
  int band_chunks = 0, band_chunks_rows = 0;  // widest krange_x3 / krange_rows range / 32
  int Mp = 0, nb = 0;
  int device = 0;
  // device table
  void* dtab = nullptr;
  int64_t* d_wstart = nullptr;
  int32_t* d_wsize = nullptr;
  int32_t* d_offset = nullptr;
  int64_t* d_part_start = nullptr;
  int32_t* d_krange = nullptr;
  int32_t* d_krange_x3 = nullptr;
  int32_t* d_krange_rows = nullptr;
  // workspace layout (byte offsets)
  int x3_cfg = -1;  // split-BF16 GEMM tile configuration (-1: library default), set by pfsm_autotune
  // batched plans: independent sub-plans solved concurrently on internal streams
  std::vector<pfsm_plan*> sub;
  std::vector<size_t> sub_off;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> fork_ev, join_ev;
  // batched plans: the submatrices of all instances with the same padded
  // order and sweep limit are solved by one eigensolver run (one launch per
  // stage for the whole group instead of one per instance)
  struct EighGroup {
    std::vector<int> members, p0;  // instances, and each one's first submatrix in the group
    int P = 0, Mp = 0, nb = 0, max_sweeps = 0;
    double floor_rel = 0.0, angle = 0.0;
    void* dtab = nullptr;
    int64_t *d_wstart = nullptr, *d_part_start = nullptr, *d_src_off = nullptr, *d_scal_off = nullptr;
    int32_t *d_wsize = nullptr, *d_offset = nullptr, *d_src_ld = nullptr, *d_info_idx = nullptr;
    size_t o_Bw = 0, o_Uw = 0, o_Rw = 0, o_rflag = 0, o_state = 0, o_stats = 0, o_sel = 0;  // in the workspace
  };
  std::vector<EighGroup> groups;
  // stage timing
  std::vector<hipEvent_t> tev;
  int t_max = 0, t_count = 0;
  size_t o_stats = 0;
  size_t o_At, o_b0, o_b1, o_Bw, o_Uw, o_Rw, o_rflag, o_state, o_sel, o_T, o_part, o_eps, o_lamu, o_sgn, o_rank,
      o_scal, o_glo, o_ghi, o_den, o_resid = 0, o_zz = 0, o_part2 = 0, total;
  // mixed-precision workspace (byte offsets)
  size_t m_At32, m_X32, m_Y32, m_S64, m_Apk, m_Vpk, m_Atpk, m_Xpk, m_Ypk, m_Rpk, m_rb;
  size_t m_oz;  // digit planes of A and V_new for the refinement product, then 2n exponents
  size_t m_split = 0, split_bytes = 0;  // K-split scratch of the lower-triangle split-BF16 products
  size_t m_gate = 0, m_bcopy = 0;  // orthonormalisation: fallback gate word, Cholesky block copies
  size_t m_Epk = 0, m_fm = 0;       // band form of the folded-spectrum products: off-diagonal At, far maxima
  size_t m_gcl = 0;                 // gate scalars of the orthonormalisation correction's band form
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bbytes && pb < pa + abytes;
}

pfsm_status hip_status(hipError_t e) { return e == hipSuccess ? PFSM_OK : PFSM_HIP_ERROR; }

// Device address of `scratch` on the current device, looked up once per
// device (at the first plan creation or static solve there) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Records the boundary event k of the current timed solve (no-op when timing is off).
struct StageClock {
  pfsm_plan* pl;
  hipStream_t s;
  int slot;
  int last = -1;
  StageClock(pfsm_plan* p, hipStream_t st) : pl(p), s(st), slot(-1) {
    if (pl->t_max > 0 && pl->t_count < pl->t_max) slot = pl->t_count++;
  }
  // Boundaries skipped since the previous mark are recorded here too, so the
  // stages they delimit read zero.
  void mark(int k) {
    if (slot < 0) return;
    for (int j = last + 1; j <= k && j < PFSM_TIMING_BOUNDS; ++j)
      (void)hipEventRecord(pl->tev[(size_t)slot * PFSM_TIMING_BOUNDS + j], s);
    if (k > last) last = k;
  }
};

#define PFSM_TRY(expr)                          \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) return PFSM_HIP_ERROR; \
  } while (0)

// The mixed path's folded-spectrum products run on plain BF16 operands (q = 2,
// unless the split is asked for), and then also in the band form.
bool mixed_band_form(const pfsm_plan* pl) {
  return pl->precision == PFSM_PREC_MIXED_BF16 && !(pl->flags & PFSM_FLAG_FS_SPLIT) && pl->q == 2 &&
         pl->iterations > 0;
}

// Rotation floor of the submatrix eigensolver: the FP64 rounding floor, or the
// looser one of the mixed path, whose start vectors are stored in FP32.
double eigh_floor(const pfsm_plan* pl) { return pl->precision == PFSM_PREC_MIXED_BF16 ? EIGH_FLOOR_MIXED : 0.0; }
// Stopping rotation of the pair problems: looser with the looser floor.
double eigh_angle(const pfsm_plan* pl) { return pl->precision == PFSM_PREC_MIXED_BF16 ? EIGH_ANGLE_MIXED : 0.0; }

// Submatrix eigensolver arguments: every pointer into the plan's workspace layout.
EighBatch eigh_batch(const pfsm_plan* pl, char* W, int* info, const double* scal) {
  EighBatch e = {};
  e.P = pl->P; e.Mp = pl->Mp; e.nb = pl->nb; e.inner_max_sweeps = EIGH_INNER_SWEEPS;
  e.Bw = (double*)(W + pl->o_Bw); e.Uw = (double*)(W + pl->o_Uw); e.Rw = (double*)(W + pl->o_Rw);
  e.rflag = (int*)(W + pl->o_rflag); e.state = (int*)(W + pl->o_state); e.sel = (int*)(W + pl->o_sel);
  e.stats = (int*)(W + pl->o_stats);
  e.wstart = pl->d_wstart; e.wsize = pl->d_wsize; e.offset = pl->d_offset; e.part_start = pl->d_part_start;
  e.info = info;
  e.scal = scal;
  e.floor_rel = eigh_floor(pl);
  e.angle = eigh_angle(pl);
  return e;
}

}  // namespace

extern "C" {

const char* pfsm_status_string(pfsm_status s) {
  switch (s) {
    case PFSM_OK: return "PFSM_OK";
    case PFSM_INVALID_ARG: return "PFSM_INVALID_ARG: invalid argument";
    case PFSM_NOT_SUPPORTED: return "PFSM_NOT_SUPPORTED: option not supported";
    case PFSM_OOM: return "PFSM_OOM: out of memory";
    case PFSM_HIP_ERROR: return "PFSM_HIP_ERROR: HIP runtime error";
    case PFSM_WORKSPACE_TOO_SMALL: return "PFSM_WORKSPACE_TOO_SMALL: workspace smaller than pfsm_workspace_size";
  }
  return "PFSM: unknown status";
}

pfsm_status pfsm_plan_create(pfsm_plan** out, const pfsm_desc* d) {
  if (!out || !d) return PFSM_INVALID_ARG;
  *out = nullptr;
  if (d->n < 1 || d->n > (int64_t)1 << 20) return PFSM_INVALID_ARG;
  if (d->num_parts < 1 || d->num_parts > d->n || !d->part_offsets) return PFSM_INVALID_ARG;
  if (d->iterations < 0 || d->iterations > 1000) return PFSM_INVALID_ARG;
  if (d->fs_power != 1 && d->fs_power != 2) return PFSM_INVALID_ARG;
  if (d->shift_mode != PFSM_SHIFT_FIXED && d->shift_mode != PFSM_SHIFT_RAYLEIGH) return PFSM_INVALID_ARG;
  if (d->precision != PFSM_PREC_FP64 && d->precision != PFSM_PREC_MIXED_BF16) return PFSM_INVALID_ARG;
  if (d->flags & ~(PFSM_FLAG_NO_REFINE | PFSM_FLAG_FS_SPLIT | PFSM_FLAG_RESIDUALS | PFSM_FLAG_BACKWARD_SPLIT))
    return PFSM_INVALID_ARG;
  if (!(d->alpha == d->alpha)) return PFSM_INVALID_ARG;  // NaN
  if (!(d->resid_tol >= 0.0)) return PFSM_INVALID_ARG;   // negative or NaN
  const int64_t n = d->n;
  const int P = d->num_parts;
  if (d->part_offsets[0] != 0 || d->part_offsets[P] != n) return PFSM_INVALID_ARG;
  int64_t mmax = 0;
  for (int p = 0; p < P; ++p) {
    int64_t m = d->part_offsets[p + 1] - d->part_offsets[p];
    if (m < 1) return PFSM_INVALID_ARG;
    mmax = std::max(mmax, m);
  }
  if (d->precision == PFSM_PREC_MIXED_BF16 && d->shift_mode != PFSM_SHIFT_FIXED) return PFSM_NOT_SUPPORTED;
  const bool want_resid = (d->flags & PFSM_FLAG_RESIDUALS) || d->resid_tol > 0.0;
  // the mixed path's residuals come from the refinement product
  if (want_resid && d->precision == PFSM_PREC_MIXED_BF16 && (d->flags & PFSM_FLAG_NO_REFINE)) return PFSM_NOT_SUPPORTED;

  pfsm_plan* pl = new (std::nothrow) pfsm_plan();
  if (!pl) return PFSM_OOM;
  pl->n = n;
  pl->P = P;
  pl->halo = d->halo < 0 ? mmax / 2 : d->halo;
  pl->iterations = d->iterations;
  pl->q = d->fs_power;
  pl->alpha = d->alpha;
  pl->shift_mode = d->shift_mode;
  pl->precision = d->precision;
  pl->max_sweeps = d->max_sweeps > 0 ? d->max_sweeps : 10;
  pl->flags = d->flags;
  pl->residuals = want_resid;
  pl->resid_tol = d->resid_tol;
  int Mmax = 0;
  for (int p = 0; p < P; ++p) {
    int64_t s = d->part_offsets[p], m = d->part_offsets[p + 1] - s;
    int64_t M = std::min<int64_t>(n, m + 2 * pl->halo);
    int64_t w = std::min<int64_t>(std::max<int64_t>(s - pl->halo, 0), n - M);
    pl->part_start.push_back(s);
    pl->part_size.push_back((int32_t)m);
    pl->wstart.push_back(w);
    pl->wsize.push_back((int32_t)M);
    pl->offset.push_back((int32_t)(s - w));
    Mmax = std::max<int>(Mmax, (int)M);
  }
  const int B2 = 2 * EIGH_B;
  pl->Mp = (Mmax + B2 - 1) / B2 * B2;
  pl->nb = pl->Mp / EIGH_B;
  // K range of each 128-column tile in the first product At * X0: the union of
  // the submatrix row ranges of the slices the tile touches, widened to BK.
  const int64_t tiles_n = (n + GEMM_BN - 1) / GEMM_BN;
  for (int64_t t = 0; t < tiles_n; ++t) {
    int64_t c0 = t * GEMM_BN, c1 = std::min<int64_t>(n, c0 + GEMM_BN);
    int64_t lo = n, hi = 0;
    for (int p = 0; p < P; ++p) {
      int64_t s = pl->part_start[p], e = s + pl->part_size[p];
      if (e <= c0 || s >= c1) continue;
      lo = std::min(lo, pl->wstart[p]);
      hi = std::max(hi, pl->wstart[p] + pl->wsize[p]);
    }
    lo = lo / GEMM_BK * GEMM_BK;
    hi = std::min<int64_t>(n, (hi + GEMM_BK - 1) / GEMM_BK * GEMM_BK);
    pl->krange.push_back((int32_t)lo);
    pl->krange.push_back((int32_t)hi);
  }
  const int64_t tiles_x3 = (n + X3_BN - 1) / X3_BN;
  for (int64_t t = 0; t < tiles_x3; ++t) {
    int64_t c0 = t * X3_BN, c1 = std::min<int64_t>(n, c0 + X3_BN);
    int64_t lo = n, hi = 0;
    for (int p = 0; p < P; ++p) {
      int64_t s = pl->part_start[p], e = s + pl->part_size[p];
      if (e <= c0 || s >= c1) continue;
      lo = std::min(lo, pl->wstart[p]);
      hi = std::max(hi, pl->wstart[p] + pl->wsize[p]);
    }
    lo = lo / 32 * 32;
    hi = std::min<int64_t>((n + 31) / 32 * 32, (hi + 31) / 32 * 32);
    pl->krange_x3.push_back((int32_t)lo);
    pl->krange_x3.push_back((int32_t)hi);
    pl->band_chunks = std::max<int>(pl->band_chunks, (int)((std::max<int64_t>(hi - lo, 0) + 31) / 32));
  }
  // per 256-row tile: the columns whose tiles' K range (submatrix rows)
  // meets the tile's rows, i.e. the k for which X(r, k) can lie inside its
  // submatrix rows (the K range of the orthonormalisation correction's band form)
  for (int64_t t = 0; t < tiles_x3; ++t) {
    const int64_t r0 = t * X3_BM, r1 = std::min<int64_t>(n, r0 + X3_BM);
    int64_t lo = -1, hi = -1;
    for (int64_t u = 0; u < tiles_x3; ++u) {
      const int64_t a = pl->krange_x3[2 * u], b = pl->krange_x3[2 * u + 1];
      if (b <= r0 || a >= r1) continue;
      if (lo < 0) lo = u;
      hi = u;
    }
    lo = lo < 0 ? 0 : lo * X3_BN;
    hi = hi < 0 ? 0 : std::min<int64_t>((n + 31) / 32 * 32, (hi + 1) * X3_BN);
    pl->krange_rows.push_back((int32_t)lo);
    pl->krange_rows.push_back((int32_t)hi);
    pl->band_chunks_rows = std::max<int>(pl->band_chunks_rows, (int)((std::max<int64_t>(hi - lo, 0) + 31) / 32));
  }
  // device table
  size_t tb = 0;
  size_t o_ws = tb; tb = align256(tb + P * sizeof(int64_t));
  size_t o_wz = tb; tb = align256(tb + P * sizeof(int32_t));
  size_t o_of = tb; tb = align256(tb + P * sizeof(int32_t));
  size_t o_ps = tb; tb = align256(tb + P * sizeof(int64_t));
  size_t o_kr = tb; tb = align256(tb + pl->krange.size() * sizeof(int32_t));
  size_t o_k3 = tb; tb = align256(tb + pl->krange_x3.size() * sizeof(int32_t));
  size_t o_kw = tb; tb = align256(tb + pl->krange_rows.size() * sizeof(int32_t));
  void* sp = nullptr;
  if (hipGetDevice(&pl->device) != hipSuccess || x3_init() != hipSuccess || oz_init() != hipSuccess ||
      scratch_address(&sp) != hipSuccess || hipMalloc(&pl->dtab, tb) != hipSuccess) {
    delete pl;
    return PFSM_HIP_ERROR;
  }
  char* base = (char*)pl->dtab;
  pl->d_wstart = (int64_t*)(base + o_ws);
  pl->d_wsize = (int32_t*)(base + o_wz);
  pl->d_offset = (int32_t*)(base + o_of);
  pl->d_part_start = (int64_t*)(base + o_ps);
  pl->d_krange = (int32_t*)(base + o_kr);
  pl->d_krange_x3 = (int32_t*)(base + o_k3);
  pl->d_krange_rows = (int32_t*)(base + o_kw);
  bool ok = hipMemcpy(pl->d_wstart, pl->wstart.data(), P * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(pl->d_wsize, pl->wsize.data(), P * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(pl->d_offset, pl->offset.data(), P * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(pl->d_part_start, pl->part_start.data(), P * sizeof(int64_t), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(pl->d_krange, pl->krange.data(), pl->krange.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(pl->d_krange_x3, pl->krange_x3.data(), pl->krange_x3.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(pl->d_krange_rows, pl->krange_rows.data(), pl->krange_rows.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    hipFree(pl->dtab);
    delete pl;
    return PFSM_HIP_ERROR;
  }
  // workspace layout
  const size_t N2 = (size_t)n * n * sizeof(double);
  const int tiles_m = (int)((n + GEMM_BM - 1) / GEMM_BM);
  const size_t Mp2 = (size_t)pl->Mp * pl->Mp * sizeof(double);
  size_t w = 0;
  // FP64 path: At; mixed path: the FP64 diagonal of its FP32 At
  pl->o_At = w; w = align256(w + (d->precision == PFSM_PREC_MIXED_BF16 ? n * sizeof(double) : N2));
  pl->o_b0 = w; w = align256(w + N2);
  pl->o_b1 = w; w = align256(w + N2);
  pl->o_Bw = w; w = align256(w + P * Mp2);
  pl->o_Uw = w; w = align256(w + P * Mp2);
  pl->o_Rw = w; w = align256(w + 2 * (size_t)P * (pl->nb / 2) * B2 * B2 * sizeof(double));  // two round buffers
  pl->o_rflag = w; w = align256(w + 2 * (size_t)P * (pl->nb / 2) * sizeof(int));
  pl->o_state = w; w = align256(w + (size_t)P * 2 * sizeof(int));
  pl->o_stats = w; w = align256(w + (size_t)P * 2 * sizeof(int));
  pl->o_sel = w; w = align256(w + (size_t)P * pl->Mp * sizeof(int));
  pl->o_T = w; w = align256(w + (size_t)((n + CHOL_NB - 1) / CHOL_NB) * CHOL_NB * CHOL_NB * sizeof(double));
  pl->o_part = w; w = align256(w + (size_t)std::max<int64_t>(tiles_m, 3) * n * sizeof(double));
  pl->o_eps = w; w = align256(w + n * sizeof(double));
  pl->o_lamu = w; w = align256(w + n * sizeof(double));
  pl->o_sgn = w; w = align256(w + n * sizeof(double));
  pl->o_rank = w; w = align256(w + n * sizeof(int));
  pl->o_scal = w; w = align256(w + 8 * sizeof(double));
  pl->o_glo = w; w = align256(w + n * sizeof(double));
  pl->o_ghi = w; w = align256(w + n * sizeof(double));
  pl->o_den = w; w = align256(w + n * sizeof(double));
  if (pl->residuals) {
    pl->o_resid = w; w = align256(w + n * sizeof(double));
    pl->o_zz = w; w = align256(w + n * sizeof(double));
    pl->o_part2 = w; w = align256(w + (size_t)std::max<int64_t>(tiles_m, 3) * n * sizeof(double));
  }
  if (pl->precision == PFSM_PREC_MIXED_BF16) {
    const size_t N4 = (size_t)n * n * sizeof(float);
    const size_t PK = (size_t)n * x3_row_stride(n) * sizeof(bf16_t);
    pl->m_At32 = w; w = align256(w + N4);
    pl->m_X32 = w; w = align256(w + N4);
    pl->m_Y32 = w; w = align256(w + N4);
    pl->m_S64 = w; w = align256(w + N2);
    pl->m_Apk = w; w = align256(w + PK);
    pl->m_Vpk = w; w = align256(w + PK);
    pl->m_Atpk = w; w = align256(w + PK);
    pl->m_Xpk = w; w = align256(w + PK);
    pl->m_Ypk = w; w = align256(w + PK);
    pl->m_Rpk = w; w = align256(w + PK);
    pl->m_rb = w; w = align256(w + (size_t)(8 * n + 8) * sizeof(double));
    pl->split_bytes = x3_split_bytes(n);
    pl->m_split = w; w = align256(w + pl->split_bytes);
    // The digit planes of the refinement (two sets of s planes plus 2n
    // exponents) always exceed the span of the three packed copies of A, V
    // and At (3 * 4 n ceil32(n) bytes), so they get a region of their own.
    const size_t oz = align256(2 * oz_plane_bytes(n, n, REFINE_OZ_SLICES)) + 2 * n * sizeof(int);
    pl->m_oz = w; w = align256(w + oz);
    pl->m_gate = w; w = align256(w + sizeof(int));
    pl->m_bcopy = w; w = align256(w + (size_t)((n + CHOL_NB - 1) / CHOL_NB) * CHOL_NB * CHOL_NB * sizeof(double));
    pl->m_Epk = w; w = align256(w + (size_t)n * x3_plain_stride(n) * sizeof(bf16_t));
    pl->m_fm = w; w = align256(w + (size_t)(2 * pl->iterations + 4) * sizeof(unsigned));
    pl->m_gcl = w; w = align256(w + 2 * sizeof(double));
  }
  pl->total = w;
  *out = pl;
  return PFSM_OK;
}

pfsm_status pfsm_workspace_size(const pfsm_plan* pl, size_t* bytes) {
  if (!pl || !bytes) return PFSM_INVALID_ARG;
  *bytes = pl->total;
  return PFSM_OK;
}

void pfsm_plan_destroy(pfsm_plan* pl) {
  if (!pl) return;
  pfsm_timing_end(pl);
  if (!pl->sub.empty() || !pl->streams.empty()) (void)hipDeviceSynchronize();
  for (pfsm_plan* q : pl->sub) pfsm_plan_destroy(q);
  for (hipStream_t st : pl->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : pl->fork_ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : pl->join_ev) (void)hipEventDestroy(ev);
  for (auto& g : pl->groups)
    if (g.dtab) (void)hipFree(g.dtab);
  if (pl->dtab) {
    (void)hipDeviceSynchronize();
    (void)hipFree(pl->dtab);
  }
  delete pl;
}

// A solve in two halves around the submatrix eigensolver, so that a batched
// call can run the eigensolver of all its instances together: PH_BEGIN runs
// up to the step length, PH_END from the start vectors on, with the
// eigensolver's results in `ext` (a view of the instance's submatrices);
// PH_ALL runs everything with the plan's own eigensolver arrays.
enum SolvePhase { PH_ALL = 0, PH_BEGIN = 1, PH_END = 2 };
static pfsm_status solve_fp64(pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv,
                              double* dLam, double* dVout, int64_t ldvo, char* W, int* info, hipStream_t s,
                              int phase, const EighBatch* ext);
static pfsm_status solve_mixed(pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv,
                               double* dLam, double* dVout, int64_t ldvo, char* W, int* info, hipStream_t s,
                               int phase, const EighBatch* ext);

pfsm_status pfsm_solve_static(pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv,
                              double* dLam, double* dVout, int64_t ldvo, int32_t* dInfo, void* stream) {
  if (!pl || !pl->sub.empty()) return PFSM_INVALID_ARG;
  if (pl->total > (size_t)PFSM_STATIC_SCRATCH_BYTES) return PFSM_WORKSPACE_TOO_SMALL;
  void* work = nullptr;
  if (scratch_address(&work) != hipSuccess) return PFSM_HIP_ERROR;
  // pfsm_solve clears what it needs cleared (the info word) with kernels and
  // allocates nothing; the scratch keeps the previous call's contents.
  return pfsm_solve(pl, dA, lda, dV, ldv, dLam, dVout, ldvo, work, PFSM_STATIC_SCRATCH_BYTES, dInfo, stream);
}

// Argument checks of one (single-instance) solve: pointers, leading
// dimensions, workspace size and alignment, outputs not overlapping the inputs,
// each other or the workspace.
static pfsm_status check_solve_args(const pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv,
                                    const double* dLam, const double* dVout, int64_t ldvo, const void* dWork,
                                    size_t work_bytes, const int32_t* dInfo) {
  if (!pl || !dA || !dV || !dLam || !dVout || !dWork || !dInfo) return PFSM_INVALID_ARG;
  if (!pl->sub.empty()) return PFSM_INVALID_ARG;  // batched plans go through pfsm_solve_batched
  const int64_t n = pl->n;
  if (lda < n || ldv < n || ldvo < n) return PFSM_INVALID_ARG;
  if (((uintptr_t)dWork) % 256 != 0) return PFSM_INVALID_ARG;
  if (work_bytes < pl->total) return PFSM_WORKSPACE_TOO_SMALL;
  const size_t bA = (size_t)(lda * (n - 1) + n) * sizeof(double);
  const size_t bV = (size_t)(ldv * (n - 1) + n) * sizeof(double);
  const size_t bVo = (size_t)(ldvo * (n - 1) + n) * sizeof(double);
  if (overlaps(dVout, bVo, dA, bA) || overlaps(dVout, bVo, dV, bV)) return PFSM_INVALID_ARG;
  if (overlaps(dVout, bVo, dWork, pl->total) || overlaps(dLam, n * sizeof(double), dWork, pl->total) ||
      overlaps(dLam, n * sizeof(double), dVout, bVo))
    return PFSM_INVALID_ARG;
  return PFSM_OK;
}

pfsm_status pfsm_solve(pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv, double* dLam,
                       double* dVout, int64_t ldvo, void* dWork, size_t work_bytes, int32_t* dInfo, void* stream) {
  const pfsm_status chk = check_solve_args(pl, dA, lda, dV, ldv, dLam, dVout, ldvo, dWork, work_bytes, dInfo);
  if (chk != PFSM_OK) return chk;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)dWork;
  int* info = (int*)dInfo;
  if (pl->precision == PFSM_PREC_MIXED_BF16)
    return solve_mixed(pl, dA, lda, dV, ldv, dLam, dVout, ldvo, W, info, s, PH_ALL, nullptr);
  return solve_fp64(pl, dA, lda, dV, ldv, dLam, dVout, ldvo, W, info, s, PH_ALL, nullptr);
}

static pfsm_status solve_fp64(pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv,
                              double* dLam, double* dVout, int64_t ldvo, char* W, int* info, hipStream_t s,
                              int phase, const EighBatch* ext) {
  const int64_t n = pl->n;
  double* At = (double*)(W + pl->o_At);
  double* buf0 = (double*)(W + pl->o_b0);
  double* buf1 = (double*)(W + pl->o_b1);
  double* eps = (double*)(W + pl->o_eps);
  double* lamu = (double*)(W + pl->o_lamu);
  double* part = (double*)(W + pl->o_part);
  double* scal = (double*)(W + pl->o_scal);
  const int tiles_m = (int)((n + GEMM_BM - 1) / GEMM_BM);

  StageClock clk(pl, s);
  if (phase != PH_END) {
  PFSM_TRY(fill_i32(info, 1, 0, s));
  clk.mark(0);

  // (1) operator in the previous basis: W = A V, At = V^T W (lower tiles, mirrored).
  {
    GemmArgs g = {};
    g.M = n; g.N = n; g.K = n;
    g.A = dA; g.lda = lda; g.B = dV; g.ldb = ldv; g.C = buf0; g.ldc = n;
    g.alpha = 1.0;
    PFSM_TRY(gemm_f64(true, false, EPI_STORE, g, s));  // A is symmetric: A V = A^T V
    GemmArgs h = {};
    h.M = n; h.N = n; h.K = n;
    h.A = dV; h.lda = ldv; h.B = buf0; h.ldb = n; h.C = At; h.ldc = n;
    h.alpha = 1.0; h.lower_only = 1;
    PFSM_TRY(gemm_f64(true, false, EPI_STORE, h, s));
    PFSM_TRY(mirror_lower(At, n, n, s));
  }
  clk.mark(1);
  // (2) step length from the Gershgorin interval (or the caller's alpha).
  PFSM_TRY(gershgorin_alpha(At, n, n, pl->q, pl->alpha, (double*)(W + pl->o_glo), (double*)(W + pl->o_ghi), scal, info, s));
  clk.mark(2);
  }
  if (phase == PH_BEGIN) return hip_status(hipGetLastError());

  // (3) submatrix eigenproblems, (4) zero-padded start vectors and shifts.
  const EighBatch e = ext ? *ext : eigh_batch(pl, W, info, scal);
  if (phase == PH_ALL) PFSM_TRY(eigh_batched_run(e, At, n, pl->max_sweeps, s));
  double* X = buf1;
  double* Wt = buf0;
  PFSM_TRY(embed_start_vectors(e, X, n, eps, n, s));
  clk.mark(3);

  // (5) folded-spectrum iterations.
  for (int it = 0; it < pl->iterations; ++it) {
    const int32_t* kr = (it == 0 && pl->shift_mode == PFSM_SHIFT_FIXED) ? pl->d_krange : nullptr;
    if (pl->shift_mode == PFSM_SHIFT_RAYLEIGH) {
      GemmArgs r = {};
      r.M = n; r.N = n; r.K = n; r.A = At; r.lda = n; r.B = X; r.ldb = n; r.D = X; r.ldd = n; r.part = part;
      r.alpha = 1.0;
      PFSM_TRY(gemm_f64(true, false, EPI_RQ, r, s));  // At symmetric
      PFSM_TRY(col_norm2(X, n, n, n, (double*)(W + pl->o_den), s));
      PFSM_TRY(rq_reduce(part, tiles_m, n, (double*)(W + pl->o_den), eps, s));
    }
    if (pl->q == 2) {
      GemmArgs g = {};
      g.M = n; g.N = n; g.K = n; g.A = At; g.lda = n; g.B = X; g.ldb = n; g.C = Wt; g.ldc = n;
      g.eps = eps; g.krange = kr;
      PFSM_TRY(gemm_f64(true, false, EPI_SHIFT, g, s));  // Y = (At - eps) X (At symmetric)
      if (it < 8) clk.mark(4 + 2 * it);
      GemmArgs h = {};
      h.M = n; h.N = n; h.K = n; h.A = At; h.lda = n; h.B = Wt; h.ldb = n; h.C = X; h.ldc = n;
      h.D = X; h.ldd = n; h.eps = eps; h.alpha_dev = scal;
      PFSM_TRY(gemm_f64(true, false, EPI_FSUPD, h, s));  // X <- X - a (At - eps) Y  (in place: reads only Y)
      if (it < 8) clk.mark(5 + 2 * it);
    } else {
      GemmArgs g = {};
      g.M = n; g.N = n; g.K = n; g.A = At; g.lda = n; g.B = X; g.ldb = n; g.C = Wt; g.ldc = n;
      g.D = X; g.ldd = n; g.eps = eps; g.alpha_dev = scal; g.krange = kr;
      if (it < 8) clk.mark(4 + 2 * it);
      PFSM_TRY(gemm_f64(true, false, EPI_FSUPD, g, s));  // X' = X - a (At - eps) X
      if (it < 8) clk.mark(5 + 2 * it);
      std::swap(X, Wt);
    }
  }

  clk.mark(19);
  // (6) Cholesky-QR: S = X^T X (lower tiles), S = L L^T, X <- X L^{-T}.
  double* S = Wt;
  {
    GemmArgs g = {};
    g.M = n; g.N = n; g.K = n; g.A = X; g.lda = n; g.B = X; g.ldb = n; g.C = S; g.ldc = n;
    g.alpha = 1.0; g.lower_only = 1;
    PFSM_TRY(gemm_f64(true, false, EPI_STORE, g, s));
    clk.mark(20);
    PFSM_TRY(cholesky_qr(S, n, X, n, n, n, (double*)(W + pl->o_T), info, s));
  }
  clk.mark(21);
  // (7) Rayleigh quotients x_j^T At x_j (and, for the residuals, ||At x_j||^2:
  // the residual of the unit vector x_j is sqrt(||At x_j||^2 - lambda_j^2),
  // equal to ||A v_j - lambda_j v_j|| for v_j = V_prev x_j).
  {
    GemmArgs r = {};
    r.M = n; r.N = n; r.K = n; r.A = At; r.lda = n; r.B = X; r.ldb = n; r.D = X; r.ldd = n; r.part = part;
    r.alpha = 1.0;
    if (pl->residuals) r.part2 = (double*)(W + pl->o_part2);
    PFSM_TRY(gemm_f64(true, false, EPI_RQ, r, s));
    PFSM_TRY(rq_reduce(part, tiles_m, n, nullptr, lamu, s));
    if (pl->residuals) PFSM_TRY(rq_reduce(r.part2, tiles_m, n, nullptr, (double*)(W + pl->o_zz), s));
  }
  clk.mark(22);
  // (8) sign convention, ascending order, back-rotation V_out = V X_perm.
  double* Xp = S;
  PFSM_TRY(finalize_order(lamu, X, n, n, Xp, n, dLam, (int*)(W + pl->o_rank), (double*)(W + pl->o_sgn), info, s));
  if (pl->residuals) {
    double* resid = (double*)(W + pl->o_resid);
    PFSM_TRY(residuals_from_rq((double*)(W + pl->o_zz), lamu, (int*)(W + pl->o_rank), n, resid, s));
    if (pl->resid_tol > 0.0) PFSM_TRY(residual_check(resid, dLam, n, pl->resid_tol, info, s));
  }
  clk.mark(23);
  {
    GemmArgs g = {};
    g.M = n; g.N = n; g.K = n; g.A = dV; g.lda = ldv; g.B = Xp; g.ldb = n; g.C = dVout; g.ldc = ldvo;
    g.alpha = 1.0;
    PFSM_TRY(gemm_f64(false, false, EPI_STORE, g, s));
    // V_prev X keeps unit columns only if V_prev is orthonormal
    PFSM_TRY(col_norm2(dVout, n, n, ldvo, (double*)(W + pl->o_den), s));
    PFSM_TRY(norm_check((double*)(W + pl->o_den), n, info, s));
  }
  clk.mark(PFSM_TIMING_BOUNDS - 1);
  return hip_status(hipGetLastError());
}


// Mixed precision: the large products on BF16 matrix cores with FP32
// accumulation (basis change, overlap and back-rotation on hi/lo split
// operands, the folded-spectrum products on plain operands unless
// PFSM_FLAG_FS_SPLIT); FP64 submatrix eigensolver; orthonormalisation to first
// order in S - I, or the FP64 Cholesky-QR of the overlap when S is farther
// from the identity; FP64 Rayleigh quotients and cluster Rayleigh-Ritz against
// A from an FP64-accurate product on the int8 matrix cores.
static pfsm_status solve_mixed(pfsm_plan* pl, const double* dA, int64_t lda, const double* dV, int64_t ldv,
                               double* dLam, double* dVout, int64_t ldvo, char* W, int* info, hipStream_t s,
                               int phase, const EighBatch* ext) {
  const int64_t n = pl->n;
  const int64_t ldp = x3_row_stride(n);
  // Plain BF16 operands for the folded-spectrum products (q = 2, unless the
  // split is asked for): At, X and Y are packed in the plain layout (row
  // stride ldq) for those products only.  The refinement against A in FP64
  // removes what the single BF16 product leaves in the vectors (at N = 8192
  // the refined eigenvalues stay 3.3e-10 from an FP64 computation).
  const bool fs_plain = mixed_band_form(pl);
  const int64_t ldq = x3_plain_stride(n);
  double* Atd = (double*)(W + pl->o_At);    // diagonal of At (FP64)
  double* B64a = (double*)(W + pl->o_b0);   // X0 (FP64), later Z = A V_new
  double* Vn64 = (double*)(W + pl->o_b1);   // V_new before ordering
  float* At32 = (float*)(W + pl->m_At32);
  float* X32 = (float*)(W + pl->m_X32);
  float* Y32 = (float*)(W + pl->m_Y32);
  double* S64 = (double*)(W + pl->m_S64);
  bf16_t* Apk = (bf16_t*)(W + pl->m_Apk);
  bf16_t* Vpk = (bf16_t*)(W + pl->m_Vpk);
  bf16_t* Atpk = (bf16_t*)(W + pl->m_Atpk);
  bf16_t* Xpk = (bf16_t*)(W + pl->m_Xpk);
  bf16_t* Ypk = (bf16_t*)(W + pl->m_Ypk);
  bf16_t* Rpk = (bf16_t*)(W + pl->m_Rpk);
  double* eps = (double*)(W + pl->o_eps);
  double* scal = (double*)(W + pl->o_scal);
  double* part = (double*)(W + pl->o_part);
  double* rb = (double*)(W + pl->m_rb);
  float* split_ws = pl->split_bytes ? (float*)(W + pl->m_split) : nullptr;
  StageClock clk(pl, s);

  auto x3 = [&](int epi, int64_t M, int64_t N, int64_t K, const bf16_t* Ap, const bf16_t* Bp, void* C, int64_t ldc,
                int c_double) {
    X3Args g = {};
    g.M = M; g.N = N; g.K = K; g.Ap = Ap; g.ldap = ldp; g.Bp = Bp; g.ldbp = ldp; g.C = C; g.ldc = ldc;
    g.c_double = c_double; g.alpha = 1.0; g.cfg = pl->x3_cfg;
    return g;
  };

  if (phase != PH_END) {
  PFSM_TRY(fill_i32(info, 1, 0, s));
  clk.mark(0);
  // (1) basis change: W = A V, At = V^T W (lower tiles, then both triangles in FP32 and the diagonal in FP64).
  PFSM_TRY(pack_x3(dA, 1, n, n, lda, 0, Apk, ldp, s));        // rows of A (= columns, A symmetric)
  PFSM_TRY(pack_x3(dV, 1, n, n, ldv, 0, Vpk, ldp, s));        // columns of V
  {
    X3Args g = x3(X3_STORE, n, n, n, Apk, Vpk, Y32, n, 0);
    if (n % 32 == 0) {  // W only feeds At = V^T W: its epilogue writes the packed copy alone
      g.pack_split = Ypk; g.ld_pack_split = ldp;
      PFSM_TRY(gemm_x3(X3_STORE_PACK, g, s));
    } else {
      PFSM_TRY(gemm_x3(X3_STORE, g, s));
      PFSM_TRY(pack_x3(Y32, 0, n, n, n, 0, Ypk, ldp, s));     // columns of W
    }
    X3Args h = x3(X3_STORE, n, n, n, Vpk, Ypk, At32, n, 0);
    h.tiles = X3_LOWER;
    h.split_ws = split_ws; h.split_bytes = pl->split_bytes;
    PFSM_TRY(gemm_x3(X3_STORE, h, s));
    PFSM_TRY(f32_mirror_lower(At32, Atd, n, s));
    if (!fs_plain) PFSM_TRY(pack_x3(At32, 0, n, n, n, 0, Atpk, ldp, s));  // (the band form packs E instead)
  }
  clk.mark(1);
  PFSM_TRY(gershgorin_alpha(At32, n, n, pl->q, pl->alpha, (double*)(W + pl->o_glo), (double*)(W + pl->o_ghi), scal,
                            info, s));
  clk.mark(2);
  }
  if (phase == PH_BEGIN) return hip_status(hipGetLastError());
  // (2) submatrix eigensolver (FP64) and start vectors.
  const EighBatch e = ext ? *ext : eigh_batch(pl, W, info, scal);
  if (phase == PH_ALL) PFSM_TRY(eigh_batched_run(e, At32, n, pl->max_sweeps, s));
  PFSM_TRY(embed_start_vectors(e, X32, n, eps, n, s));
  unsigned* fm = (unsigned*)(W + pl->m_fm);
  const bool band = fs_plain;
  // Plain operands of the folded-spectrum products: with the band form, the
  // rows a band-form product reads, then the others only when the product's
  // gate (fm[gate], the same test) sends it to the full form.
  auto pack_fs = [&](const float* src, bf16_t* dst, int gate) -> hipError_t {
    if (!band) return pack_x3(src, 0, n, n, n, fs_plain ? PACK_PLAIN : 0, dst, fs_plain ? ldq : ldp, s);
    hipError_t err = pack_x3_band(src, 0, n, n, n, PACK_PLAIN, dst, ldq, pl->d_krange_x3, pl->band_chunks, s);
    if (err == hipSuccess)
      err = pack_x3_far_gated(src, 0, n, n, n, PACK_PLAIN, dst, ldq, pl->d_krange_x3, fm + gate, scal + 3, s);
    return err;
  };
  if (band) PFSM_TRY(fill_i32((int*)fm, 2 * pl->iterations + 4, 0, s));
  PFSM_TRY(pack_fs(X32, Xpk, 0));
  clk.mark(3);
  // (3) folded-spectrum iterations (X master copy in FP32).
  // Band form (plain operands): (At - eps) B = E B_band + (D - eps) B + E B_far
  // with D the diagonal of At, E the rest, B_band the rows of the operand
  // inside the K range of its column tile (the submatrix rows) and B_far the
  // others.  The first two terms are computed, the product on E restricted to
  // that K range, the diagonal term exactly in the epilogue; the third is
  // dropped when its bound, rho max |B_far| (rho: largest off-diagonal
  // absolute row sum of At), is at most 2^-20 of the Gershgorin bound, far
  // below the rounding of a plain BF16 product of the whole matrix (2^-9).
  // Every product is enqueued in both forms behind a device gate on that
  // bound (the other launch returns at once), and every epilogue records the
  // largest far-row output for the gate of the next product: a static launch
  // sequence.  X0 has no far rows (zero padding), so fm[0] = 0.
  if (band) PFSM_TRY(pack_x3(At32, 0, n, n, n, PACK_PLAIN | PACK_OFFDIAG, (bf16_t*)(W + pl->m_Epk), ldq, s));
  // the product in the band and full forms; f_in / f_out: far maxima of operand and output
  auto fs_gemm = [&](int epi, X3Args g, int f_in, int f_out) -> hipError_t {
    if (!band) return gemm_x3(epi, g, s);
    g.far_krange = pl->d_krange_x3; g.farmax_out = fm + f_out;
    g.gate_far = fm + f_in; g.gate_cl = scal + 3;  // {rho, 2^-20 Gershgorin bound}
    // both forms on E with the diagonal term in the epilogue: the full form
    // adds E B_far, so At itself is never packed
    g.Ap = (const bf16_t*)(W + pl->m_Epk); g.diag = Atd; g.diag_stride = 1;
    X3Args b = g;
    b.krange = pl->d_krange_x3;
    b.gate_band = 1; b.band_count = fm + 2 * pl->iterations + 3;
    hipError_t e1 = gemm_x3(epi, b, s);
    if (e1 != hipSuccess) return e1;
    g.gate_band = 0;
    return gemm_x3(epi, g, s);
  };
  for (int it = 0; it < pl->iterations; ++it) {
    const int32_t* kr = (it == 0) ? pl->d_krange_x3 : nullptr;
    if (pl->q == 2) {
      X3Args g = x3(X3_SHIFT, n, n, n, Atpk, Xpk, Y32, n, 0);
      g.B32 = X32; g.ldb32 = n; g.eps = eps; g.krange = kr;
      if (fs_plain) { g.products = 1; g.ldap = g.ldbp = ldq; }
      PFSM_TRY(fs_gemm(X3_SHIFT, g, 2 * it, 2 * it + 1));  // Y = (At - eps) X
      PFSM_TRY(pack_fs(Y32, Ypk, 2 * it + 1));
      if (it < 8) clk.mark(4 + 2 * it);
      X3Args h = x3(X3_FSUPD, n, n, n, Atpk, Ypk, X32, n, 0);
      h.B32 = Y32; h.ldb32 = n; h.D = X32; h.ldd = n; h.eps = eps; h.alpha_dev = scal;
      if (fs_plain) { h.products = 1; h.ldap = h.ldbp = ldq; }
      PFSM_TRY(fs_gemm(X3_FSUPD, h, 2 * it + 1, 2 * it + 2));  // X <- X - a (At - eps) Y
    } else {
      if (it < 8) clk.mark(4 + 2 * it);
      X3Args h = x3(X3_FSUPD, n, n, n, Atpk, Xpk, X32, n, 0);
      h.B32 = X32; h.ldb32 = n; h.D = X32; h.ldd = n; h.eps = eps; h.alpha_dev = scal; h.krange = kr;
      PFSM_TRY(fs_gemm(X3_FSUPD, h, 2 * it, 2 * it + 2));  // X <- X - a (At - eps) X (operand read from the packed copy)
    }
    if (it < 8) clk.mark(5 + 2 * it);  // the update stage holds exactly one GEMM launch
    // the next iteration's operand, or the split operand of the overlap
    const bool plain_next = fs_plain && it + 1 < pl->iterations;
    if (plain_next) PFSM_TRY(pack_fs(X32, Xpk, 2 * it + 2));
    else PFSM_TRY(pack_x3(X32, 0, n, n, n, 0, Xpk, ldp, s));
  }
  clk.mark(19);
  // (4) overlap S = X^T X (FP64 output, lower tiles) and X <- X L^{-T}.
  {
    X3Args g = x3(X3_STORE, n, n, n, Xpk, Xpk, S64, n, 1);
    g.tiles = X3_LOWER;
    g.split_ws = split_ws; g.split_bytes = pl->split_bytes;
    PFSM_TRY(gemm_x3(X3_STORE, g, s));
  }
  clk.mark(20);
  // X <- X L^{-T} with S = L L^T.  S is the identity up to the folded-spectrum
  // residual E = S - I, so L = I + Phi(E) + O(|E|^2) (Phi: strictly lower part
  // plus half the diagonal) and L^{-T} = I - Phi(E)^T + O(|E|^2).  While
  // max |E| <= 1e-3 the dropped terms lie below the rounding of the split-BF16
  // products themselves, and the FP64 refinement against A sees them only to
  // second order: that first-order step is the fast path.  The product
  // X Phi(E)^T is upper triangular in its k range (KPREFIX tiles).  Its size
  // is of order |E| (3e-6 at N = 8192), so with the plain folded-spectrum
  // products it takes plain BF16 operands too: the single product's rounding,
  // 2^-9 of that, is far below the split products' own.
  // When max |E| > 1e-3 (start vectors far from orthogonal) a device gate
  // switches on the FP64 Cholesky-QR of S: an FP64 copy of X taken before the
  // first-order step is factored with S (one launch per 64-wide block column,
  // every launch returning at once when the gate is off, so the launch
  // sequence does not depend on the data) and replaces X.
  int* gate = (int*)(W + pl->m_gate);
  double* X64 = B64a;  // free until the refinement product
  double* gcl = (double*)(W + pl->m_gcl);
  PFSM_TRY(lower_minus_identity_check(S64, n, n, ORTHO_FIRST_ORDER_MAX, rb, gate, band ? gcl : nullptr, s));
  PFSM_TRY(convert_f32_f64_gated(X32, n, X64, n, n, n, 1, gate, s));
  {
    const int pf = fs_plain ? PACK_PLAIN : 0;
    const int64_t ldc = fs_plain ? ldq : ldp;
    PFSM_TRY(pack_x3(S64, 1, n, n, n, PACK_SUB_I | PACK_LOWER | PACK_HALF_DIAG | PACK_BY_ROWS | pf, Ypk, ldc, s));
    if (band) {  // rows of X: their band part, and the rest only for the full form (the same gate)
      PFSM_TRY(pack_x3_band(X32, 0, n, n, n, PACK_BY_ROWS | pf, Rpk, ldc, pl->d_krange_rows, pl->band_chunks_rows, s));
      PFSM_TRY(pack_x3_far_gated(X32, 0, n, n, n, PACK_BY_ROWS | pf, Rpk, ldc, pl->d_krange_rows,
                                 fm + 2 * pl->iterations, gcl, s));
    } else {
      PFSM_TRY(pack_x3(X32, 0, n, n, n, PACK_BY_ROWS | pf, Rpk, ldc, s));  // rows of X
    }
    X3Args h = x3(X3_ADD, n, n, n, Rpk, Ypk, X32, n, 0);  // Ypk: columns of Phi(E)^T = rows of Phi(E)
    h.alpha = -1.0; h.D = X32; h.ldd = n; h.d_double = 0; h.tiles = X3_KPREFIX;
    if (fs_plain) { h.products = 1; h.ldap = h.ldbp = ldq; }
    if (band) {
      // Band form: X(r, k) lies inside the submatrix rows of column k only for
      // the k of a contiguous range per row tile (krange_rows); the rest are
      // far entries of X, at most m = the last update's far maximum, so the
      // dropped sum is at most n max|E| m (|Phi(E)| <= |E| entrywise), gated
      // against 2^-20 (the entries of X are at most 1).
      h.gate_far = fm + 2 * pl->iterations; h.gate_cl = gcl;
      X3Args b = h;
      b.krange_rows = pl->d_krange_rows; b.gate_band = 1; b.band_count = fm + 2 * pl->iterations + 2;
      PFSM_TRY(gemm_x3(X3_ADD, b, s));
      h.gate_band = 0;
    }
    PFSM_TRY(gemm_x3(X3_ADD, h, s));  // X <- X - X Phi(E)^T (in place: the operand comes from the packed copy)
  }
  PFSM_TRY(cholesky_qr_gated(S64, n, X64, n, n, n, (double*)(W + pl->o_T), (double*)(W + pl->m_bcopy), info, gate, s));
  PFSM_TRY(convert_f32_f64_gated(X32, n, X64, n, n, n, 0, gate, s));
  clk.mark(21);
  // (5) sign convention; V_new = V + V (X - I) (FP64 output).
  PFSM_TRY(col_sign_f32(X32, n, n, (double*)(W + pl->o_sgn), s));
  const bool refine = !(pl->flags & PFSM_FLAG_NO_REFINE);
  if (!refine) {
    // eigenvalue estimates of the reduced-precision step: x_j^T At x_j
    if (fs_plain) PFSM_TRY(pack_x3(At32, 0, n, n, n, 0, Atpk, ldp, s));  // split layout again
    PFSM_TRY(pack_x3(X32, 0, n, n, n, 0, Xpk, ldp, s));
    X3Args r = x3(X3_RQ, n, n, n, Atpk, Xpk, nullptr, n, 0);
    r.D = X32; r.ldd = n; r.part = part;
    PFSM_TRY(gemm_x3(X3_RQ, r, s));
    PFSM_TRY(rq_reduce(part, (int)((n + X3_BM - 1) / X3_BM), n, nullptr, (double*)(W + pl->o_lamu), s));
  }
  clk.mark(22);
  clk.mark(23);  // the ordering comes with the refinement, after the back-rotation
  // V_new = V + V (X - I), the sum over k split in two: the rows of X that
  // belong to the submatrices of a column tile (the K range of the first
  // folded-spectrum product) on split operands, where X - I holds the
  // rotations, which are of order one inside clusters; the other rows on
  // plain operands, where X holds only the small components the folded-spectrum
  // iterations added outside the submatrices (about 1e-4 per column at
  // N = 8192), so the plain product's rounding, 2^-9 of those, stays far
  // below the split product's on the first part.  The identity lies inside
  // the first part, so the second is X itself with those rows zeroed.
  // columns of X - I, in the rows the split product reads
  PFSM_TRY(pack_x3_band(X32, 0, n, n, n, PACK_SUB_I, Xpk, ldp, pl->d_krange_x3, pl->band_chunks, s));
  // rows of V, split for the product below and plain (Atpk, free by now) for the second one
  PFSM_TRY(pack_x3_split_and_plain(dV, 1, n, n, ldv, PACK_BY_ROWS, Rpk, ldp, Atpk, ldq, s));
  {
    X3Args g = x3(X3_ADD, n, n, n, Rpk, Xpk, Vn64, n, 1);
    g.D = dV; g.ldd = ldv; g.d_double = 1; g.krange = pl->d_krange_x3;
    PFSM_TRY(gemm_x3(X3_ADD, g, s));
  }
  PFSM_TRY(zero_krange_rows(X32, n, n, n, pl->d_krange_x3, X3_BN, s));
  PFSM_TRY(pack_x3(X32, 0, n, n, n, PACK_PLAIN, Ypk, ldq, s));                  // columns of X outside those rows
  {
    X3Args h = x3(X3_ADD, n, n, n, Atpk, Ypk, Vn64, n, 1);
    h.D = Vn64; h.ldd = n; h.d_double = 1; h.products = 1; h.ldap = h.ldbp = ldq;
    PFSM_TRY(gemm_x3(X3_ADD, h, s));
  }
  if (!refine) {
    clk.mark(24);
    clk.mark(25);
    int* rank = (int*)(W + pl->o_rank);
    PFSM_TRY(finalize_order_values((double*)(W + pl->o_lamu), n, dLam, rank, info, s));
    PFSM_TRY(permute_f64_cols(Vn64, n, rank, dVout, ldvo, n, n, s));
    PFSM_TRY(col_norm2(dVout, n, n, ldvo, (double*)(W + pl->o_den), s));
    PFSM_TRY(norm_check((double*)(W + pl->o_den), n, info, s));
    clk.mark(26);
    return hip_status(hipGetLastError());
  }
  // (6) FP64 refinement: Z = A V_new, Rayleigh quotients, cluster Rayleigh-Ritz, order.
  {
    // Z = A V_new to FP64 accuracy on the int8 matrix cores: digits of the
    // rows of A (its columns, A symmetric) and of the columns of V_new.
    int8_t* ozA = (int8_t*)(W + pl->m_oz);
    int8_t* ozV = ozA + oz_plane_bytes(n, n, REFINE_OZ_SLICES);
    int* ozE = (int*)(W + pl->m_oz + align256(2 * oz_plane_bytes(n, n, REFINE_OZ_SLICES)));
    PFSM_TRY(oz_split(dA, lda, n, n, REFINE_OZ_SLICES, ozA, ozE, info, s));
    PFSM_TRY(oz_split(Vn64, n, n, n, REFINE_OZ_SLICES, ozV, ozE + n, info, s));
    clk.mark(24);  // the product stage holds exactly one launch
    PFSM_TRY(gemm_oz(n, n, n, REFINE_OZ_SLICES, ozA, ozE, ozV, ozE + n, B64a, n, s));
    clk.mark(25);
    RefineBufs b;
    b.d = rb; b.nn = rb + n; b.lam_s = rb + 2 * n;
    b.rank = (int*)(rb + 3 * n); b.inv = (int*)(rb + 4 * n); b.cstart = (int*)(rb + 5 * n);
    b.csize = (int*)(rb + 6 * n); b.clus = (int*)(rb + 7 * n);
    if (pl->residuals) {
      b.zz = rb + 7 * n + 8;
      b.resid = (double*)(W + pl->o_resid);
    }
    PFSM_TRY(refine_rr(Vn64, n, B64a, n, n, REFINE_TAU, dLam, dVout, ldvo, b, info, s));
    if (pl->resid_tol > 0.0) PFSM_TRY(residual_check(b.resid, dLam, n, pl->resid_tol, info, s));
  }
  clk.mark(26);
  return hip_status(hipGetLastError());
}

pfsm_status pfsm_g2s_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes || n < 1) return PFSM_INVALID_ARG;
  *bytes = g2s_workspace_bytes(n);
  return PFSM_OK;
}

pfsm_status pfsm_generalized_to_standard(int64_t n, const double* dA, int64_t lda, const double* dB, int64_t ldb,
                                         int32_t iterations, double* dZ, int64_t ldz, void* dWork,
                                         size_t work_bytes, double* dResidual, int32_t* dInfo, void* stream) {
  if (n < 1 || !dA || !dB || !dZ || !dWork || !dInfo || iterations < 0) return PFSM_INVALID_ARG;
  if (lda < n || ldb < n || ldz < n) return PFSM_INVALID_ARG;
  if (((uintptr_t)dWork) % 256 != 0) return PFSM_INVALID_ARG;
  const size_t need = g2s_workspace_bytes(n);
  if (work_bytes < need) return PFSM_WORKSPACE_TOO_SMALL;
  const size_t bA = (size_t)(lda * (n - 1) + n) * sizeof(double);
  const size_t bB = (size_t)(ldb * (n - 1) + n) * sizeof(double);
  const size_t bZ = (size_t)(ldz * (n - 1) + n) * sizeof(double);
  if (overlaps(dZ, bZ, dA, bA) || overlaps(dZ, bZ, dB, bB) || overlaps(dZ, bZ, dWork, need)) return PFSM_INVALID_ARG;
  if (dResidual && (overlaps(dResidual, (size_t)iterations * sizeof(double), dZ, bZ) ||
                    overlaps(dResidual, (size_t)iterations * sizeof(double), dWork, need)))
    return PFSM_INVALID_ARG;
  return hip_status(g2s_run(n, dA, lda, dB, ldb, iterations, dZ, ldz, g2s_carve(dWork, n), dResidual, dInfo,
                            (hipStream_t)stream));
}

pfsm_status pfsm_debug_stats(pfsm_plan* pl, const void* dWork, size_t work_bytes, int32_t* out, int32_t capacity,
                             int32_t* count) {
  if (!pl || !dWork || !out || !count || work_bytes < pl->total) return PFSM_INVALID_ARG;
  const int64_t n = pl->n;
  const int32_t need = 2 * pl->P + 5;
  if (capacity < need) return PFSM_INVALID_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return PFSM_HIP_ERROR;
  if (hipMemcpy(out, (const char*)dWork + pl->o_stats, 2 * pl->P * sizeof(int32_t), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return PFSM_HIP_ERROR;
  out[2 * pl->P] = out[2 * pl->P + 1] = out[2 * pl->P + 2] = out[2 * pl->P + 3] = out[2 * pl->P + 4] = 0;
  if (pl->precision == PFSM_PREC_MIXED_BF16) {
    // refinement clusters: count, then the largest cluster size
    const double* rb = (const double*)((const char*)dWork + pl->m_rb);
    int cnt = 0;
    if (hipMemcpy(&cnt, (const int*)(rb + 7 * n), sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return PFSM_HIP_ERROR;
    std::vector<int> sizes((size_t)std::max(cnt, 0));
    if (cnt > 0 && hipMemcpy(sizes.data(), (const int*)(rb + 6 * n), cnt * sizeof(int), hipMemcpyDeviceToHost) !=
                       hipSuccess)
      return PFSM_HIP_ERROR;
    int multi = 0, mx = 0;
    for (int v : sizes) {
      multi += v > 1;
      mx = std::max(mx, v);
    }
    out[2 * pl->P] = cnt;
    out[2 * pl->P + 1] = multi;
    out[2 * pl->P + 2] = mx;
    if (mixed_band_form(pl)) {  // folded-spectrum products that ran in the band form
      unsigned bc[2] = {0, 0};  // the correction's count, then the folded-spectrum products'
      if (hipMemcpy(bc, (const char*)dWork + pl->m_fm + (2 * pl->iterations + 2) * sizeof(unsigned), sizeof(bc),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return PFSM_HIP_ERROR;
      out[2 * pl->P + 3] = (int32_t)bc[1];
      out[2 * pl->P + 4] = (int32_t)bc[0];
    }
  }
  *count = need;
  return PFSM_OK;
}


pfsm_status pfsm_plan_create_batched(pfsm_plan** out, const pfsm_desc* descs, int32_t count) {
  if (!out || !descs || count < 1 || count > 4096) return PFSM_INVALID_ARG;
  *out = nullptr;
  pfsm_plan* pl = new (std::nothrow) pfsm_plan();
  if (!pl) return PFSM_OOM;
  size_t w = 0;
  for (int32_t i = 0; i < count; ++i) {
    pfsm_plan* q = nullptr;
    pfsm_status st = pfsm_plan_create(&q, &descs[i]);
    if (st != PFSM_OK) {
      pfsm_plan_destroy(pl);
      return st;
    }
    pl->sub.push_back(q);
    pl->sub_off.push_back(w);
    w = align256(w + q->total);
  }
  pl->n = 0;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    pfsm_plan_destroy(pl);
    return PFSM_HIP_ERROR;
  }
  // eigensolver groups: instances with the same padded submatrix order, sweep
  // limit, rotation floor and stopping angle, their submatrices numbered consecutively
  for (int32_t i = 0; i < count; ++i) {
    const pfsm_plan* q = pl->sub[i];
    pfsm_plan::EighGroup* g = nullptr;
    for (auto& h : pl->groups)
      if (h.Mp == q->Mp && h.max_sweeps == q->max_sweeps && h.floor_rel == eigh_floor(q) && h.angle == eigh_angle(q))
        g = &h;
    if (!g) {
      pl->groups.emplace_back();
      g = &pl->groups.back();
      g->Mp = q->Mp;
      g->nb = q->nb;
      g->max_sweeps = q->max_sweeps;
      g->floor_rel = eigh_floor(q);
      g->angle = eigh_angle(q);
    }
    g->members.push_back(i);
    g->p0.push_back(g->P);
    g->P += q->P;
  }
  const int B2 = 2 * EIGH_B;
  for (auto& g : pl->groups) {
    std::vector<int64_t> ws, ps, so, sc;
    std::vector<int32_t> wz, of, sl, ii;
    for (size_t m = 0; m < g.members.size(); ++m) {
      const int i = g.members[m];
      const pfsm_plan* q = pl->sub[i];
      for (int p = 0; p < q->P; ++p) {
        ws.push_back(q->wstart[p]);
        ps.push_back(q->part_start[p]);
        wz.push_back(q->wsize[p]);
        of.push_back(q->offset[p]);
        // the instance's At: FP64, or FP32 on the mixed path
        so.push_back((int64_t)(pl->sub_off[i] + (q->precision == PFSM_PREC_MIXED_BF16 ? q->m_At32 : q->o_At)));
        sl.push_back((int32_t)q->n);
        sc.push_back((int64_t)(pl->sub_off[i] + q->o_scal));
        ii.push_back(i);
      }
    }
    const size_t P = (size_t)g.P;
    size_t tb = 0;
    const size_t t_ws = tb; tb = align256(tb + P * sizeof(int64_t));
    const size_t t_ps = tb; tb = align256(tb + P * sizeof(int64_t));
    const size_t t_so = tb; tb = align256(tb + P * sizeof(int64_t));
    const size_t t_sc = tb; tb = align256(tb + P * sizeof(int64_t));
    const size_t t_wz = tb; tb = align256(tb + P * sizeof(int32_t));
    const size_t t_of = tb; tb = align256(tb + P * sizeof(int32_t));
    const size_t t_sl = tb; tb = align256(tb + P * sizeof(int32_t));
    const size_t t_ii = tb; tb = align256(tb + P * sizeof(int32_t));
    if (hipMalloc(&g.dtab, tb) != hipSuccess) {
      pfsm_plan_destroy(pl);
      return PFSM_HIP_ERROR;
    }
    char* b = (char*)g.dtab;
    g.d_wstart = (int64_t*)(b + t_ws); g.d_part_start = (int64_t*)(b + t_ps);
    g.d_src_off = (int64_t*)(b + t_so); g.d_scal_off = (int64_t*)(b + t_sc);
    g.d_wsize = (int32_t*)(b + t_wz); g.d_offset = (int32_t*)(b + t_of);
    g.d_src_ld = (int32_t*)(b + t_sl); g.d_info_idx = (int32_t*)(b + t_ii);
    const bool ok = hipMemcpy(g.d_wstart, ws.data(), P * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_part_start, ps.data(), P * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_src_off, so.data(), P * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_scal_off, sc.data(), P * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_wsize, wz.data(), P * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_offset, of.data(), P * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_src_ld, sl.data(), P * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(g.d_info_idx, ii.data(), P * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
      pfsm_plan_destroy(pl);
      return PFSM_HIP_ERROR;
    }
    const size_t Mp2 = (size_t)g.Mp * g.Mp * sizeof(double);
    g.o_Bw = w; w = align256(w + P * Mp2);
    g.o_Uw = w; w = align256(w + P * Mp2);
    g.o_Rw = w; w = align256(w + 2 * P * (g.nb / 2) * B2 * B2 * sizeof(double));  // two round buffers
    g.o_rflag = w; w = align256(w + 2 * P * (g.nb / 2) * sizeof(int));
    g.o_state = w; w = align256(w + P * 2 * sizeof(int));
    g.o_stats = w; w = align256(w + P * 2 * sizeof(int));
    g.o_sel = w; w = align256(w + P * g.Mp * sizeof(int));
  }
  pl->total = w;
  // Instances run concurrently on a few internal streams (default priority),
  // joined back into the caller's stream with events, so that a stream
  // capture of pfsm_solve_batched yields one graph with parallel branches.
  const int ns = std::min<int32_t>(count, 4);
  for (int k = 0; k < ns; ++k) {
    hipStream_t st;
    hipEvent_t a, b;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
      pfsm_plan_destroy(pl);
      return PFSM_HIP_ERROR;
    }
    pl->streams.push_back(st);
    pl->fork_ev.push_back(a);
    pl->join_ev.push_back(b);
  }
  *out = pl;
  return PFSM_OK;
}

pfsm_status pfsm_solve_batched(pfsm_plan* pl, const double* const* dA, const int64_t* lda, const double* const* dV,
                               const int64_t* ldv, double* const* dLam, double* const* dVout, const int64_t* ldvo,
                               void* dWork, size_t work_bytes, int32_t* dInfo, void* stream) {
  if (!pl || pl->sub.empty() || !dA || !lda || !dV || !ldv || !dLam || !dVout || !ldvo || !dWork || !dInfo)
    return PFSM_INVALID_ARG;
  if (((uintptr_t)dWork) % 256 != 0) return PFSM_INVALID_ARG;
  if (work_bytes < pl->total) return PFSM_WORKSPACE_TOO_SMALL;
  const int count = (int)pl->sub.size();
  // Validate every instance before enqueuing anything: each instance's own
  // checks (as pfsm_solve), and no output range of one instance overlapping an
  // output or input range of another (the instances run concurrently).
  struct Range {
    const char* p;
    size_t b;
  };
  std::vector<Range> outs, ins;
  for (int i = 0; i < count; ++i) {
    const pfsm_plan* q = pl->sub[i];
    const int64_t n = q->n;
    if (!dA[i] || !dV[i] || !dLam[i] || !dVout[i]) return PFSM_INVALID_ARG;
    const pfsm_status st = check_solve_args(q, dA[i], lda[i], dV[i], ldv[i], dLam[i], dVout[i], ldvo[i],
                                            (char*)dWork + pl->sub_off[i], q->total, dInfo + i);
    if (st != PFSM_OK) return st;
    outs.push_back({(const char*)dLam[i], (size_t)n * sizeof(double)});
    outs.push_back({(const char*)dVout[i], (size_t)(ldvo[i] * (n - 1) + n) * sizeof(double)});
    ins.push_back({(const char*)dA[i], (size_t)(lda[i] * (n - 1) + n) * sizeof(double)});
    ins.push_back({(const char*)dV[i], (size_t)(ldv[i] * (n - 1) + n) * sizeof(double)});
  }
  for (size_t a = 0; a < outs.size(); ++a) {
    const int ia = (int)(a / 2);
    if (overlaps(outs[a].p, outs[a].b, dInfo, count * sizeof(int32_t)) ||
        overlaps(outs[a].p, outs[a].b, dWork, pl->total))
      return PFSM_INVALID_ARG;
    for (size_t b = 0; b < outs.size(); ++b)
      if ((int)(b / 2) != ia && overlaps(outs[a].p, outs[a].b, outs[b].p, outs[b].b)) return PFSM_INVALID_ARG;
    for (size_t b = 0; b < ins.size(); ++b)
      if ((int)(b / 2) != ia && overlaps(outs[a].p, outs[a].b, ins[b].p, ins[b].b)) return PFSM_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  const int ns = (int)pl->streams.size();
  for (int k = 0; k < ns; ++k) {
    PFSM_TRY(hipEventRecord(pl->fork_ev[k], s));
    PFSM_TRY(hipStreamWaitEvent(pl->streams[k], pl->fork_ev[k], 0));
  }
  // largest instances first, round-robin over the streams
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pl->sub[a]->n > pl->sub[b]->n; });
  char* W = (char*)dWork;
  auto half = [&](int i, int phase, const EighBatch* view, hipStream_t st) {
    pfsm_plan* q = pl->sub[i];
    char* Wi = W + pl->sub_off[i];
    if (q->precision == PFSM_PREC_MIXED_BF16)
      return solve_mixed(q, dA[i], lda[i], dV[i], ldv[i], dLam[i], dVout[i], ldvo[i], Wi, dInfo + i, st, phase,
                         view);
    return solve_fp64(q, dA[i], lda[i], dV[i], ldv[i], dLam[i], dVout[i], ldvo[i], Wi, dInfo + i, st, phase, view);
  };
  // join every internal stream back into the caller's stream (also after a
  // failed enqueue, so that nothing enqueued so far is left unjoined)
  auto join = [&](pfsm_status r) {
    for (int k = 0; k < ns; ++k) {
      const hipError_t e1 = hipEventRecord(pl->join_ev[k], pl->streams[k]);
      const hipError_t e2 = hipStreamWaitEvent(s, pl->join_ev[k], 0);
      if (r == PFSM_OK && (e1 != hipSuccess || e2 != hipSuccess)) r = PFSM_HIP_ERROR;
    }
    return r;
  };
  // 1. every instance up to its submatrices (basis change, step length)
  pfsm_status result = PFSM_OK;
  for (int t = 0; t < count && result == PFSM_OK; ++t) result = half(order[t], PH_BEGIN, nullptr, pl->streams[t % ns]);
  result = join(result);
  if (result != PFSM_OK) return result;
  // 2. one eigensolver run per group of instances, on the caller's stream
  for (const auto& g : pl->groups) {
    EighBatch e = {};
    e.P = g.P; e.Mp = g.Mp; e.nb = g.nb; e.inner_max_sweeps = EIGH_INNER_SWEEPS;
    e.Bw = (double*)(W + g.o_Bw); e.Uw = (double*)(W + g.o_Uw); e.Rw = (double*)(W + g.o_Rw);
    e.rflag = (int*)(W + g.o_rflag); e.state = (int*)(W + g.o_state); e.stats = (int*)(W + g.o_stats);
    e.sel = (int*)(W + g.o_sel);
    e.wstart = g.d_wstart; e.wsize = g.d_wsize; e.offset = g.d_offset; e.part_start = g.d_part_start;
    e.wbase = W; e.src_off = g.d_src_off; e.src_ld = g.d_src_ld; e.scal_off = g.d_scal_off;
    e.src_f32 = g.floor_rel > 0.0;  // a mixed-precision group (its instances' At in FP32)
    e.info_base = dInfo; e.info_idx = g.d_info_idx;
    e.floor_rel = g.floor_rel;
    e.angle = g.angle;
    PFSM_TRY(eigh_batched_run(e, (const double*)nullptr, 0, g.max_sweeps, s));
  }
  // 3. every instance from its start vectors on, reading its submatrices'
  // eigenpairs through a view of its group's arrays
  for (int k = 0; k < ns; ++k) {
    PFSM_TRY(hipEventRecord(pl->fork_ev[k], s));
    PFSM_TRY(hipStreamWaitEvent(pl->streams[k], pl->fork_ev[k], 0));
  }
  std::vector<EighBatch> views(count);
  for (const auto& g : pl->groups)
    for (size_t m = 0; m < g.members.size(); ++m) {
      const int i = g.members[m];
      const pfsm_plan* q = pl->sub[i];
      const size_t p0 = (size_t)g.p0[m];
      EighBatch& v = views[i];
      v = {};
      v.P = q->P; v.Mp = g.Mp; v.nb = g.nb; v.inner_max_sweeps = EIGH_INNER_SWEEPS; v.floor_rel = g.floor_rel;
      v.angle = g.angle;
      v.Bw = (double*)(W + g.o_Bw) + p0 * g.Mp * g.Mp;
      v.Uw = (double*)(W + g.o_Uw) + p0 * g.Mp * g.Mp;
      v.Rw = nullptr;  // the pair rotations are not read after the eigensolver run
      v.rflag = nullptr;
      v.state = (int*)(W + g.o_state) + 2 * p0;
      v.stats = (int*)(W + g.o_stats) + 2 * p0;
      v.sel = (int*)(W + g.o_sel) + p0 * g.Mp;
      v.wstart = q->d_wstart; v.wsize = q->d_wsize; v.offset = q->d_offset; v.part_start = q->d_part_start;
      v.info = dInfo + i;
      v.scal = (const double*)(W + pl->sub_off[i] + q->o_scal);
    }
  for (int t = 0; t < count && result == PFSM_OK; ++t) {
    const int i = order[t];
    result = half(i, PH_END, &views[i], pl->streams[t % ns]);
  }
  return join(result);
}

int32_t pfsm_batch_count(const pfsm_plan* pl) { return pl ? (int32_t)pl->sub.size() : 0; }

int32_t pfsm_refine_digit_count(void) { return REFINE_OZ_SLICES; }

pfsm_status pfsm_residuals(const pfsm_plan* pl, const void* dWork, size_t work_bytes, double* dR, void* stream) {
  if (!pl || !dWork || !dR || !pl->sub.empty()) return PFSM_INVALID_ARG;
  if (!pl->residuals) return PFSM_NOT_SUPPORTED;
  if (work_bytes < pl->total) return PFSM_WORKSPACE_TOO_SMALL;
  const size_t bytes = (size_t)pl->n * sizeof(double);
  if (overlaps(dR, bytes, dWork, pl->total)) return PFSM_INVALID_ARG;
  return hip_status(hipMemcpyAsync(dR, (const char*)dWork + pl->o_resid, bytes, hipMemcpyDeviceToDevice,
                                   (hipStream_t)stream));
}

// Tile autotuning for the split-BF16 products: time each configuration of
// the N x N x N product on the plan's workspace, on pseudo-random operands
// packed like real ones (the clock under these products depends on the
// data), and keep the fastest.  Choices are remembered per process and, when
// PFSM_TUNE_CACHE names a file, persisted there as lines
// "<gfx arch> <HIP runtime version> x3 <n> <cfg> <ms>", so a later process on
// the same architecture and runtime takes the stored choice without timing.
namespace {
std::mutex g_tune_mu;
std::vector<std::pair<std::string, int>> g_tune;  // key -> configuration
bool g_tune_loaded = false;

std::string tune_key(int64_t n) {
  int dev = 0, ver = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch = arch.substr(0, c);
  }
  (void)hipRuntimeGetVersion(&ver);
  return arch + " " + std::to_string(ver) + " x3 " + std::to_string((long long)n);
}

void tune_load() {  // g_tune_mu held
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("PFSM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char a[128], k[16];
  long long ver = 0, n = 0;
  int cfg = -1;
  double ms = 0.0;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    if (std::sscanf(line, "%127s %lld %15s %lld %d %lf", a, &ver, k, &n, &cfg, &ms) == 6 && cfg >= 0 &&
        cfg < X3_NUM_CFG)
      g_tune.push_back({std::string(a) + " " + std::to_string(ver) + " " + k + " " + std::to_string(n), cfg});
  }
  std::fclose(f);
}

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load();
  for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
    if (it->first == key) return it->second;
  return -1;
}

void tune_store(const std::string& key, int cfg, float ms) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load();
  g_tune.push_back({key, cfg});
  const char* path = std::getenv("PFSM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %.4f\n", key.c_str(), cfg, (double)ms);
  std::fclose(f);
}
}  // namespace

pfsm_status pfsm_autotune(pfsm_plan* pl, void* dWork, size_t work_bytes, int32_t* chosen, void* stream) {
  if (!pl || !dWork || work_bytes < pl->total) return PFSM_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (!pl->sub.empty()) {
    for (size_t i = 0; i < pl->sub.size(); ++i) {
      pfsm_status st = pfsm_autotune(pl->sub[i], (char*)dWork + pl->sub_off[i], pl->sub[i]->total, nullptr, stream);
      if (st != PFSM_OK) return st;
    }
    if (chosen) *chosen = -1;
    return PFSM_OK;
  }
  if (pl->precision != PFSM_PREC_MIXED_BF16) {
    if (chosen) *chosen = -1;
    return PFSM_OK;
  }
  const int64_t n = pl->n;
  const std::string key = tune_key(n);
  const int known = tune_lookup(key);
  if (known >= 0) {
    pl->x3_cfg = known;
    if (chosen) *chosen = known;
    return PFSM_OK;
  }
  const int64_t ldp = x3_row_stride(n);
  char* W = (char*)dWork;
  float* Y32 = (float*)(W + pl->m_Y32);
  // operands: pseudo-random matrices through the regular packing
  PFSM_TRY(fill_hash_f32(Y32, n * n, 0x1234567u, s));
  PFSM_TRY(pack_x3(Y32, 0, n, n, n, 0, (bf16_t*)(W + pl->m_Apk), ldp, s));
  PFSM_TRY(fill_hash_f32(Y32, n * n, 0x89abcdefu, s));
  PFSM_TRY(pack_x3(Y32, 0, n, n, n, 0, (bf16_t*)(W + pl->m_Vpk), ldp, s));
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PFSM_HIP_ERROR;
  float best = 1e30f;
  int best_cfg = 0;
  pfsm_status st = PFSM_OK;
  for (int cfg = 0; cfg < X3_NUM_CFG && st == PFSM_OK; ++cfg) {
    X3Args g = {};
    g.M = n; g.N = n; g.K = n; g.Ap = (bf16_t*)(W + pl->m_Apk); g.ldap = ldp; g.Bp = (bf16_t*)(W + pl->m_Vpk);
    g.ldbp = ldp; g.C = Y32; g.ldc = n; g.alpha = 1.0; g.cfg = cfg;
    float ms = 0.f;
    if (gemm_x3(X3_STORE, g, s) != hipSuccess || hipEventRecord(e0, s) != hipSuccess) { st = PFSM_HIP_ERROR; break; }
    for (int r = 0; r < 3 && st == PFSM_OK; ++r)
      if (gemm_x3(X3_STORE, g, s) != hipSuccess) st = PFSM_HIP_ERROR;
    if (st != PFSM_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = PFSM_HIP_ERROR;
      break;
    }
    if (ms < best) {
      best = ms;
      best_cfg = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PFSM_OK) return st;
  pl->x3_cfg = best_cfg;
  tune_store(key, best_cfg, best / 3.0f);
  if (chosen) *chosen = best_cfg;
  return PFSM_OK;
}

pfsm_status pfsm_set_tile_config(pfsm_plan* pl, int32_t cfg) {
  if (!pl || cfg < -1 || cfg >= X3_NUM_CFG) return PFSM_INVALID_ARG;
  pl->x3_cfg = cfg;
  for (pfsm_plan* q : pl->sub) q->x3_cfg = cfg;
  return PFSM_OK;
}

pfsm_status pfsm_timing_begin(pfsm_plan* pl, int32_t max_solves) {
  if (!pl || max_solves < 1 || max_solves > 4096) return PFSM_INVALID_ARG;
  pfsm_timing_end(pl);
  pl->tev.resize((size_t)max_solves * PFSM_TIMING_BOUNDS);
  for (auto& ev : pl->tev)
    if (hipEventCreate(&ev) != hipSuccess) return PFSM_HIP_ERROR;
  pl->t_max = max_solves;
  pl->t_count = 0;
  return PFSM_OK;
}

pfsm_status pfsm_timing_read(pfsm_plan* pl, float* ms, int32_t capacity, int32_t* solves) {
  if (!pl || !ms || !solves) return PFSM_INVALID_ARG;
  const int per = PFSM_TIMING_BOUNDS - 1;
  if (capacity < pl->t_count * per) return PFSM_INVALID_ARG;
  for (int sv = 0; sv < pl->t_count; ++sv) {
    hipEvent_t* e = &pl->tev[(size_t)sv * PFSM_TIMING_BOUNDS];
    if (hipEventSynchronize(e[PFSM_TIMING_BOUNDS - 1]) != hipSuccess) return PFSM_HIP_ERROR;
    for (int k = 0; k < per; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, e[k], e[k + 1]) != hipSuccess) return PFSM_HIP_ERROR;
      ms[sv * per + k] = t;
    }
  }
  *solves = pl->t_count;
  return PFSM_OK;
}

pfsm_status pfsm_timing_end(pfsm_plan* pl) {
  if (!pl) return PFSM_INVALID_ARG;
  for (auto& ev : pl->tev) (void)hipEventDestroy(ev);
  pl->tev.clear();
  pl->t_max = 0;
  pl->t_count = 0;
  return PFSM_OK;
}

pfsm_status pfsm_backward(pfsm_plan* pl, const double* dLam, const double* dV, int64_t ldv, const double* gLam,
                          const double* gV, int64_t ldg, double eta, double* dGradA, int64_t ldga, void* dWork,
                          size_t work_bytes, int32_t* dInfo, void* stream) {
  if (!pl || !dLam || !dV || !dGradA || !dWork || !dInfo) return PFSM_INVALID_ARG;
  const int64_t n = pl->n;
  if (ldv < n || ldga < n || (gV && ldg < n)) return PFSM_INVALID_ARG;
  if (!(eta >= 0.0)) return PFSM_INVALID_ARG;
  if (((uintptr_t)dWork) % 256 != 0) return PFSM_INVALID_ARG;
  if (work_bytes < pl->total) return PFSM_WORKSPACE_TOO_SMALL;
  const size_t bG = (size_t)(ldga * (n - 1) + n) * sizeof(double);
  const size_t bV = (size_t)(ldv * (n - 1) + n) * sizeof(double);
  if (overlaps(dGradA, bG, dV, bV) || overlaps(dGradA, bG, dWork, pl->total) ||
      overlaps(dGradA, bG, dLam, n * sizeof(double)))
    return PFSM_INVALID_ARG;
  if (gV && overlaps(dGradA, bG, gV, (size_t)(ldg * (n - 1) + n) * sizeof(double))) return PFSM_INVALID_ARG;
  if (gLam && overlaps(dGradA, bG, gLam, n * sizeof(double))) return PFSM_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)dWork;
  double* T = (double*)(W + pl->o_b0);
  double* G = (double*)(W + pl->o_b1);
  PFSM_TRY(fill_i32((int*)dInfo, 1, 0, s));
  if (pl->precision == PFSM_PREC_MIXED_BF16 && (pl->flags & PFSM_FLAG_BACKWARD_SPLIT)) {
    // split-BF16 products (about 16 significant bits); the middle factor in FP64
    const int64_t ldp = x3_row_stride(n);
    bf16_t* Pa = (bf16_t*)(W + pl->m_Apk);
    bf16_t* Pb = (bf16_t*)(W + pl->m_Vpk);
    bf16_t* Pr = (bf16_t*)(W + pl->m_Rpk);
    auto x3 = [&](const bf16_t* Ap, const bf16_t* Bp, void* C, int64_t ldc, int c_double) {
      // split-BF16 product with FP64 output
      X3Args g = {};
      g.M = n; g.N = n; g.K = n; g.Ap = Ap; g.ldap = ldp; g.Bp = Bp; g.ldbp = ldp; g.C = C; g.ldc = ldc;
      g.c_double = c_double; g.alpha = 1.0; g.cfg = pl->x3_cfg;
      return gemm_x3(X3_STORE, g, s);
    };
    if (gV) {
      // T = V^T gV in FP64: its antisymmetric part is multiplied by 1/gap in the middle factor
      GemmArgs g = {};
      g.M = n; g.N = n; g.K = n; g.A = dV; g.lda = ldv; g.B = gV; g.ldb = ldg; g.C = T; g.ldc = n; g.alpha = 1.0;
      PFSM_TRY(gemm_f64(true, false, EPI_STORE, g, s));
    }
    PFSM_TRY(adjoint_middle(T, n, n, dLam, gLam, eta, gV != nullptr, s));  // symmetric M
    PFSM_TRY(pack_x3(dV, 1, n, n, ldv, PACK_BY_ROWS, Pr, ldp, s));  // rows of V
    PFSM_TRY(pack_x3(T, 1, n, n, n, 0, Pb, ldp, s));                // columns of M
    PFSM_TRY(x3(Pr, Pb, G, n, 1));                                  // G = V M
    PFSM_TRY(pack_x3(G, 1, n, n, n, PACK_BY_ROWS, Pa, ldp, s));     // rows of G
    PFSM_TRY(x3(Pa, Pr, dGradA, ldga, 1));                          // dA = G V^T (columns of V^T = rows of V)
    PFSM_TRY(symmetrize(dGradA, n, ldga, s));
    return hip_status(hipGetLastError());
  }
  if (gV) {
    GemmArgs g = {};
    g.M = n; g.N = n; g.K = n; g.A = dV; g.lda = ldv; g.B = gV; g.ldb = ldg; g.C = T; g.ldc = n; g.alpha = 1.0;
    PFSM_TRY(gemm_f64(true, false, EPI_STORE, g, s));  // T = V^T gV
  }
  PFSM_TRY(adjoint_middle(T, n, n, dLam, gLam, eta, gV != nullptr, s));  // M = diag(glam) + F o T
  {
    GemmArgs g = {};
    g.M = n; g.N = n; g.K = n; g.A = dV; g.lda = ldv; g.B = T; g.ldb = n; g.C = G; g.ldc = n; g.alpha = 1.0;
    PFSM_TRY(gemm_f64(false, false, EPI_STORE, g, s));  // G = V M
    GemmArgs h = {};
    h.M = n; h.N = n; h.K = n; h.A = G; h.lda = n; h.B = dV; h.ldb = ldv; h.C = dGradA; h.ldc = ldga; h.alpha = 1.0;
    PFSM_TRY(gemm_f64(false, true, EPI_STORE, h, s));  // dA = G V^T
  }
  PFSM_TRY(symmetrize(dGradA, n, ldga, s));
  return hip_status(hipGetLastError());
}

pfsm_status pfsm_diagnostics(pfsm_plan* pl, const double* dA, int64_t lda, const double* dLam, const double* dV,
                             int64_t ldv, double* dOut, void* dWork, size_t work_bytes, void* stream) {
  if (!pl || !dA || !dLam || !dV || !dOut || !dWork) return PFSM_INVALID_ARG;
  const int64_t n = pl->n;
  if (lda < n || ldv < n) return PFSM_INVALID_ARG;
  if (((uintptr_t)dWork) % 256 != 0) return PFSM_INVALID_ARG;
  if (work_bytes < pl->total) return PFSM_WORKSPACE_TOO_SMALL;
  const size_t bV = (size_t)(ldv * (n - 1) + n) * sizeof(double);
  if (overlaps(dV, bV, dWork, pl->total) || overlaps(dLam, n * sizeof(double), dWork, pl->total))
    return PFSM_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)dWork;
  double* AV = (double*)(W + pl->o_b0);
  double* G = (double*)(W + pl->o_b1);
  double* part = (double*)(W + pl->o_part);
  GemmArgs g = {};
  g.M = n; g.N = n; g.K = n; g.A = dA; g.lda = lda; g.B = dV; g.ldb = ldv; g.C = AV; g.ldc = n; g.alpha = 1.0;
  PFSM_TRY(gemm_f64(true, false, EPI_STORE, g, s));  // A symmetric
  GemmArgs h = {};
  h.M = n; h.N = n; h.K = n; h.A = dV; h.lda = ldv; h.B = dV; h.ldb = ldv; h.C = G; h.ldc = n; h.alpha = 1.0;
  PFSM_TRY(gemm_f64(true, false, EPI_STORE, h, s));
  PFSM_TRY(diag_sums(dA, lda, AV, n, dV, ldv, dLam, G, n, n, part, dOut, s));
  return hip_status(hipGetLastError());
}

}  // extern "C"
