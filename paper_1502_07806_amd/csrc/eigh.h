// Batched submatrix eigensolver interface (internal to libpfsm).
#pragma once
#include "common.h"

namespace pfsm {

constexpr int EIGH_B = 32;                 // column-block width; pair problems are 2b x 2b
constexpr double EIGH_PAD_DIAG = 1e200;    // decoupled padding eigenvalue (sorts last)
constexpr int PFSM_INFO_EIGH_NOCONV = -3;  // a submatrix needed rotations in its last sweep
constexpr int EIGH_INNER_SWEEPS = 30;      // sweep limit of the in-LDS pair solver (4-6 are typical)
// Rotation floor of the mixed path, relative to the Gershgorin bound of the
// full matrix: 2^-24, the unit roundoff of FP32.  That path forms the
// projected matrix with split-BF16 products, whose rounding (about 2^-16
// relative) lies far above this floor, and rounds its start vectors to FP32;
// rotating entries below 2^-24 ||B|| would resolve nothing the inputs hold.
constexpr double EIGH_FLOOR_MIXED = 5.9604644775390625e-08;  // 2^-24
// Stopping rule of that path's pair problems: a one-sided Jacobi sweep whose
// rotations all had |sin| <= 2^-14 ends the iteration.  Cyclic Jacobi
// converges quadratically, so the column inner products left are of order
// 2^-28 relative, a sixteenth of the rotation floor above; the FP64 path
// iterates to its rounding level instead.
constexpr double EIGH_ANGLE_MIXED = 6.103515625e-05;  // 2^-14

struct EighBatch {
  int P;                   // number of submatrices
  int Mp;                  // padded order (multiple of 2b), common to all
  int nb;                  // Mp / b (even)
  int inner_max_sweeps;    // sweeps of the in-LDS pair solver
  double floor_rel;        // rotation floor relative to the Gershgorin bound (0: the FP64 rounding floor)
  double angle;            // pair-problem stopping rotation |sin| (0: the FP64 one)
  double* Bw;              // [P][Mp][Mp] working matrices (column-major)
  double* Uw;              // [P][Mp][Mp] accumulated eigenvectors
  double* Rw;              // [2][P][nb/2][2b][2b] pair rotations, by round parity
  int* rflag;              // [2][P][nb/2] 1 if the pair's rotation is not the identity, by round parity
  int* state;              // [P][2] {done, rotated-this-sweep}
  int* stats;              // [P][2] {sweep found converged (0: not), rotating pair problems}
  int* sel;                // [P][Mp] ascending rank -> local index
  const int64_t* wstart;   // [P] first row/column of the submatrix in At
  const int32_t* wsize;    // [P] order M_p
  const int32_t* offset;   // [P] rank of the slice's first eigenpair inside the submatrix
  const int64_t* part_start;  // [P] first global column of the slice
  int* info;               // device info word (first error wins)
  const double* scal;      // device scalars; scal[1], scal[2] = Gershgorin interval of the full matrix
  // Submatrices of several independent instances solved together (all null
  // for one instance): submatrix p reads its matrix at wbase + src_off[p]
  // (bytes; leading dimension src_ld[p]), its Gershgorin scalars at
  // wbase + scal_off[p], and reports to info_base[info_idx[p]].
  const char* wbase;
  const int64_t* src_off;
  int src_f32;             // those matrices are FP32 (the mixed path's At)
  const int32_t* src_ld;
  const int64_t* scal_off;
  int* info_base;
  const int32_t* info_idx;
};

// The submatrices are read from At (FP64, or FP32 widened exactly); with
// src_off they come from each instance's own matrix, FP32 when src_f32.
hipError_t eigh_batched_run(const EighBatch& e, const double* At, int64_t ldat, int max_sweeps, hipStream_t s);
hipError_t eigh_batched_run(const EighBatch& e, const float* At, int64_t ldat, int max_sweeps, hipStream_t s);
hipError_t embed_start_vectors(const EighBatch& e, double* X, int64_t ldx, double* eps, int64_t n, hipStream_t s);
// The same with X0 rounded to FP32 (the mixed path's master copy).
hipError_t embed_start_vectors(const EighBatch& e, float* X, int64_t ldx, double* eps, int64_t n, hipStream_t s);

}  // namespace pfsm
