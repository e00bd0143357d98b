// Total order used to rank eigenvalues (shared by device kernels and the
// host-side unit test).  NaN sorts after +inf; equal keys are ordered by
// index, so the ranks of any input -- including NaN and infinities -- form a
// permutation of 0..n-1 and can be used as indices.
#pragma once
#ifdef __HIPCC__
#define PFSM_HD __host__ __device__
#else
#define PFSM_HD
#endif

namespace pfsm {

PFSM_HD inline bool order_before(double xj, long long j, double xi, long long i) {
  const bool nj = xj != xj, ni = xi != xi;  // NaN tests without <cmath>
  if (nj || ni) {
    if (nj && ni) return j < i;
    return ni;  // a number comes before NaN
  }
  return xj < xi || (xj == xi && j < i);
}

}  // namespace pfsm
