// Host check: ranks computed with pfsm::order_before form a permutation for
// inputs with NaN, infinities and ties (the property the ranking kernels rely
// on before using ranks as indices).
#include <cmath>
#include <cstdio>
#include <limits>
#include <vector>
#include "../../paper_1502_07806_amd/csrc/order_key.h"

static int check(const std::vector<double>& x) {
  const long long n = (long long)x.size();
  std::vector<int> seen(n, 0);
  for (long long i = 0; i < n; ++i) {
    long long r = 0;
    for (long long j = 0; j < n; ++j) r += pfsm::order_before(x[j], j, x[i], i);
    if (r < 0 || r >= n || seen[r]++) return 1;
  }
  // finite values keep ascending stable order
  for (long long i = 0; i < n; ++i)
    for (long long j = 0; j < n; ++j)
      if (!std::isnan(x[i]) && !std::isnan(x[j]) && x[j] < x[i] && !pfsm::order_before(x[j], j, x[i], i)) return 2;
  return 0;
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  std::vector<std::vector<double>> cases = {
      {3, 1, 2},
      {nan, nan, nan, nan},
      {1, nan, -inf, inf, nan, 1, 0, -0.0, inf},
      {1e200, nan, 1e200, 2, nan},
      {},
  };
  int bad = 0;
  for (size_t c = 0; c < cases.size(); ++c) {
    int r = check(cases[c]);
    if (r) printf("case %zu failed (%d)\n", c, r);
    bad |= r;
  }
  printf(bad ? "FAIL\n" : "OK\n");
  return bad;
}
