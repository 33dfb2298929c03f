// Host-side accuracy check of the kernels' branch-free logarithm against the C library log.
// Prints: max error in ulps of the result, number of samples, and special-case results.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include "../../paper_2404_02628_amd/csrc/fast_exp.h"

int main() {
  double worst = 0.0, worst_x = 0.0;
  long n = 0;
  uint64_t s = 88172645463325252ull;
  for (long i = 0; i < 4000000; ++i) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    double u = (double)(s >> 11) * 0x1.0p-53;          // [0,1)
    double x = std::exp2(-1000.0 + 2000.0 * u);         // 2^-1000 .. 2^1000
    if (i % 4 == 1) x = 1.0 + 0x1.0p64 * u;              // the recursion's range [1, 2^64]
    if (i % 4 == 2) x = 0.5 + u;                         // around 1
    if (i % 4 == 3) x = (double)(1 + (s >> 44));         // integers up to 2^20
    double ref = std::log(x), got = pimd::fast_log(x);
    double ulp = std::fabs(ref) > 0 ? std::ldexp(1.0, std::ilogb(ref) - 52) : 0x1.0p-1074;
    double err = std::fabs(got - ref) / ulp;
    if (err > worst) { worst = err; worst_x = x; }
    ++n;
  }
  printf("max_ulp %.3f at %.17g samples %ld\n", worst, worst_x, n);
  printf("special %g %g %g %d %d %g\n", pimd::fast_log(1.0), pimd::fast_log(0.0), pimd::fast_log(INFINITY),
         (int)std::isnan(pimd::fast_log(-1.0)), (int)std::isnan(pimd::fast_log(NAN)),
         pimd::fast_log(0x1.0p-1070) / std::log(0x1.0p-1070));
  return 0;
}
