// Host-side accuracy check of the kernels' table-driven exp against the C library exp.
// Prints: max relative error (ulps of 2^-52), number of samples, and special-case results.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include "../../paper_2404_02628_amd/csrc/fast_exp.h"

int main() {
  double tab[pimd::kExpTable];
  for (int j = 0; j < pimd::kExpTable; ++j) tab[j] = pimd::exp_table_entry(j);
  double worst = 0.0, worst_x = 0.0;
  long n = 0;
  uint64_t s = 88172645463325252ull;
  for (long i = 0; i < 4000000; ++i) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    double u = (double)(s >> 11) * 0x1.0p-53;         // [0,1)
    double x = -745.0 + 1450.0 * u;                   // [-745, 705)
    if (i % 4 == 1) x = -40.0 * u;                    // dense where the kernels live
    if (i % 4 == 2) x = 1e-3 * (u - 0.5);             // around 0
    double ref = std::exp(x), got = pimd::fast_exp(x, tab);
    if (ref < 1e-300) continue;                       // skip the subnormal range
    double rel = std::fabs(got - ref) / ref / 0x1.0p-52;
    if (rel > worst) { worst = rel; worst_x = x; }
    ++n;
  }
  printf("max_ulp %.3f at %.17g samples %ld\n", worst, worst_x, n);
  printf("special %g %g %g %g %d\n", pimd::fast_exp(0.0, tab), pimd::fast_exp(-INFINITY, tab),
         pimd::fast_exp(-800.0, tab), pimd::fast_exp(-744.0, tab) / std::exp(-744.0),
         (int)std::isnan(pimd::fast_exp(NAN, tab)));
  printf("overflow %d %d %d\n", (int)std::isinf(pimd::fast_exp(1000.0, tab)),
         (int)std::isinf(pimd::fast_exp(INFINITY, tab)), (int)std::isfinite(pimd::fast_exp(709.0, tab)));
  return 0;
}
