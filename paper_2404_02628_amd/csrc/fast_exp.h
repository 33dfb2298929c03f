// fast_exp.h -- table-driven double-precision exponential for the FP64 kernels.
//
// Method: P. T. P. Tang, "Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15 (1989) 144.  Write x = (256 m + j) ln2/256 + r with
// integers m, j in [0, 255] and |r| <= ln2/512; then e^x = 2^m * 2^(j/256) * e^r.  2^(j/256)
// comes from a 256-entry table (2 KiB, built once per workgroup in LDS), e^r - 1 from its Taylor
// polynomial of degree 4 (truncation below 4e-17 for |r| <= 0.00136), and 2^m from ldexp, which
// also produces the gradual underflow to 0 for very negative x.  ln2/256 is split into a 32-bit
// high part (k * hi is exact for |k| < 2^21) and a low correction:
//   256/ln2 = 369.3299304675746, hi = 0x1.62e42fee00000p-9, lo = 0x1.a39ef35793c76p-41.
// The integer k nearest to x 256/ln2 comes from one fused multiply-add with 1.5 * 2^52, whose
// result has unit spacing, so the sum is rounded to an integer and k sits in its low word (valid
// for |k| < 2^31; here |k| < 2^19): one operation fewer than rounding and converting.
// About 15 vector instructions instead of ~26 for the library exp; results are within a few
// ulp, far below the 1e-10 parity bar.  The function has no branches, so the compiler can
// interleave independent calls instead of running each one's exec-masked regions in turn: the
// argument is clamped to [-800, 709.8], where ldexp itself produces the limits (exactly 0 below
// about -745.2, inf above ln(DBL_MAX) = 709.78), and only NaN is selected at the end.
#pragma once
#include <hip/hip_runtime.h>

namespace pimd {

constexpr int kExpTable = 256;

__host__ __device__ inline double exp_table_entry(int j) { return exp2((double)j / kExpTable); }

// Fills tab[0..kExpTable-1] with 2^(j/256) using every thread of the workgroup; call before
// __syncthreads().
__device__ inline void fill_exp_table(double* tab) {
  for (int j = (int)threadIdx.x; j < kExpTable; j += (int)blockDim.x) tab[j] = exp_table_entry(j);
}

// Without the NaN pass-through (one compare and two selects fewer), for the exchange sums: a NaN
// argument gives a finite weight there, but the NaN that caused it (a coordinate) also enters the
// weighted payload sums, which take it on.
__host__ __device__ inline double fast_exp_finite(double x, const double* tab) {
  const double kInvL = 369.3299304675746;          // 256 / ln 2
  const double kL1 = 0x1.62e42fee00000p-9;         // high 32 bits of ln2 / 256
  const double kL2 = 0x1.a39ef35793c76p-41;        // ln2 / 256 - kL1
  const double kShift = 6755399441055744.0;        // 1.5 * 2^52
  const double xc = fmin(fmax(x, -800.0), 709.8);  // -inf -> -800 -> 0; NaN -> -800
  const double kds = fma(xc, kInvL, kShift);       // 1.5 * 2^52 + k
  const int k = (int)(unsigned)__builtin_bit_cast(unsigned long long, kds);
  const double kd = kds - kShift;
  double r = fma(-kd, kL1, xc);
  r = fma(-kd, kL2, r);
  const int j = k & (kExpTable - 1);
  const int m = k >> 8;                            // floor(k / 256): k = 256 m + j
  // e^r - 1 = r + r^2 (1/2 + r (1/6 + r/24))
  double q = fma(r, 1.0 / 24.0, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r * r, r);
  const double t = tab[j];
  return ldexp(fma(t, q, t), m);
}

__host__ __device__ inline double fast_exp(double x, const double* tab) {
  const double v = fast_exp_finite(x, tab);
  return x != x ? x : v;
}

// Natural logarithm for the FP64 kernels, branch-free and without tables.  Write
// x = 2^e m with m in [sqrt(1/2), sqrt(2)); with u = (m - 1)/(m + 1), |u| <= 0.1716,
//   log m = 2 atanh u = 2u (1 + u^2/3 + u^4/5 + ... + u^18/19) + O(u^21/21)
// (the neglected terms are below 3e-17 of the result), and log x = e ln2 + log m with ln2 split
// into a 42-bit high part (e * hi is exact for |e| < 2^11) and a low correction:
//   hi = 0x1.62e42fefa3800p-1, lo = 0x1.ef35793c76730p-45.
// About 35 vector instructions instead of ~110 for the library log (which carries double-double
// intermediate precision); results are within a few ulp.  0 gives -inf, +inf gives +inf, and
// negative arguments and NaN give NaN.
__host__ __device__ inline double fast_log(double x) {
  const double kL2hi = 0x1.62e42fefa3800p-1;
  const double kL2lo = 0x1.ef35793c76730p-45;
  int e;
  double m = frexp(x, &e);                          // x = m 2^e, m in [1/2, 1)
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double u = (m - 1.0) / (m + 1.0);
  const double z = u * u;
  double q = fma(z, 1.0 / 19.0, 1.0 / 17.0);
  q = fma(q, z, 1.0 / 15.0);
  q = fma(q, z, 1.0 / 13.0);
  q = fma(q, z, 1.0 / 11.0);
  q = fma(q, z, 1.0 / 9.0);
  q = fma(q, z, 1.0 / 7.0);
  q = fma(q, z, 1.0 / 5.0);
  q = fma(q, z, 1.0 / 3.0);
  const double u2 = 2.0 * u;
  const double lm = fma(u2 * z, q, u2);             // 2u + 2u z q
  const double de = (double)e;
  const double v = fma(de, kL2hi, fma(de, kL2lo, lm));
  const double inf = __builtin_huge_val();
  return (x > 0.0 && x < inf) ? v : (x == 0.0 ? -inf : (x == inf ? inf : __builtin_nan("")));
}

}  // namespace pimd
