// nhc.h -- massive Nose-Hoover chain propagator shared by the integrator kernels.
//
// Every Cartesian bead coordinate has its own chain of length M with masses Q and target
// k_B T = 1/beta; NHC(tau) is the Suzuki-Yoshida factorised chain propagator of Martyna,
// Tuckerman, Tobias and Klein (Mol. Phys. 87, 1117 (1996)) with one multiple-time-step cycle.
// The streaming integrator and the persistent small-replica kernel both call it, so the two
// paths apply the same arithmetic to every degree of freedom, except that the streaming one may
// take a wider polynomial tier for the momentum's scale factor where the other runs the library
// exponential (results within an ulp or two of each other).
#pragma once
#include <hip/hip_runtime.h>

namespace pimd {

// Suzuki-Yoshida weights w[0..n-1], and the Taylor coefficients ec = 1/10!, 1/9!, ..., 1/3! of
// the exponentials below.  The coefficients travel as kernel arguments so that they sit in scalar
// registers: FP64 constants other than a few inline values (0.5, 1.0, ...) cannot be immediate
// operands, and kept in vector registers each one is first copied into the accumulator of a
// two-operand multiply-add.
struct SyW { double w[5]; double ec[8]; int n; };

// exp(x) for the thermostat scale factors, whose arguments (h v / 4 and h v with h a fraction
// of dt) are small.  Taylor polynomials replace the library exponential when every lane of the
// wavefront is within their bound: degree 7 for |x| <= 1/32 (remainder below 3e-17 relative),
// and, for the momentum's factor exp(-h v_1) in the streaming integrator, degree 10 for
// |x| <= 1/8 (remainder below 1.2e-18): its argument exceeds 1/32 in a few percent of lanes at
// equilibrium, so that nearly every wavefront of 64 degrees of freedom would otherwise run the
// library exponential (fused integrator 320 -> 310 us at 128 replicas of N = 1600).
__device__ inline double taylor_exp7(double x, const double (&ec)[8]) {
  double q = fma(x, ec[3], ec[4]);
  q = fma(q, x, ec[5]);
  q = fma(q, x, ec[6]);
  q = fma(q, x, ec[7]);
  q = fma(q, x, 0.5);
  q = fma(q, x, 1.0);
  return fma(q, x, 1.0);
}

__device__ inline double chain_exp(double x, const double (&ec)[8]) {
  if (__all(fabs(x) <= 0.03125)) return taylor_exp7(x, ec);
  return exp(x);
}

__device__ inline double momentum_exp(double x, const double (&ec)[8]) {
  if (__all(fabs(x) <= 0.03125)) return taylor_exp7(x, ec);
  if (__all(fabs(x) <= 0.125)) {
    double q = fma(x, ec[0], ec[1]);
#pragma unroll
    for (int k = 2; k < 8; ++k) q = fma(q, x, ec[k]);
    q = fma(q, x, 0.5);
    q = fma(q, x, 1.0);
    return fma(q, x, 1.0);
  }
  return exp(x);
}

// The chain forces are G_1 = (p^2/m' - kT)/Q and G_k = (Q v_{k-1}^2 - kT)/Q = v_{k-1}^2 - kT/Q,
// evaluated with precomputed reciprocals.  The scale factor exp(-h v_{k+1}/4) of element k is
// the same number in the inward and the outward sweep (v_{k+1} is not touched in between), so
// it is computed once per sub-step.  The chain positions eta_k only enter the conserved quantity
// H' (through kT sum_k eta_k), so the propagator adds their increments h v_k into one number,
// eta_sum, instead of keeping every eta_k.
// kWide: the momentum's factor may take the degree-10 polynomial (the streaming integrator); the
// persistent small-replica kernel, bound by its own instruction issue and whose small systems
// nearly always stay within the degree-7 bound, runs without that tier (with it, 2% slower).
template <bool kWide>
__device__ inline void nhc_propagate(double& p, double inv_mp, double& eta_sum, double* v, int M, double inv_q,
                                     double kT, double tau, const SyW& sy) {
  const double kTq = kT * inv_q;
  for (int iw = 0; iw < sy.n; ++iw) {
    const double h = sy.w[iw] * tau;
    double sc[kMaxNhc];
    {
      double Gm = (M == 1) ? fma(p * p, inv_mp * inv_q, -kTq) : fma(v[M - 2], v[M - 2], -kTq);
      v[M - 1] += 0.5 * h * Gm;
    }
    for (int k = M - 2; k >= 0; --k) {
      sc[k] = chain_exp(-0.25 * h * v[k + 1], sy.ec);
      double Gk = (k == 0) ? fma(p * p, inv_mp * inv_q, -kTq) : fma(v[k - 1], v[k - 1], -kTq);
      v[k] = (v[k] * sc[k] + 0.5 * h * Gk) * sc[k];
    }
    p *= kWide ? momentum_exp(-h * v[0], sy.ec) : chain_exp(-h * v[0], sy.ec);
    double vs = 0.0;
    for (int k = 0; k < M; ++k) vs += v[k];
    eta_sum = fma(h, vs, eta_sum);
    for (int k = 0; k <= M - 2; ++k) {
      double Gk = (k == 0) ? fma(p * p, inv_mp * inv_q, -kTq) : fma(v[k - 1], v[k - 1], -kTq);
      v[k] = (v[k] * sc[k] + 0.5 * h * Gk) * sc[k];
    }
    {
      double Gm = (M == 1) ? fma(p * p, inv_mp * inv_q, -kTq) : fma(v[M - 2], v[M - 2], -kTq);
      v[M - 1] += 0.5 * h * Gm;
    }
  }
}

// Suzuki-Yoshida weights of order 1, 3 or 5.
SyW sy_weights(int order);

}  // namespace pimd
