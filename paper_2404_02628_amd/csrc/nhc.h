// nhc.h -- massive Nose-Hoover chain propagator shared by the integrator kernels.
//
// Every Cartesian bead coordinate has its own chain of length M with masses Q and target
// k_B T = 1/beta; NHC(tau) is the Suzuki-Yoshida factorised chain propagator of Martyna,
// Tuckerman, Tobias and Klein (Mol. Phys. 87, 1117 (1996)) with one multiple-time-step cycle.
// The streaming integrator and the persistent small-replica kernel both call it, so the two
// paths apply the same arithmetic to every degree of freedom.
#pragma once
#include <hip/hip_runtime.h>

namespace pimd {

// Suzuki-Yoshida weights w[0..n-1], and the Taylor coefficients 1/7!, 1/6!, ..., 1/3! of
// chain_exp.  The coefficients travel as kernel arguments so that they sit in scalar registers:
// FP64 constants cannot be immediate operands, and kept in vector registers each one is first
// copied into the accumulator of a two-operand multiply-add.
struct SyW { double w[5]; double ec[5]; int n; };

// exp(x) for the thermostat scale factors, whose arguments (h v / 4 and h v with h a fraction
// of dt) are small: when every lane of the wavefront has |x| <= 1/32 the Taylor polynomial of
// degree 7 (remainder below 3e-17 relative) replaces the library exponential.  The scale factors
// of the chain elements, exp(-h v_{k+1} / 4), nearly always take the polynomial; the momentum's,
// exp(-h v_1), takes the library exponential in most wavefronts (|h v_1| exceeds 1/32 in a few
// percent of lanes at equilibrium).
__device__ inline double chain_exp(double x, const double (&ec)[5]) {
  if (__all(fabs(x) <= 0.03125)) {
    double q = fma(x, ec[0], ec[1]);
    q = fma(q, x, ec[2]);
    q = fma(q, x, ec[3]);
    q = fma(q, x, ec[4]);
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
    p *= chain_exp(-h * v[0], sy.ec);
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
