// k_integrate.hip -- velocity Verlet with massive Nose-Hoover chains, estimators, density.
//
// The paper samples exp(-beta (V_xi + U/P)) by molecular dynamics with massive Nose-Hoover
// chains (Sec. IV.A).  Every Cartesian bead coordinate has its own chain of length M with
// masses Q and target k_B T = 1/beta.  A step is
//   NHC(dt/2); p += F dt/2; x += p dt/m'; F = force(x); p += F dt/2; NHC(dt/2),
// where NHC(tau) is the Suzuki-Yoshida factorised chain propagator of Martyna, Tuckerman,
// Tobias and Klein (Mol. Phys. 87, 1117 (1996)) with one multiple-time-step cycle.
// All of it is FP64 and elementwise over degrees of freedom (HBM-bound).
#include "pimd_internal.h"
#include "device_util.h"
#include "nhc.h"

namespace pimd {

// Thread -> degree of freedom.  Work item {rep, first dof} covers kIntBlock consecutive dofs of
// one replica; dofs are elementwise-independent, so the launch is a flat coalesced stream.
// mode 0: first half  (NHC(dt/2), p += F dt/2, x += p dt/m')
// mode 1: second half (F = F + F_pair, then p += F dt/2, NHC(dt/2))
// mode 2: F = F + F_pair only (force evaluation without integration)
// mode 3: second half of this step fused with the first half of the next one
// A thread whose force, momentum or new position is not finite raises the non-finite status
// word; once a status word is raised no integrator pass writes anything.  The chain positions
// are kept as sums only (they enter nothing but H'): each wave adds its increment to its own
// slot of etasum, in a fixed order, so the sums are reproducible.
// One degree of freedom of k_integrate, from its operands in registers: writes x, p, f and the
// chain velocities (and raises the status word on a non-finite value) only when `store` is set;
// the chain-position increments go to es.  The arithmetic runs whether or not the lane stores, so
// that its operands are loaded unconditionally at the top of the kernel and the status word is
// only waited for at the first store.
template <int M, int MODE>
__device__ inline void integrate_one(const RepDev& R, int rep, long long gi, double fv, double fpv, double pv,
                                     double xv, double& es, double (&v)[M > 0 ? M : 1], double* __restrict__ x,
                                     double* __restrict__ p, double* __restrict__ f, double* __restrict__ veta,
                                     long long G, double hdt, const SyW& sy, bool store, int* status) {
  constexpr bool kPair = MODE != 0;
  constexpr bool kChain = M > 0 && MODE != 2;
  if (kPair) fv = R.amp > 0.0 ? fv + fpv : fv;
  if (MODE == 0) {
    if (M > 0) nhc_propagate<true>(pv, R.inv_mp, es, v, M, R.inv_q, R.kT, hdt, sy);
    pv += hdt * fv;
    const double xn = xv + R.dt_mp * pv;
    if (!store) return;
    if (!isfinite(fv) || !isfinite(xn)) status_nonfinite(status, rep);
    x[gi] = xn;
    p[gi] = pv;
  } else {
    if (MODE == 2) {
      if (!store) return;
      f[gi] = fv;
      if (!isfinite(fv)) status_nonfinite(status, rep);
      return;
    }
    const double ftot = fv;
    pv += hdt * fv;
    if (M > 0) nhc_propagate<true>(pv, R.inv_mp, es, v, M, R.inv_q, R.kT, hdt, sy);
    double xn = 0.0;
    if (MODE == 3) {
      // second thermostat half-step of this step and first of the next, chain in registers
      if (M > 0) nhc_propagate<true>(pv, R.inv_mp, es, v, M, R.inv_q, R.kT, hdt, sy);
      pv += hdt * fv;
      xn = xv + R.dt_mp * pv;
    }
    if (!store) return;
    // the total force is kept for readers of the last evaluation; in the fused pass the next
    // evaluation overwrites it unread
    if (MODE != 3) f[gi] = ftot;
    if (MODE == 3) x[gi] = xn;
    if (!isfinite(fv) || !isfinite(pv) || !isfinite(xn)) status_nonfinite(status, rep);
    p[gi] = pv;
  }
  if (kChain) {
#pragma unroll
    for (int k = 0; k < M; ++k) veta[k * G + gi] = v[k];
  }
}

template <int M, int MODE>
__global__ __launch_bounds__(kIntBlock) void k_integrate(const RepDev* __restrict__ reps,
                                                         const int4* __restrict__ work, double* __restrict__ x,
                                                         double* __restrict__ p, double* __restrict__ f,
                                                         const double* __restrict__ fpair,
                                                         double* __restrict__ etasum, double* __restrict__ veta,
                                                         long long G, SyW sy, int* status) {
  const int4 wk = work[blockIdx.x];
  const bool ok = (int)threadIdx.x < wk.y;
  const long long gi = int_work_first(wk) + (ok ? (int)threadIdx.x : 0);
  const RepDev& R = reps[wk.x];   // read while the loads below are in flight
  const double hdt = 0.5 * R.dt;
  // Every operand is loaded up front, so a thread waits out one memory latency rather than one
  // per dependence.  The pair forces are read even without a pair term (the buffer is part of
  // the workspace either way) and selected away.
  constexpr bool kX = MODE == 0 || MODE == 3;
  constexpr bool kP = MODE != 2;
  constexpr bool kPair = MODE != 0;
  constexpr bool kChain = M > 0 && MODE != 2;
  const double fv = f[gi];
  const double fpv = kPair ? fpair[gi] : 0.0;
  const double pv = kP ? p[gi] : 0.0;
  const double xv = kX ? x[gi] : 0.0;
  const bool halted = status_halted(status);
  double es = 0.0, v[M > 0 ? M : 1];
#pragma unroll
  for (int k = 0; k < (M > 0 ? M : 1); ++k) v[k] = kChain ? veta[k * G + gi] : 0.0;
  const bool store = ok && !halted;
  integrate_one<M, MODE>(R, wk.x, gi, fv, fpv, pv, xv, es, v, x, p, f, veta, G, hdt, sy, store, status);
  if constexpr (kChain) {
    // every lane takes part in its wave's chain-position sum
    es = wave_sum(store ? es : 0.0);
    if ((threadIdx.x & 63) == 0 && !halted) etasum[(long long)blockIdx.x * kEtaSlots + (threadIdx.x >> 6)] += es;
  }
}

// One workgroup per replica: kinetic and thermostat energies over all dofs plus the
// partial sums left by the spring, pair and end-bead kernels, in a fixed order.
__global__ __launch_bounds__(256) void k_estimators(const RepDev* __restrict__ reps, const double* __restrict__ p,
                                                    const double* __restrict__ etasum, const double* __restrict__ veta,
                                                    const double* __restrict__ gf,
                                                    const double* __restrict__ springpart,
                                                    const double* __restrict__ pairpart,
                                                    const double* __restrict__ reducepart, double* __restrict__ rec,
                                                    double* __restrict__ trace, long long* __restrict__ tracecount,
                                                    long long G, int M, int D, int P, int cap, long long step,
                                                    int record, const int* status) {
  __shared__ double lds[2 * 4];
  __shared__ int halted;
  if (threadIdx.x == 0) halted = status_halted(status) ? 1 : 0;
  __syncthreads();
  if (halted) return;   // a halted run records nothing more
  const int r = blockIdx.x;
  const RepDev& R = reps[r];
  double acc[2] = {0.0, 0.0};
  const double kT = 1.0 / R.beta;
  // p is NULL for an evaluation without momenta (the kinetic and thermostat terms are then 0)
  for (long long li = threadIdx.x; p != nullptr && li < R.ndof; li += blockDim.x) {
    const long long gi = R.dof + li;
    const double pv = p[gi];
    acc[0] += 0.5 * pv * pv / R.mp;
    for (int k = 0; k < M; ++k) {
      const double v = veta[k * G + gi];
      acc[1] += 0.5 * R.q * v * v;
    }
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x != 0) return;
  if (M > 0) {
    double es = 0.0;
    for (long long g = R.es0; g < R.es1; ++g) es += etasum[g];
    acc[1] += kT * es;
  }
  double eint = 0.0, lk = 0.0, ut = 0.0;
  for (long long g = R.spw0; g < R.spw1; ++g) {
    eint += springpart[4 * g + 0];
    lk += springpart[4 * g + 1];
    ut += springpart[4 * g + 2];
  }
  double up = 0.0, wp = 0.0;
  if (R.amp > 0.0) {
    for (long long g = R.pw0; g < R.pw1; ++g) {
      up += pairpart[2 * g + 0];
      wp += pairpart[2 * g + 1];
    }
  }
  double sx = 0.0;
  for (long long g = R.rw0; g < R.rw1; ++g) sx += reducepart[2 * g + 0];
  const int N = R.n;
  const double S = eint + sx;
  const double V = eint + lk - gf[R.part + N] / R.beta;
  const double U = ut + up;
  double* o = rec + (long long)kRec * r;
  o[kVExch] = V;
  o[kUTrap] = ut;
  o[kUPair] = up;
  o[kSpring] = S;
  o[kVirial] = 2.0 * ut + wp;
  o[kEPrim] = (double)D * N * P / (2.0 * R.beta) - S + U / (double)P;
  o[kEVir] = (2.0 * ut + wp) / (double)P;
  o[kKinetic] = acc[0];
  o[kNhcE] = acc[1];
  o[kHCons] = acc[0] + V + U / (double)P + acc[1];
  o[kStep] = (double)step;
  o[kEintSum] = eint;
  o[kLinkSum] = lk;
  o[kPairW] = wp;
  o[kValid] = 1.0;
  o[kRecPad] = 0.0;
  if (record && cap > 0) {
    const long long c = tracecount[r];
    double* t = trace + ((long long)r * cap + (c % cap)) * kRec;
    for (int k = 0; k < kRec; ++k) t[k] = o[k];
    tracecount[r] = c + 1;
  }
}

// Radial histogram of every bead of every replica (one workgroup per spring work item,
// i.e. 256 particles, all slices).  Integer counts are exact, so atomics are deterministic.
template <int D>
__global__ __launch_bounds__(256) void k_density(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                                 const double* __restrict__ x, unsigned long long* __restrict__ dens,
                                                 long long* __restrict__ nsamp, int P, int bins, double rmax,
                                                 const int* status) {
  extern __shared__ unsigned int hist[];
  __shared__ int halted;
  if (threadIdx.x == 0) halted = status_halted(status) ? 1 : 0;
  __syncthreads();
  if (halted) return;   // a halted run records nothing more
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  const int N = R.n;
  for (int b = threadIdx.x; b <= bins; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  const int l = wk.y + threadIdx.x;
  if (l < N) {
    const double* xr = x + R.dof;
    for (int j = 0; j < P; ++j) {
      // the bin is an integer decided by floating point: evaluate |r| exactly as
      // sum of squares in component order (no contraction), then (|r|/rmax)*bins
      double r2 = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double v = xr[((long long)a * P + j) * N + l];
        r2 = __dadd_rn(r2, __dmul_rn(v, v));
      }
      double rr = __dsqrt_rn(r2);
      // NaN and |r| >= rmax go to the overflow bin
      int b = (rr < rmax) ? (int)__dmul_rn(__ddiv_rn(rr, rmax), (double)bins) : bins;
      if (b < 0) b = 0;
      if (b > bins) b = bins;
      atomicAdd(&hist[b], 1u);
    }
  }
  __syncthreads();
  unsigned long long* dr = dens + (long long)wk.x * (bins + 1);
  for (int b = threadIdx.x; b <= bins; b += blockDim.x)
    if (hist[b]) atomicAdd(&dr[b], (unsigned long long)hist[b]);
  if (threadIdx.x == 0 && blockIdx.x == R.spw0) nsamp[wk.x] += 1;
}

SyW sy_weights(int order) {
  SyW s{};
  if (order == 1) { s.w[0] = 1.0; s.n = 1; }
  else if (order == 3) {
    double a = 1.0 / (2.0 - cbrt(2.0));
    s.w[0] = a; s.w[1] = 1.0 - 2.0 * a; s.w[2] = a; s.n = 3;
  } else {
    double a = 1.0 / (4.0 - pow(4.0, 1.0 / 3.0));
    s.w[0] = a; s.w[1] = a; s.w[2] = 1.0 - 4.0 * a; s.w[3] = a; s.w[4] = a; s.n = 5;
  }
  // 1/10!, 1/9!, ..., 1/3!
  s.ec[0] = 1.0 / 3628800.0; s.ec[1] = 1.0 / 362880.0; s.ec[2] = 1.0 / 40320.0; s.ec[3] = 1.0 / 5040.0;
  s.ec[4] = 1.0 / 720.0; s.ec[5] = 1.0 / 120.0; s.ec[6] = 1.0 / 24.0; s.ec[7] = 1.0 / 6.0;
  return s;
}

template <int MODE>
static hipError_t launch_integrate_mode(const Dims& d, const DevPtrs& w, hipStream_t s) {
  if (d.nintwg == 0) return hipSuccess;
  dim3 grid((unsigned)d.nintwg), block(kIntBlock);
  const SyW sy = sy_weights(d.sy_order);
#define L(MM) hipLaunchKernelGGL((k_integrate<MM, MODE>), grid, block, 0, s, w.reps, w.intwork, w.x, w.p, w.f, \
                                 w.fpair, w.etasum, w.veta, d.G, sy, w.err)
  switch (d.M) {
    case 0: L(0); break; case 1: L(1); break; case 2: L(2); break; case 3: L(3); break;
    case 4: L(4); break; case 5: L(5); break; case 6: L(6); break; case 7: L(7); break; case 8: L(8); break;
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

hipError_t launch_integrate_first(const Dims& d, const DevPtrs& w, hipStream_t s) {
  return launch_integrate_mode<0>(d, w, s);
}

hipError_t launch_integrate_second(const Dims& d, const DevPtrs& w, bool kick, hipStream_t s) {
  return kick ? launch_integrate_mode<1>(d, w, s) : launch_integrate_mode<2>(d, w, s);
}

hipError_t launch_integrate_fused(const Dims& d, const DevPtrs& w, hipStream_t s) {
  return launch_integrate_mode<3>(d, w, s);
}

hipError_t launch_estimators(const Dims& d, const DevPtrs& w, long long step, bool record, hipStream_t s) {
  hipLaunchKernelGGL(k_estimators, dim3(d.R), dim3(256), 0, s, w.reps, w.p, w.etasum, w.veta, w.gf, w.springpart,
                     w.pairpart, w.reducepart, w.rec, w.trace, w.tracecount, d.G, d.M, d.D, d.P, d.cap, step,
                     record ? 1 : 0, w.err);
  return hipGetLastError();
}

hipError_t launch_density(const Dims& d, const DevPtrs& w, hipStream_t s) {
  if (d.nspringwg == 0) return hipSuccess;
  dim3 grid((unsigned)d.nspringwg), block(256);
  size_t sh = sizeof(unsigned int) * (size_t)(d.bins + 1);
  switch (d.D) {
    case 1: hipLaunchKernelGGL(k_density<1>, grid, block, sh, s, w.reps, w.springwork, w.x, w.dens, w.denssamples, d.P, d.bins, d.rmax, w.err); break;
    case 2: hipLaunchKernelGGL(k_density<2>, grid, block, sh, s, w.reps, w.springwork, w.x, w.dens, w.denssamples, d.P, d.bins, d.rmax, w.err); break;
    case 3: hipLaunchKernelGGL(k_density<3>, grid, block, sh, s, w.reps, w.springwork, w.x, w.dens, w.denssamples, d.P, d.bins, d.rmax, w.err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pimd
