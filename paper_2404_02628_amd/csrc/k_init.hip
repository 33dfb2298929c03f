// k_init.hip -- seeded initial state on the device.
//
// Positions N(0, sigma_r^2) and momenta N(0, m'/beta) (Maxwell-Boltzmann at beta for the bead
// mass) for every coordinate of every replica, thermostat chains at rest.  The deviates come
// from the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC11), keyed
// by the replica's seed, through the Box-Muller transform, so every element is a pure function
// of (seed, array, element index): element e of array a (0 = x, 1 = p, [dim][P][N] order) is
// deviate e mod 2 of the pair drawn with counter {k mod 2^32, k / 2^32, a, 0}, k = e/2.
// One thread per element (the two threads of a pair both evaluate its generator call).
#include "pimd_internal.h"

namespace pimd {

// Ten Philox rounds: per round the products 0xD2511F53 c0 and 0xCD9E8D57 c2 give
// (c0, c1, c2, c3) <- (hi(B) ^ c1 ^ k0, lo(B), hi(A) ^ c3 ^ k1, lo(A)) with A = M0 c0,
// B = M1 c2, and the key advances by the Weyl constants (0x9E3779B9, 0xBB67AE85).
__device__ inline uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t a_lo = 0xD2511F53u * c.x, a_hi = __umulhi(0xD2511F53u, c.x);
    const uint32_t b_lo = 0xCD9E8D57u * c.z, b_hi = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(b_hi ^ c.y ^ k.x, b_lo, a_hi ^ c.w ^ k.y, a_lo);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// 53 bits from two words, centred in (0, 1): never 0, so log is finite.
__device__ inline double open_unit(uint32_t hi, uint32_t lo) {
  const unsigned long long m = ((unsigned long long)hi << 21) | (unsigned long long)(lo >> 11);
  return ((double)m + 0.5) * 0x1p-53;
}

__device__ inline double gaussian(unsigned long long seed, uint32_t array, unsigned long long e) {
  const unsigned long long k = e >> 1;
  const uint4 w = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)(k >> 32), array, 0u),
                                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
  const double u1 = open_unit(w.y, w.x), u2 = open_unit(w.w, w.z);
  const double rad = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586476925286766559 * u2;
  return (e & 1) ? rad * sin(th) : rad * cos(th);
}

// params: per replica {sigma, seed (bit pattern of a uint64 stored in a double slot)}.
__global__ __launch_bounds__(kIntBlock) void k_init_state(const RepDev* __restrict__ reps,
                                                          const int4* __restrict__ work,
                                                          const double* __restrict__ params,
                                                          double* __restrict__ x, double* __restrict__ p,
                                                          double* __restrict__ veta, long long G, int M) {
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  if ((int)threadIdx.x >= wk.y) return;
  const long long gi = int_work_first(wk) + threadIdx.x;
  const long long li = gi - R.dof;   // index within the replica (the generator's counter)
  const double sigma = params[2LL * wk.x];
  const unsigned long long seed = (unsigned long long)__double_as_longlong(params[2LL * wk.x + 1]);
  x[gi] = sigma * gaussian(seed, 0u, (unsigned long long)li);
  p[gi] = sqrt(R.mp / R.beta) * gaussian(seed, 1u, (unsigned long long)li);
  for (int k = 0; k < M; ++k) veta[k * G + gi] = 0.0;
}

hipError_t launch_init_state(const Dims& d, const DevPtrs& w, const double* params, hipStream_t s) {
  if (d.nintwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)d.nintwg), dim3(kIntBlock), 0, s, w.reps, w.intwork, params, w.x,
                     w.p, w.veta, d.G, d.M);
  return hipGetLastError();
}

}  // namespace pimd
