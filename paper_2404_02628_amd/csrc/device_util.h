// device_util.h -- small device helpers shared by the libpimd kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace pimd {

// Index of this wavefront in its workgroup, in a scalar register: the compiler cannot tell
// that threadIdx.x >> 6 is the same in every lane, and branches, loop bounds and addresses
// derived from it would otherwise run on the vector ALU under exec masks.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Sum over the 64 lanes of a wavefront, identical result in every lane.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Workgroup sum of K values per thread in a fixed order (waves summed in index
// order), result valid in thread 0.  `lds` needs K * (blockDim.x / 64) doubles.
template <int K>
__device__ inline void block_sum(double (&v)[K], double* lds) {
  const int lane = threadIdx.x & 63, wave = wave_id(), nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * nw + wave] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[k * nw + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Broadcast lane `src` of a double to the whole wavefront (src uniform).
__device__ inline double read_lane(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// v of lane (lane & ~3) + K, i.e. lane K of each aligned group of four (DPP quad permutation).
template <int K>
__device__ inline double quad_lane(double v) {
  constexpr int kCtrl = K | (K << 2) | (K << 4) | (K << 6);
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Work item of workgroup b in a launch of n workgroups.  Workgroups are dealt round-robin over
// the kXcds accelerator dies (b runs on die b mod kXcds, each die with its own L2); this gives
// each die one contiguous range of work items, so items listed next to each other (the tiles of
// one slice) read their shared inputs through one L2.
constexpr int kXcds = 8;
__device__ inline int xcd_work_index(int b, int n) {
  const int x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + min(x, r) + k;
}

// log of xi^k with 0^0 = 1; lnxi = log(xi) (-inf for xi = 0), k >= 0.
__device__ inline double xi_pow_log(int k, double lnxi) { return k == 0 ? 0.0 : (double)k * lnxi; }

}  // namespace pimd
