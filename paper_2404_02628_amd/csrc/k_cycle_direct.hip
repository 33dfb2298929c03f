// k_cycle_direct.hip -- the cycle energies E^{[u,v]} by their definition, entry by entry.
//
// E^{[u,v]} (Eq. 7) is the spring energy of the single ring that particles u..v form when each
// one's last bead joins the next one's first bead and v's last bead closes back onto u's first:
//   E^{[u,v]} = (1/2) m omega_P^2 [ sum_{l=u}^{v} sum_{j=1}^{P-1} |r_l^{j+1} - r_l^j|^2
//                                 + sum_{l=u}^{v-1} |r_{l+1}^1 - r_l^P|^2 + |r_u^1 - r_v^P|^2 ].
// Evaluated independently for every entry this costs O((v-u+1) P d) per entry and O(N^3 P) for
// the table (Sec. III): the original algorithm that the quadratic scheme replaces.  The exchange
// path never forms this table (its recursions regroup E into per-particle terms); this kernel
// exists as an independent cross-check of those terms and as a cost reference.
//
// Mapping: one wavefront per (row u, 64 consecutive columns v), one entry per lane.  The wave
// walks the particles l = u, u+1, ... in chunks of 64: lane k loads the beads of particle c0+k
// (coalesced) and forms that particle's ring term sum_j |r^{j+1} - r^j|^2 and its outgoing link;
// then every lane adds, in order of l, the terms of the particles its own ring contains
// (l <= v, links for l < v), reading them from the loading lanes.  Each entry is still its own
// sum over its (v-u+1) particles; only the per-particle bead sums are shared by the 64 entries
// of a wave, which cuts the serial load latency of one lane walking all beads by itself.
// Waves whose columns all lie left of the diagonal write zeros.
#include "pimd_internal.h"
#include "device_util.h"

namespace pimd {

constexpr int kDirectWaves = 4;

template <int D>
__global__ __launch_bounds__(64 * kDirectWaves) void k_cycle_direct(const RepDev* __restrict__ reps, int r,
                                                                    const double* __restrict__ x, int P, int row0,
                                                                    int nrows, double* __restrict__ out) {
  const RepDev& R = reps[r];
  const int N = R.n;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nvb = (N + kTile - 1) / kTile;
  const long long item = (long long)blockIdx.x * kDirectWaves + wave;
  if (item >= (long long)nrows * nvb) return;
  const int ul = (int)(item / nvb), vb = (int)(item % nvb);
  const int u = row0 + ul;           // 0-based first particle of the ring
  const int v = vb * kTile + lane;   // 0-based last particle of the ring (this lane's entry)
  double* row = out + (long long)ul * N;
  if (vb * kTile + kTile - 1 < u) {  // the whole wave is left of the diagonal
    if (v < N) row[v] = 0.0;
    return;
  }
  const double* xr = x + R.dof;
  const long long PN = (long long)P * N;
  const int vend = min(N - 1, vb * kTile + kTile - 1);
  double acc = 0.0;
  for (int c0 = u; c0 <= vend; c0 += kTile) {
    const int l = c0 + lane;   // particle whose terms this lane forms
    double e = 0.0, lk = 0.0;
    if (l <= vend) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double* xa = xr + a * PN + l;
        double prev = xa[0];
#pragma unroll 8
        for (int j = 1; j < P; ++j) {
          const double cur = xa[(long long)j * N];
          const double d = cur - prev;
          e = fma(d, d, e);
          prev = cur;
        }
        if (l + 1 < N) {
          const double d = xa[1] - prev;   // r_{l+1}^1 - r_l^P
          lk = fma(d, d, lk);
        }
      }
    }
    const int cnt = min(kTile, vend - c0 + 1);
    for (int k = 0; k < cnt; ++k) {
      const double ek = read_lane(e, k), lkk = read_lane(lk, k);
      if (c0 + k <= v) acc += ek;
      if (c0 + k < v) acc += lkk;
    }
  }
  double cl = 0.0;
  if (v < N) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double d = xr[a * PN + u] - xr[a * PN + (long long)(P - 1) * N + v];
      cl = fma(d, d, cl);
    }
  }
  if (v < N) row[v] = (v >= u) ? R.c * (acc + cl) : 0.0;
}

hipError_t launch_cycle_direct(const Dims& d, const DevPtrs& w, int r, int n, int row0, int nrows, double* out,
                               hipStream_t s) {
  const long long items = (long long)nrows * ((n + kTile - 1) / kTile);
  if (items == 0) return hipSuccess;
  dim3 grid((unsigned)((items + kDirectWaves - 1) / kDirectWaves)), block(64 * kDirectWaves);
#define L(DD) hipLaunchKernelGGL(k_cycle_direct<DD>, grid, block, 0, s, w.reps, r, w.x, d.P, row0, nrows, out)
  switch (d.D) {
    case 1: L(1); break;
    case 2: L(2); break;
    case 3: L(3); break;
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

}  // namespace pimd
