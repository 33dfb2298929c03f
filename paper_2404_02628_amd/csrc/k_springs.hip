// k_springs.hip -- ring-polymer springs and the harmonic trap (HBM-bound).
//
// For every particle l of every replica, one pass over its P beads:
//   * interior spring forces  -m omega_P^2 (2 r^j - r^{j+1} - r^{j-1}),  j = 2..P-1   (Eq. 17)
//   * trap forces             -(1/P) m omega^2 r^j on every bead                      (Eqs. 4, 19)
//   * E_int^{(l)} = (1/2) m omega_P^2 sum_{j<P} |r^{j+1} - r^j|^2                       (Eq. 9)
//   * link_l = (1/2) m omega_P^2 |r_l^P - r_{l+1}^1|^2 (the inter-ring term of Eq. 7), 0 for l = N
//     and for the last particle of the first species (no allowed cycle contains that link)
//   * the end beads r_l^1, r_l^P used by the exchange recursion (Eqs. 6-16)
//   * in mixed precision, the FP32 shadow of the positions for the pair kernel, stored
//     slice-major [P][N][dp] and pre-scaled by sqrt(log2 e)/s so the pair kernel evaluates
//     exp(-|r|^2/s^2) as one exp2.
// End-bead exchange forces (Eqs. 15-16) are added later by the probability reduction.
// Per-workgroup partial sums (E_int, links, trap energy) go to springpart in a fixed order.
// Workgroup 0 also advances the launch stamp that the cooperative exchange recursion of the
// same evaluation uses to mark its progress flags (a device counter, so that a replayed graph
// of the step gets a new stamp each time).
#include "pimd_internal.h"
#include "device_util.h"

namespace pimd {

constexpr int kBeadChunk = 8;   // beads loaded together per particle

template <int D, bool SHADOW>
__global__ __launch_bounds__(kSpringBlock) void k_springs(const RepDev* __restrict__ reps,
                                                          const int4* __restrict__ work,
                                                          const double* __restrict__ x, double* __restrict__ f,
                                                          double* __restrict__ ends, double* __restrict__ link,
                                                          double* __restrict__ eint, float* __restrict__ xs,
                                                          double* __restrict__ springpart, int* __restrict__ epoch,
                                                          int P) {
  __shared__ double lds[3 * (kSpringBlock / 64)];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int e = *epoch;
    *epoch = (e <= 0 || e >= 0x7ffffffe) ? 1 : e + 1;
  }
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  const int N = R.n;
  const int l = wk.y + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};  // E_int, link, U_trap
  if (l < N) {
    const double* xr = x + R.dof;
    double* fr = f + R.dof;
    const double kap = R.kappa, trap = R.trap_p;
    double e_int = 0.0, lk = 0.0, ut = 0.0;
    double* a_out = ends + 2LL * D * R.part;
    double* b_out = a_out + (long long)D * R.npp;
    const float kscale = R.pair_k;
    const int dp = shadow_dp(D);
    float* xsr = xs + R.shadow;
    const long long PN = (long long)P * N;
    // the shadow row of bead j holds all components of particle l: one vector store per bead
    auto shadow = [&](int j, const double (&r)[D]) {
      float* o = xsr + ((long long)j * R.npad + l) * dp;
      if (D == 1) {
        o[0] = (float)r[0] * kscale;
      } else if (D == 2) {
        *reinterpret_cast<float2*>(o) = make_float2((float)r[0] * kscale, (float)r[D > 1 ? 1 : 0] * kscale);
      } else {
        *reinterpret_cast<float4*>(o) = make_float4((float)r[0] * kscale, (float)r[D > 1 ? 1 : 0] * kscale,
                                                    (float)r[D > 2 ? 2 : 0] * kscale, 0.f);
      }
    };
    // beads 1 and 2 (P >= 2), every component
    double rm[D], rc[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      rm[a] = xr[a * PN + l];
      rc[a] = xr[a * PN + N + l];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double r0 = rm[a];
      a_out[(long long)a * R.npp + l] = r0;
      fr[a * PN + l] = -trap * r0;
      ut += r0 * r0;
      const double d = rc[a] - r0;
      e_int += d * d;
    }
    if (SHADOW) shadow(0, rm);
    // interior beads in chunks: the loads of a chunk (all components) are issued together, so
    // each chunk waits out one memory latency (the sums keep their bead order per component)
    for (int j0 = 1; j0 < P - 1; j0 += kBeadChunk) {
      double nx[kBeadChunk][D];
#pragma unroll
      for (int u = 0; u < kBeadChunk; ++u) {
        const long long jn = (long long)min(j0 + u + 1, P - 1) * N + l;
#pragma unroll
        for (int a = 0; a < D; ++a) nx[u][a] = xr[a * PN + jn];
      }
#pragma unroll
      for (int u = 0; u < kBeadChunk; ++u) {
        const int j = j0 + u;
        if (j < P - 1) {
          if (SHADOW) shadow(j, rc);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const double rn = nx[u][a];
            fr[a * PN + (long long)j * N + l] = -kap * (2.0 * rc[a] - rn - rm[a]) - trap * rc[a];
            ut += rc[a] * rc[a];
            const double dd = rn - rc[a];
            e_int += dd * dd;
            rm[a] = rc[a];
            rc[a] = rn;
          }
        }
      }
    }
    // rc is bead P
    if (SHADOW) shadow(P - 1, rc);
    const bool has_link = l + 1 < N && l + 1 != R.na;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      fr[a * PN + (long long)(P - 1) * N + l] = -trap * rc[a];
      ut += rc[a] * rc[a];
      b_out[(long long)a * R.npp + l] = rc[a];
      if (has_link) {
        const double dl = rc[a] - xr[a * PN + l + 1];
        lk += dl * dl;
      }
    }
    e_int *= R.c;
    lk *= R.c;
    ut *= 0.5 * R.mw2;
    eint[R.part + l] = e_int;
    link[R.part + l] = lk;   // zero for the last particle of each species
    acc[0] = e_int; acc[1] = lk; acc[2] = ut;
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    double* sp = springpart + 4LL * blockIdx.x;
    sp[0] = acc[0]; sp[1] = acc[1]; sp[2] = acc[2]; sp[3] = 0.0;
  }
}

hipError_t launch_springs(const Dims& d, const DevPtrs& w, hipStream_t s) {
  if (d.nspringwg == 0) return hipSuccess;
  dim3 grid((unsigned)d.nspringwg), block(kSpringBlock);
  const bool sh = d.precision == 1;
#define L(DD, SH) hipLaunchKernelGGL((k_springs<DD, SH>), grid, block, 0, s, w.reps, w.springwork, w.x, w.f, \
                                     w.ends, w.link, w.eint, w.xs, w.springpart, w.err + 1, d.P)
  switch (d.D * 2 + (sh ? 1 : 0)) {
    case 2: L(1, false); break;
    case 3: L(1, true); break;
    case 4: L(2, false); break;
    case 5: L(2, true); break;
    case 6: L(3, false); break;
    case 7: L(3, true); break;
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

}  // namespace pimd
