// k_pair.hip -- all-pairs Gaussian interaction of every imaginary-time slice.
//
// U = sum_j V(slice j) (Eq. 5) with V = sum_{l<l'} A exp(-|r_l - r_l'|^2 / s^2) (Eq. 20, each
// unordered pair once).  The sampled weight carries U/P (Eq. 4), so the force on bead (l, j) is
//   F = (2A / (P s^2)) sum_{l'} exp(-|r_l - r_l'|^2/s^2) (r_l - r_l').
// Each lane owns one particle i of one slice and sweeps the partner index j, which is the
// same for the whole wavefront, so partner coordinates are wave-uniform loads.  Ordered pairs
// are evaluated (i sees every j), which needs no write conflicts; the i = j term contributes
// zero force and is masked out of the energies.
//
// Mixed precision: coordinates come from the FP32 shadow, pre-scaled by sqrt(log2 e)/s, so a
// term is exp2(-|dr|^2) (one v_exp_f32); FP32 sums run over runs of kFold partners and are then
// folded into FP64 accumulators.  FP64 mode reads the FP64 positions and uses the branch-free table
// exponential of fast_exp.h (at most 2 ulp).
//
// Estimator sums (only when requested): sum over ordered pairs of u and of u |dr|^2, giving
// U_pair and the pair part of the virial W = sum_pairs u (1 - r^2/s^2).
#include "pimd_internal.h"
#include "device_util.h"
#include "fast_exp.h"

namespace pimd {

constexpr int kFold = 128;

template <int D>
struct Vec { float v[D == 3 ? 4 : D]; };

// JS waves share one 64-particle tile, each sweeping 1/JS of the partners.
template <int D, bool EST, int JS>
__global__ __launch_bounds__(256) void k_pair_f32(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                                  const float* __restrict__ xs, double* __restrict__ fpair,
                                                  double* __restrict__ pairpart, int P) {
  constexpr int DP = D == 3 ? 4 : D;
  constexpr int IT = 4 / JS;          // 64-particle tiles per workgroup
  __shared__ double red[4][D + 2][64];
  const int g = xcd_work_index((int)blockIdx.x, (int)gridDim.x);
  const int4 wk = work[g];
  const RepDev& R = reps[wk.x];
  const int N = R.n, slice = wk.y;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int itile = wave / JS, jpart = wave % JS;
  const int i = wk.z + itile * 64 + lane;
  const float* xsl = xs + R.shadow + (long long)slice * R.npad * DP;
  float xi[D];
  const int ii = i < N ? i : N - 1;
#pragma unroll
  for (int a = 0; a < D; ++a) xi[a] = xsl[(long long)ii * DP + a];
  const int jchunk = (N + JS - 1) / JS;
  const int j0 = jpart * jchunk;
  const int j1 = min(N, j0 + jchunk);
  double F[D], U = 0.0, W = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) F[a] = 0.0;
  for (int jb = j0; jb < j1; jb += kFold) {
    const int je = min(j1, jb + kFold);
    float f[D], u32 = 0.f, w32 = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) f[a] = 0.f;
#pragma unroll 4
    for (int j = jb; j < je; ++j) {
      float d[D], r2 = 0.f;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        d[a] = xi[a] - xsl[(long long)j * DP + a];
        r2 = __builtin_fmaf(d[a], d[a], r2);
      }
      float u = __builtin_amdgcn_exp2f(-r2);
#pragma unroll
      for (int a = 0; a < D; ++a) f[a] = __builtin_fmaf(u, d[a], f[a]);
      if (EST) {
        float um = (j == i) ? 0.f : u;
        u32 += um;
        w32 = __builtin_fmaf(um, r2, w32);
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] += (double)f[a];
    if (EST) { U += (double)u32; W += (double)w32; }
  }
  if (i >= N) { U = 0.0; W = 0.0; }
  if (JS > 1) {
#pragma unroll
    for (int a = 0; a < D; ++a) red[wave][a][lane] = F[a];
    __syncthreads();
    if (jpart == 0) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s = 0.0;
        for (int q = 0; q < JS; ++q) s += red[wave + q][a][lane];
        F[a] = s;
      }
    }
    __syncthreads();
  }
  if (jpart == 0 && i < N) {
    // F = (2A/(P s^2 k)) * sum u (r'_i - r'_j) with r' = k r, k = sqrt(log2 e)/s
    const double k = sqrt(1.4426950408889634) / R.width;
    const double scale = 2.0 * R.amp / ((double)P * R.width * R.width * k);
    double* fr = fpair + R.dof;
#pragma unroll
    for (int a = 0; a < D; ++a) fr[((long long)a * P + slice) * N + i] = scale * F[a];
  }
  if (EST) {
    double v[2] = {U, W};
    block_sum<2>(v, &red[0][0][0]);
    if (threadIdx.x == 0) {
      // u r'^2 = u r^2 log2(e)/s^2  ->  r^2/s^2 = r'^2 / log2(e)
      pairpart[2LL * g + 0] = 0.5 * R.amp * v[0];
      pairpart[2LL * g + 1] = 0.5 * R.amp * (v[0] - v[1] / 1.4426950408889634);
    }
  }
}

template <int D, bool EST, int JS>
__global__ __launch_bounds__(256) void k_pair_f64(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                                  const double* __restrict__ x, double* __restrict__ fpair,
                                                  double* __restrict__ pairpart, int P) {
  constexpr int IT = 4 / JS;
  __shared__ double red[4][D + 2][64];
  __shared__ double tab[kExpTable];   // table of the branch-free exponential (2 ulp)
  fill_exp_table(tab);
  __syncthreads();
  const int g = xcd_work_index((int)blockIdx.x, (int)gridDim.x);
  const int4 wk = work[g];
  const RepDev& R = reps[wk.x];
  const int N = R.n, slice = wk.y;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int itile = wave / JS, jpart = wave % JS;
  const int i = wk.z + itile * 64 + lane;
  const double inv_s = 1.0 / R.width;
  const double* xr = x + R.dof;
  double xi[D];
  const int ii = i < N ? i : N - 1;
#pragma unroll
  for (int a = 0; a < D; ++a) xi[a] = xr[((long long)a * P + slice) * N + ii] * inv_s;
  const int jchunk = (N + JS - 1) / JS;
  const int j0 = jpart * jchunk;
  const int j1 = min(N, j0 + jchunk);
  double F[D], U = 0.0, W = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) F[a] = 0.0;
#pragma unroll 2
  for (int j = j0; j < j1; ++j) {
    double d[D], r2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      d[a] = xi[a] - xr[((long long)a * P + slice) * N + j] * inv_s;
      r2 = fma(d[a], d[a], r2);
    }
    double u = fast_exp(-r2, tab);
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = fma(u, d[a], F[a]);
    if (EST) {
      double um = (j == i) ? 0.0 : u;
      U += um;
      W = fma(um, r2, W);
    }
  }
  if (i >= N) { U = 0.0; W = 0.0; }
  if (JS > 1) {
#pragma unroll
    for (int a = 0; a < D; ++a) red[wave][a][lane] = F[a];
    __syncthreads();
    if (jpart == 0) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s = 0.0;
        for (int q = 0; q < JS; ++q) s += red[wave + q][a][lane];
        F[a] = s;
      }
    }
    __syncthreads();
  }
  if (jpart == 0 && i < N) {
    // F = (2A/(P s^2)) sum u (r_i - r_j) = (2A/(P s)) sum u (r'_i - r'_j), r' = r/s
    const double scale = 2.0 * R.amp / ((double)P * R.width);
    double* fr = fpair + R.dof;
#pragma unroll
    for (int a = 0; a < D; ++a) fr[((long long)a * P + slice) * N + i] = scale * F[a];
  }
  if (EST) {
    double v[2] = {U, W};
    block_sum<2>(v, &red[0][0][0]);
    if (threadIdx.x == 0) {
      pairpart[2LL * g + 0] = 0.5 * R.amp * v[0];
      pairpart[2LL * g + 1] = 0.5 * R.amp * (v[0] - v[1]);
    }
  }
}

template <int D, bool EST>
static void launch_pair_js(const Dims& d, const DevPtrs& w, int js, hipStream_t s) {
  dim3 grid((unsigned)d.npairwork), block(256);
  if (d.precision == 1) {
    if (js == 4) hipLaunchKernelGGL((k_pair_f32<D, EST, 4>), grid, block, 0, s, w.reps, w.pairwork, w.xs, w.fpair, w.pairpart, d.P);
    else if (js == 2) hipLaunchKernelGGL((k_pair_f32<D, EST, 2>), grid, block, 0, s, w.reps, w.pairwork, w.xs, w.fpair, w.pairpart, d.P);
    else hipLaunchKernelGGL((k_pair_f32<D, EST, 1>), grid, block, 0, s, w.reps, w.pairwork, w.xs, w.fpair, w.pairpart, d.P);
  } else {
    if (js == 4) hipLaunchKernelGGL((k_pair_f64<D, EST, 4>), grid, block, 0, s, w.reps, w.pairwork, w.x, w.fpair, w.pairpart, d.P);
    else if (js == 2) hipLaunchKernelGGL((k_pair_f64<D, EST, 2>), grid, block, 0, s, w.reps, w.pairwork, w.x, w.fpair, w.pairpart, d.P);
    else hipLaunchKernelGGL((k_pair_f64<D, EST, 1>), grid, block, 0, s, w.reps, w.pairwork, w.x, w.fpair, w.pairpart, d.P);
  }
}

// ------------------------------------------------------------------ symmetric variant
//
// One workgroup per slice evaluates every unordered pair once.  The slice is cut into tiles of
// 64 particles; a wave takes a pair of tiles (I, J) and covers its 64 x 64 pairs as an 8 x 8
// block per step: lane l pairs particle I[l%8 + 8a] with J[l/8 + 8b] for a, b = 0..7, so the
// eight i-positions and eight j-positions of a lane stay in registers and each term feeds both
// sides: F_i += u d and F_j -= u d (Newton's third law per slice), with per-lane accumulators
// indexed by a and by b.  After the tile pair, a transpose through LDS sums the eight lanes
// that share a particle (reduce-scatter: lane L = c0 + 8 k0 ends with the total of particle L of
// tile I and of particle k0 + 8 c0 of tile J, which keeps the J side's reads on distinct banks),
// and the totals are added to the slice's forces in LDS.  Tile pairs are scheduled as a
// round-robin tournament (circle method): within a round no two tile pairs share a tile, so
// the LDS force updates need no atomics and their order is fixed (results are reproducible).
// The diagonal tiles (I, I) run first with the pairs j <= i masked out.  Padding particles sit
// at distinct far-away positions, so their terms underflow to exactly zero.
//
// Two precisions share this schedule.  Mixed (T = float): the FP32 shadow, pre-scaled so that a
// term is exp2(-|dr|^2) (one v_exp_f32), tile sums and the slice's force accumulators in FP32
// (a particle's force adds one partial per tile, so at N = 1600 a sum of 25 partials: rounding
// of order 1e-7 of the force, against the mixed mode's 1e-5 bar).  FP32 accumulators halve that
// part of the LDS (3.4% less pair time in the step at 128 replicas of N = 1600 than with FP64
// accumulators).  FP64 (T = double): the positions scaled by 1/s, a term is exp(-|dr|^2) by the
// table exponential (its table in LDS), everything in FP64.
//
// Waves per workgroup (kWaves): wave w runs on SIMD w mod 4, and the waves of one SIMD together
// take the tile pairs k = w (mod 4) of every round, so eight waves split a round's work over the
// SIMDs exactly as four do, with two waves per SIMD to cover each other's latencies.  Mixed
// precision uses eight (44.2 KB of LDS per workgroup at N = 1600: three per compute unit, two
// beside a batched recursion workgroup; 2.8% less pair time in the step than four waves); FP64
// keeps four, since its transpose buffer is twice as large and eight waves would halve the
// workgroups per compute unit and the largest slice it serves.  Six waves would load two SIMDs
// twice as much as the other two.
constexpr int kRedStride = 9;   // LDS row stride of the per-wave transpose (conflict-free reads)

template <class T> struct SymPrec;
template <> struct SymPrec<float> {
  template <int D> static constexpr int dp() { return D == 3 ? 4 : D; }   // shadow row (float4 in 3-D)
  static constexpr int kWaves = 8;
  static constexpr int kTab = 0;
  static __device__ inline float term(float r2, const double*) { return __builtin_amdgcn_exp2f(-r2); }
};
template <> struct SymPrec<double> {
  template <int D> static constexpr int dp() { return D; }
  static constexpr int kWaves = 4;
  static constexpr int kTab = kExpTable;
  static __device__ inline double term(double r2, const double* tab) { return fast_exp_finite(-r2, tab); }
};

template <class T, int D>
__host__ __device__ inline int sym_lds_bytes(int npad) {
  constexpr int DP = SymPrec<T>::template dp<D>();
  constexpr int W = SymPrec<T>::kWaves;
  return npad * (DP + D) * (int)sizeof(T) + W * 64 * kRedStride * (int)sizeof(T) + 2 * W * 8 + SymPrec<T>::kTab * 8;
}

template <class T, int D, bool EST, bool DIAG>
__device__ inline void sym_tile_pair(const T* __restrict__ pos, T* __restrict__ Fs, T* __restrict__ red,
                                     const double* __restrict__ tab, int npad, int I, int J, double& Ud, double& Wd) {
  constexpr int DP = SymPrec<T>::template dp<D>();
  const int lane = threadIdx.x & 63;
  const int c0 = lane & 7, k0 = lane >> 3;
  T xi[8][D], xj[8][D], Fi[8][D], Fj[8][D];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      xi[a][c] = pos[(I * 64 + c0 + 8 * a) * DP + c];
      xj[a][c] = pos[(J * 64 + k0 + 8 * a) * DP + c];
      Fi[a][c] = T(0);
      Fj[a][c] = T(0);
    }
  }
  T U = T(0), W = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      T d[D], r2 = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        d[c] = xi[a][c] - xj[b][c];
        r2 = fma(d[c], d[c], r2);
      }
      T u = SymPrec<T>::term(r2, tab);
      if (DIAG) u = (k0 + 8 * b > c0 + 8 * a) ? u : T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        Fi[a][c] = fma(u, d[c], Fi[a][c]);
        Fj[b][c] = fma(-u, d[c], Fj[b][c]);
      }
      if (EST) {
        U += u;
        W = fma(u, r2, W);
      }
    }
  }
  if (EST) { Ud += (double)U; Wd += (double)W; }
  // reduce-scatter through LDS: lane L receives the sums for particle L of tile I, then of J
#pragma unroll
  for (int c = 0; c < D; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) red[lane * kRedStride + a] = Fi[a][c];
    // (the sums start from their first element: 0 + x is not folded for floating point)
    T si = red[c0 * kRedStride + k0];
#pragma unroll
    for (int k = 1; k < 8; ++k) si += red[(c0 + 8 * k) * kRedStride + k0];
#pragma unroll
    for (int b = 0; b < 8; ++b) red[lane * kRedStride + b] = Fj[b][c];
    // lane (c0, k0) sums particle k0 + 8 c0 of tile J over the eight lanes that share k0 (rows
    // q + 8 k0, column c0: distinct banks across each half wave)
    T sj = red[8 * k0 * kRedStride + c0];
#pragma unroll
    for (int q = 1; q < 8; ++q) sj += red[(q + 8 * k0) * kRedStride + c0];
    Fs[c * npad + I * 64 + lane] += si;
    Fs[c * npad + J * 64 + k0 + 8 * c0] += sj;
  }
}

// Slice positions into LDS: the mixed shadow as stored, or the FP64 positions scaled by 1/s.
template <class T, int D>
__device__ inline void sym_load_slice(T* __restrict__ pos, const RepDev& R, const float* __restrict__ xs,
                                      const double* __restrict__ x, int slice, int P) {
  constexpr int DP = SymPrec<T>::template dp<D>();
  const int N = R.n, npad = R.npad;
  if constexpr (sizeof(T) == 4) {
    const float* xsl = xs + R.shadow + (long long)slice * npad * DP;
    for (int l = threadIdx.x; l < npad; l += blockDim.x) {
#pragma unroll
      for (int c = 0; c < DP; ++c) pos[l * DP + c] = l < N ? xsl[(long long)l * DP + c] : 1.0e4f * (float)(l + 1);
    }
  } else {
    const double inv_s = 1.0 / R.width;
    const double* xr = x + R.dof;
    for (int l = threadIdx.x; l < npad; l += blockDim.x) {
#pragma unroll
      for (int c = 0; c < D; ++c)
        pos[l * DP + c] = l < N ? xr[((long long)c * P + slice) * N + l] * inv_s : 1.0e4 * (double)(l + 1);
    }
  }
}

template <class T, int D, bool EST>
__device__ inline void pair_sym_body(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                     const float* __restrict__ xs, const double* __restrict__ x,
                                     double* __restrict__ fpair, double* __restrict__ pairpart, int P,
                                     unsigned char* lds) {
  constexpr int DP = SymPrec<T>::template dp<D>();
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  const int N = R.n, slice = wk.y, npad = R.npad;
  // with the wave index in a scalar register the tournament's tile arithmetic (two modulos per
  // tile pair) runs on the scalar unit
  const int lane = threadIdx.x & 63, wave = wave_id();
  T* Fs = reinterpret_cast<T*>(lds);                                   // [D][npad]
  double* tab = reinterpret_cast<double*>(Fs + (long long)D * npad);  // [kTab] (FP64 only)
  T* pos = reinterpret_cast<T*>(tab + SymPrec<T>::kTab);           // [npad][DP]
  T* red = pos + (long long)npad * DP + wave * 64 * kRedStride;
  constexpr int W = SymPrec<T>::kWaves;
  double* part = reinterpret_cast<double*>(pos + (long long)npad * DP + W * 64 * kRedStride);   // [W][2]
  if constexpr (SymPrec<T>::kTab > 0) fill_exp_table(tab);
  sym_load_slice<T, D>(pos, R, xs, x, slice, P);
  for (int l = threadIdx.x; l < npad; l += blockDim.x) {
#pragma unroll
    for (int c = 0; c < D; ++c) Fs[c * npad + l] = T(0);
  }
  __syncthreads();
  const int T_ = npad / 64;
  double Ud = 0.0, Wd = 0.0;
  for (int t = wave; t < T_; t += W) sym_tile_pair<T, D, EST, true>(pos, Fs, red, tab, npad, t, t, Ud, Wd);
  __syncthreads();
  if (T_ > 1) {
    const int Tp = T_ + (T_ & 1), m = Tp - 1;
    for (int r = 0; r < m; ++r) {
      for (int k = wave; k < Tp / 2; k += W) {
        const int p = k == 0 ? r : (r + k) % m;
        const int q = k == 0 ? m : (r - k + m) % m;
        if (p < T_ && q < T_) sym_tile_pair<T, D, EST, false>(pos, Fs, red, tab, npad, min(p, q), max(p, q), Ud, Wd);
      }
      __syncthreads();
    }
  }
  // mixed: F = (2A/(P s^2 k)) sum u (r'_i - r'_j) with r' = k r, k = sqrt(log2 e)/s;
  // FP64:  F = (2A/(P s)) sum u (r'_i - r'_j) with r' = r/s
  const double kk = sizeof(T) == 4 ? sqrt(1.4426950408889634) / R.width : 1.0 / R.width;
  const double scale = 2.0 * R.amp / ((double)P * R.width * R.width * kk);
  double* fr = fpair + R.dof;
  for (int l = threadIdx.x; l < N; l += blockDim.x) {
#pragma unroll
    for (int c = 0; c < D; ++c) fr[((long long)c * P + slice) * N + l] = scale * (double)Fs[c * npad + l];
  }
  if (EST) {
    // unordered pairs: U_slice = A sum u, virial part A sum u (1 - r^2/s^2)
    // (mixed: r'^2 = r^2 log2(e)/s^2, so r^2/s^2 = r'^2 / log2(e))
    Ud = wave_sum(Ud);
    Wd = wave_sum(Wd);
    if (lane == 0) { part[2 * wave] = Ud; part[2 * wave + 1] = Wd; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double u = 0.0, w = 0.0;
      for (int q = 0; q < W; ++q) { u += part[2 * q]; w += part[2 * q + 1]; }
      const double wscale = sizeof(T) == 4 ? 1.0 / 1.4426950408889634 : 1.0;
      pairpart[2LL * blockIdx.x + 0] = R.amp * u;
      pairpart[2LL * blockIdx.x + 1] = R.amp * (u - w * wscale);
    }
  }
}

template <int D, bool EST>
__global__ __launch_bounds__(SymPrec<float>::kWaves * 64) void k_pair_sym_f32(const RepDev* __restrict__ reps,
                                                                 const int4* __restrict__ work,
                                                                 const float* __restrict__ xs,
                                                                 double* __restrict__ fpair,
                                                                 double* __restrict__ pairpart, int P) {
  extern __shared__ __align__(16) unsigned char sym_lds[];
  pair_sym_body<float, D, EST>(reps, work, xs, nullptr, fpair, pairpart, P, sym_lds);
}

template <int D, bool EST>
__global__ __launch_bounds__(SymPrec<double>::kWaves * 64) void k_pair_sym_f64(const RepDev* __restrict__ reps,
                                                                 const int4* __restrict__ work,
                                                                 const double* __restrict__ x,
                                                                 double* __restrict__ fpair,
                                                                 double* __restrict__ pairpart, int P) {
  extern __shared__ __align__(16) unsigned char sym_lds[];
  pair_sym_body<double, D, EST>(reps, work, nullptr, x, fpair, pairpart, P, sym_lds);
}

template <int D, bool EST>
static void launch_pair_sym(const Dims& d, const DevPtrs& w, hipStream_t s) {
  const int npad = (d.pair_maxn + 63) / 64 * 64;
  dim3 grid((unsigned)d.npairwork);
  if (d.precision == 1)
    hipLaunchKernelGGL((k_pair_sym_f32<D, EST>), grid, dim3(SymPrec<float>::kWaves * 64), (sym_lds_bytes<float, D>(npad)), s, w.reps, w.pairwork,
                       w.xs, w.fpair, w.pairpart, d.P);
  else
    hipLaunchKernelGGL((k_pair_sym_f64<D, EST>), grid, dim3(SymPrec<double>::kWaves * 64), (sym_lds_bytes<double, D>(npad)), s, w.reps, w.pairwork,
                       w.x, w.fpair, w.pairpart, d.P);
}

int pair_sym_lds_bytes(int D, int maxn, int precision) {
  const int npad = (maxn + 63) / 64 * 64;
  if (precision == 1)
    return D == 1 ? sym_lds_bytes<float, 1>(npad) : (D == 2 ? sym_lds_bytes<float, 2>(npad) : sym_lds_bytes<float, 3>(npad));
  return D == 1 ? sym_lds_bytes<double, 1>(npad) : (D == 2 ? sym_lds_bytes<double, 2>(npad) : sym_lds_bytes<double, 3>(npad));
}

// jsplit: waves per 64-particle tile (1, 2 or 4) of the ordered kernels, or 0 for the symmetric
// per-slice kernel; the work list was built for this value.
hipError_t launch_pair(const Dims& d, const DevPtrs& w, bool est, int jsplit, hipStream_t s) {
  if (d.npairwork == 0) return hipSuccess;
  if (jsplit == 0) {
    switch (d.D) {
      case 1: est ? launch_pair_sym<1, true>(d, w, s) : launch_pair_sym<1, false>(d, w, s); break;
      case 2: est ? launch_pair_sym<2, true>(d, w, s) : launch_pair_sym<2, false>(d, w, s); break;
      case 3: est ? launch_pair_sym<3, true>(d, w, s) : launch_pair_sym<3, false>(d, w, s); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (d.D) {
    case 1: est ? launch_pair_js<1, true>(d, w, jsplit, s) : launch_pair_js<1, false>(d, w, jsplit, s); break;
    case 2: est ? launch_pair_js<2, true>(d, w, jsplit, s) : launch_pair_js<2, false>(d, w, jsplit, s); break;
    case 3: est ? launch_pair_js<3, true>(d, w, jsplit, s) : launch_pair_js<3, false>(d, w, jsplit, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pimd
