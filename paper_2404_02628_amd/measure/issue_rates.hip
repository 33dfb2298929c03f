// issue_rates.hip -- measures the issue cost of the instructions that bound the pair kernel.
//
// A standalone program (`python -m paper_2404_02628_amd.build --issue-rates`), not part of libpimd.  Each
// kernel fills the GPU (2048 workgroups of 256 threads, 8 waves per SIMD) with a loop of one
// instruction kind carried by independent dependency chains, so that throughput, not latency,
// sets its time; the time is converted to cycles per wave instruction and SIMD at the 2.4 GHz
// peak engine clock (1024 SIMDs).  The kinds:
//   fma      v_fma_f32 (compiled with packed FP32 disabled, as the library is)
//   exp      v_exp_f32 (exp2), the pair term's one transcendental
//   mfma16   v_mfma_f32_16x16x4_f32 (1024 multiply-adds)
//   mfma4    v_mfma_f32_4x4x1_16b_f32 (16 blocks, 256 multiply-adds)
//   mix      four mfma4 and eight exp per iteration, independent of each other: if the matrix
//            unit and the transcendental unit overlapped, this would cost max(), not the sum
//   pair     the pair kernel's inner step for d = 2 (two differences, |d|^2 by one multiply and
//            one FMA, one exp2, four FMAs for the forces on both particles), per pair
//   copy, copy4, triad   FP64 streams over 512 MiB arrays (y = x; z = x + s y) in two launch
//            shapes: what a plain kernel gets out of HBM, for comparison with the memory-bound
//            kernels (springs, integrator)
//   int14, int8   the fused integrator's HBM pattern over 13.1M degrees of freedom (128 replicas
//            of 1600 particles, 32 beads, d = 2): per degree of freedom 8 doubles read and 6
//            written, either as 14 separate arrays (the thermostat's 4 chain velocities in
//            4 arrays, as the library stores them) or with the 4 chain velocities of a degree of
//            freedom next to each other (8 streams: one 32-byte read and write instead of 4)
//   lse2     latency, not throughput: one wavefront runs X <- -log(a + exp(c - X)) with the
//            library's FP64 exponential and logarithm, every iteration depending on the last.
//            This is the least a sequential exchange recursion (Eqs. 6, 11) must spend per row
//            if everything but the newest term is summed off the chain: the model against
//            which the recursion kernels' time per row is read.
//   f64:*    FP64 instruction costs, each measured as that instruction plus one FP64 multiply
//            per chain step (the multiply keeps the chain's value in range), so the
//            instruction's own cost is the kind's figure minus `f64:mul`:
//            fma, mul, add, max, ldexp, rndne, cvt (double -> int -> double counts two)
//   exp64    the library's FP64 exponential (fast_exp.h): throughput per call, plus one add and
//            the multiply
// The results decide the pair kernel's design: whether a Gram-matrix formulation on the matrix
// cores (|r_i - r_j|^2 = |r_i|^2 + |r_j|^2 - 2 r_i.r_j) can beat the plain vector form; and the
// FP64 exponential's form in the exchange sums and the FP64 pair kernel.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#include "../csrc/fast_exp.h"

typedef float f4 __attribute__((ext_vector_type(4)));

#define CK(x)                                                                     \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

constexpr int kBlocks = 2048, kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_fma(float* out, int iters) {
  float v[8];
  for (int q = 0; q < 8; ++q) v[q] = 0.1f * q + threadIdx.x * 1e-4f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = __builtin_fmaf(v[q], 0.999f, 1e-4f);
  }
  float s = 0.f;
  for (int q = 0; q < 8; ++q) s += v[q];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_exp(float* out, int iters) {
  float v[8];
  for (int q = 0; q < 8; ++q) v[q] = 0.1f * q + threadIdx.x * 1e-4f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = __builtin_amdgcn_exp2f(-v[q]);   // stays in (0, 1]
  }
  float s = 0.f;
  for (int q = 0; q < 8; ++q) s += v[q];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int SHAPE>
__global__ __launch_bounds__(kThreads) void k_mfma(float* out, int iters) {
  f4 acc[4];
  for (int q = 0; q < 4; ++q) acc[q] = (f4){0.f, 0.f, 0.f, 0.f};
  const float a = 1e-3f * threadIdx.x, b = 2e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (SHAPE == 16) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
      else acc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[q], 0, 0, 0);
    }
  }
  float s = 0.f;
  for (int q = 0; q < 4; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_mix(float* out, int iters) {
  f4 acc[4];
  for (int q = 0; q < 4; ++q) acc[q] = (f4){0.f, 0.f, 0.f, 0.f};
  float v[8];
  for (int q = 0; q < 8; ++q) v[q] = 0.1f * q + threadIdx.x * 1e-4f;
  const float a = 1e-3f * threadIdx.x, b = 2e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[q], 0, 0, 0);
      v[2 * q] = __builtin_amdgcn_exp2f(-v[2 * q]);
      v[2 * q + 1] = __builtin_amdgcn_exp2f(-v[2 * q + 1]);
    }
  }
  float s = 0.f;
  for (int q = 0; q < 4; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  for (int q = 0; q < 8; ++q) s += v[q];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Eight partners per iteration; the particle's position moves with its accumulated force so
// that nothing is loop-invariant, and the eight pairs of an iteration are independent.
__global__ __launch_bounds__(kThreads) void k_pair(float* out, int iters) {
  float xj[8][2], Fj[8][2];
  for (int b = 0; b < 8; ++b) {
    xj[b][0] = 0.37f * b - 1.1f + threadIdx.x * 1e-3f;
    xj[b][1] = 0.21f * b - 0.7f;
    Fj[b][0] = Fj[b][1] = 0.f;
  }
  float x0 = 0.05f, x1 = -0.03f, F0 = 0.f, F1 = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const float d0 = x0 - xj[b][0], d1 = x1 - xj[b][1];
      float r2 = d0 * d0;
      r2 = __builtin_fmaf(d1, d1, r2);
      const float u = __builtin_amdgcn_exp2f(-r2);
      F0 = __builtin_fmaf(u, d0, F0);
      F1 = __builtin_fmaf(u, d1, F1);
      Fj[b][0] = __builtin_fmaf(-u, d0, Fj[b][0]);
      Fj[b][1] = __builtin_fmaf(-u, d1, Fj[b][1]);
    }
    x0 = __builtin_fmaf(F0, 1e-9f, x0);
    x1 = __builtin_fmaf(F1, 1e-9f, x1);
  }
  float s = F0 + F1;
  for (int b = 0; b < 8; ++b) s += Fj[b][0] + Fj[b][1];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

enum F64Kind { kF64Fma, kF64Mul, kF64Add, kF64Max, kF64Ldexp, kF64Rndne, kF64Cvt, kExp64 };

template <int KIND>
__global__ __launch_bounds__(kThreads) void k_f64(float* out, int iters) {
  __shared__ double tab[pimd::kExpTable];
  pimd::fill_exp_table(tab);
  __syncthreads();
  double v[8];
  for (int q = 0; q < 8; ++q) v[q] = 0.5 + 0.01 * q + threadIdx.x * 1e-5;
  const int e = (int)(blockIdx.x >> 20);   // 0 at run time, unknown to the compiler
  const double c = 0.25 + e;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double w = v[q];
      if (KIND == kF64Fma) w = fma(w, 0.999, 1e-4);
      if (KIND == kF64Add) w = w + c;
      if (KIND == kF64Max) w = fmax(w, c);
      if (KIND == kF64Ldexp) w = ldexp(w, e);
      if (KIND == kF64Rndne) w = rint(w);
      if (KIND == kF64Cvt) w = (double)(int)w + c;
      if (KIND == kExp64) w = pimd::fast_exp_finite(-w, tab) + c;
      v[q] = w * 0.9999;   // the multiply every kind carries (f64:mul alone is just this)
    }
  }
  double s = 0.0;
  for (int q = 0; q < 8; ++q) s += v[q];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ x, double2* __restrict__ y, long long n2) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n2; i += (long long)gridDim.x * 256) y[i] = x[i];
}

// one workgroup per 4 x 256 double2: each thread moves four, all loads issued before the stores
__global__ __launch_bounds__(256) void k_copy4(const double2* __restrict__ x, double2* __restrict__ y, long long n2) {
  const long long base = blockIdx.x * 1024LL + threadIdx.x;
  double2 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long i = base + 256LL * k;
    v[k] = i < n2 ? x[i] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long i = base + 256LL * k;
    if (i < n2) y[i] = v[k];
  }
}

__global__ __launch_bounds__(256) void k_triad(const double2* __restrict__ x, const double2* __restrict__ y,
                                               double2* __restrict__ z, double s, long long n2) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n2; i += (long long)gridDim.x * 256) {
    const double2 a = x[i], b = y[i];
    z[i] = make_double2(a.x + s * b.x, a.y + s * b.y);
  }
}

// the integrator's streams: f, fp, p, x, v0..v3 read; x, p, v0..v3 written (separate arrays)
__global__ __launch_bounds__(256) void k_int14(const double* __restrict__ f, const double* __restrict__ fp,
                                               double* __restrict__ p, double* __restrict__ x,
                                               double* __restrict__ v, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const double a = f[i] + fp[i], pv = p[i], xv = x[i];
  double w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = v[k * n + i];
  const double pn = fma(0.01, a, pv) * (1.0 - 1e-3 * w[0]);
  x[i] = fma(0.01, pn, xv);
  p[i] = pn;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k * n + i] = fma(w[k], 0.999, 1e-3 * a);
}

// the same with the four chain velocities of a degree of freedom in one 32-byte record
__global__ __launch_bounds__(256) void k_int8(const double* __restrict__ f, const double* __restrict__ fp,
                                              double* __restrict__ p, double* __restrict__ x,
                                              double4* __restrict__ v, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const double a = f[i] + fp[i], pv = p[i], xv = x[i];
  const double4 w = v[i];
  const double pn = fma(0.01, a, pv) * (1.0 - 1e-3 * w.x);
  x[i] = fma(0.01, pn, xv);
  p[i] = pn;
  v[i] = make_double4(fma(w.x, 0.999, 1e-3 * a), fma(w.y, 0.999, 1e-3 * a), fma(w.z, 0.999, 1e-3 * a),
                      fma(w.w, 0.999, 1e-3 * a));
}

// best of five launches, in GB/s for `bytes` moved per launch
template <typename L>
static double stream_gbs(L launch, double bytes) {
  hipEvent_t a, b;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  launch();
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int k = 0; k < 5; ++k) {
    CK(hipEventRecord(a));
    launch();
    CK(hipEventRecord(b));
    CK(hipEventSynchronize(b));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, a, b));
    if (ms < best) best = ms;
  }
  CK(hipEventDestroy(a));
  CK(hipEventDestroy(b));
  return bytes / (best * 1e-3) / 1e9;
}

// One wavefront: a dependent chain of two-term log-sum-exps (see lse2 above).
__global__ __launch_bounds__(64) void k_lse2_chain(double* out, int iters) {
  __shared__ double tab[pimd::kExpTable];
  pimd::fill_exp_table(tab);
  __syncthreads();
  double x = 0.1 * threadIdx.x;
  const double a = 1.0 + 1e-3 * threadIdx.x, c = 0.25;
  for (int i = 0; i < iters; ++i) x = -pimd::fast_log(a + pimd::fast_exp(c - x, tab));
  out[threadIdx.x] = x;
}

template <typename K>
static double time_ms(K kern, float* out, int iters) {
  hipEvent_t a, b;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  hipLaunchKernelGGL(kern, dim3(kBlocks), dim3(kThreads), 0, 0, out, iters);   // warm-up
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  CK(hipEventRecord(a));
  hipLaunchKernelGGL(kern, dim3(kBlocks), dim3(kThreads), 0, 0, out, iters);
  CK(hipEventRecord(b));
  CK(hipEventSynchronize(b));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, a, b));
  CK(hipEventDestroy(a));
  CK(hipEventDestroy(b));
  return ms;
}

int main() {
  const int iters = 20000;
  const double waves = kBlocks * (kThreads / 64.0), simds = 1024.0, hz = 2.4e9;
  float* out = nullptr;
  CK(hipMalloc(&out, sizeof(float) * kBlocks * kThreads));
  // cycles per SIMD for `per_iter` units of the kind in every loop iteration of every wave
  auto cycles = [&](double ms, double per_iter) { return ms * 1e-3 * hz * simds / (waves * iters * per_iter); };
  double ms;
  ms = time_ms(k_fma, out, iters);
  std::printf("fma     %8.3f ms  %6.2f cycles per wave instruction\n", ms, cycles(ms, 8));
  ms = time_ms(k_exp, out, iters);
  std::printf("exp     %8.3f ms  %6.2f cycles per wave instruction\n", ms, cycles(ms, 8));
  ms = time_ms(k_mfma<16>, out, iters);
  std::printf("mfma16  %8.3f ms  %6.2f cycles per instruction\n", ms, cycles(ms, 4));
  ms = time_ms(k_mfma<4>, out, iters);
  std::printf("mfma4   %8.3f ms  %6.2f cycles per instruction\n", ms, cycles(ms, 4));
  ms = time_ms(k_mix, out, iters);
  std::printf("mix     %8.3f ms  %6.2f cycles per iteration (4 mfma4 + 8 exp)\n", ms, cycles(ms, 1));
  ms = time_ms(k_pair, out, iters);
  std::printf("pair    %8.3f ms  %6.2f cycles per 64 pairs (one wave step)\n", ms, cycles(ms, 8));
  {
    const int it64 = iters / 4;
    auto f64 = [&](const char* name, auto kern) {
      const double m = time_ms(kern, out, it64);
      std::printf("%-12s %8.3f ms  %6.2f cycles per wave step\n", name, m,
                  m * 1e-3 * hz * simds / (waves * it64 * 8.0));
    };
    f64("f64:mul", k_f64<kF64Mul>);
    f64("f64:fma", k_f64<kF64Fma>);
    f64("f64:add", k_f64<kF64Add>);
    f64("f64:max", k_f64<kF64Max>);
    f64("f64:ldexp", k_f64<kF64Ldexp>);
    f64("f64:rndne", k_f64<kF64Rndne>);
    f64("f64:cvt", k_f64<kF64Cvt>);
    f64("exp64", k_f64<kExp64>);
  }
  CK(hipFree(out));

  {
    double* o64 = nullptr;
    CK(hipMalloc(&o64, 64 * sizeof(double)));
    const int chain = 200000;
    hipEvent_t a, b;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
    hipLaunchKernelGGL(k_lse2_chain, dim3(1), dim3(64), 0, 0, o64, 1000);   // warm-up
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(a));
    hipLaunchKernelGGL(k_lse2_chain, dim3(1), dim3(64), 0, 0, o64, chain);
    CK(hipEventRecord(b));
    CK(hipEventSynchronize(b));
    float lms = 0.f;
    CK(hipEventElapsedTime(&lms, a, b));
    const double ns = lms * 1e6 / chain;
    std::printf("lse2    %8.3f ms  %6.1f ns (%5.0f cycles at 2.4 GHz) per dependent two-term log-sum-exp\n",
                lms, ns, ns * 2.4);
    CK(hipEventDestroy(a));
    CK(hipEventDestroy(b));
    CK(hipFree(o64));
  }

  const long long n = 64LL << 20;   // doubles per array: 512 MiB
  double *x = nullptr, *y = nullptr, *z = nullptr;
  CK(hipMalloc(&x, n * sizeof(double)));
  CK(hipMalloc(&y, n * sizeof(double)));
  CK(hipMalloc(&z, n * sizeof(double)));
  CK(hipMemset(x, 0, n * sizeof(double)));
  CK(hipMemset(y, 0, n * sizeof(double)));
  const unsigned grid = 256 * 16;
  const long long n2 = n / 2;
  const double gc = stream_gbs([&] { hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0,
                                                        (const double2*)x, (double2*)z, n2); },
                               2.0 * n * sizeof(double));
  std::printf("copy    %8.1f GB/s (read 512 MiB, write 512 MiB; 4096 workgroups, grid stride)\n", gc);
  const unsigned grid4 = (unsigned)((n2 + 1023) / 1024);
  const double gc4 = stream_gbs([&] { hipLaunchKernelGGL(k_copy4, dim3(grid4), dim3(256), 0, 0,
                                                         (const double2*)x, (double2*)z, n2); },
                                2.0 * n * sizeof(double));
  std::printf("copy4   %8.1f GB/s (read 512 MiB, write 512 MiB; one workgroup per 16 KiB)\n", gc4);
  const double gt = stream_gbs([&] { hipLaunchKernelGGL(k_triad, dim3(grid), dim3(256), 0, 0, (const double2*)x,
                                                        (const double2*)y, (double2*)z, 0.5, n2); },
                               3.0 * n * sizeof(double));
  std::printf("triad   %8.1f GB/s (read 2 x 512 MiB, write 512 MiB)\n", gt);
  CK(hipFree(x));
  CK(hipFree(y));
  CK(hipFree(z));

  {
    const long long nd = 128LL * 1600 * 32 * 2;   // degrees of freedom
    double *f = nullptr, *fp = nullptr, *pp = nullptr, *xx = nullptr, *vv = nullptr;
    CK(hipMalloc(&f, nd * sizeof(double)));
    CK(hipMalloc(&fp, nd * sizeof(double)));
    CK(hipMalloc(&pp, nd * sizeof(double)));
    CK(hipMalloc(&xx, nd * sizeof(double)));
    CK(hipMalloc(&vv, 4 * nd * sizeof(double)));
    CK(hipMemset(f, 0, nd * sizeof(double)));
    CK(hipMemset(fp, 0, nd * sizeof(double)));
    CK(hipMemset(pp, 0, nd * sizeof(double)));
    CK(hipMemset(xx, 0, nd * sizeof(double)));
    CK(hipMemset(vv, 0, 4 * nd * sizeof(double)));
    const unsigned gi = (unsigned)((nd + 255) / 256);
    const double bytes = 14.0 * 8.0 * nd;
    const double g14 = stream_gbs([&] { hipLaunchKernelGGL(k_int14, dim3(gi), dim3(256), 0, 0, f, fp, pp, xx, vv, nd); },
                                  bytes);
    std::printf("int14   %8.1f GB/s (%.1f us; 14 arrays of 8-byte elements)\n", g14, bytes / g14 * 1e-3);
    const double g8 = stream_gbs([&] { hipLaunchKernelGGL(k_int8, dim3(gi), dim3(256), 0, 0, f, fp, pp, xx,
                                                          (double4*)vv, nd); },
                                 bytes);
    std::printf("int8    %8.1f GB/s (%.1f us; chain velocities as 32-byte records)\n", g8, bytes / g8 * 1e-3);
    CK(hipFree(f));
    CK(hipFree(fp));
    CK(hipFree(pp));
    CK(hipFree(xx));
    CK(hipFree(vv));
  }
  return 0;
}
