// k_exchange.hip -- exchange potentials, connection probabilities and end-bead forces.
//
// Notation (1-based particles).  c = (1/2) m omega_P^2, a_l = r_l^1, b_l = r_l^P,
// link_l = c |b_l - a_{l+1}|^2 (link_N = 0), close(v,u) = c |b_v - a_u|^2, and
// E^{[u,v]} = sum_{l=u}^v E_int^{(l)} + sum_{l=u}^{v-1} link_l + close(v,u), which is Eq. 7 for
// the ring u..v regrouped (the quantity the iteration of Eq. 10 accumulates).
//
// Normalised recursions.  Substituting this E into Eq. 6 and Eq. 11, every E_int and every
// link of a block except the first factor out of the sums.  With
//   H_n = beta V^{[1,n]} - beta sum_{l<=n} (E_int^{(l)} + link_l)                (forward)
//   K_u = beta V^{[u,N]} - beta (sum_{l>=u} E_int^{(l)} + sum_{l=u-1}^{N-1} link_l)  (backward)
// Eq. 6 and Eq. 11 become, with G^f_n = -H_n and G^b_i = -K_{N+1-i} (G_0 = 0 in both),
//   G_i = log sum_{j<i} exp(alpha_{i,j} + G_j),
//   alpha_{i,j} = (i-1-j) log xi + rho_i + gamma_j - beta c |p_i - q_j|^2,
// forward : rho_i = beta link_i - log i,  gamma_j = 0,           p_i = b_i,       q_j = a_{j+1}
// backward: rho_i = beta link_{N-i},      gamma_j = -log(N - j), p_i = a_{N+1-i}, q_j = b_{N-j}
// so both are one lower-triangular log-sum-exp recursion whose terms need only end beads and
// links: no prefix sums and no O(N^2) table.  Then V_xi^{[1,N]} = sum E_int + sum link - G^f_N/beta,
// and Eqs. 12-13 read
//   Pr[l -> l'] = exp((l-l') log xi - log l + G^f_{l'-1} + G^b_{N-l} - G^f_N - beta close(l,l'))  (l' <= l)
//   Pr[l -> l+1] = -expm1(G^f_l + G^b_{N-l} - G^f_N - beta link_l).
//
// Recursion schedule (one workgroup per replica and direction).  Rows are processed in
// blocks of 64 (lane = row).  For a block: (1) the four waves sum the contributions of all
// earlier columns in log-sum-exp form; (2) wave 0 runs a max-plus pass over the in-block
// columns that gives each row a scale D_i with every scaled coefficient <= 1; (3) all waves
// evaluate the scaled coefficients exp(alpha + D_j - D_i); (4) wave 0 solves the scaled
// in-block triangular system by forward substitution with lane broadcasts; G_i = D_i + log w_i.
// The scaled unknowns satisfy 1 <= w_i <= 2^64, so nothing overflows whatever the dynamic
// range of the cycle weights.
#include "pimd_internal.h"
#include "device_util.h"

namespace pimd {

constexpr int kRecThreads = 256;

template <int D>
struct RecMap {
  const double* a; const double* b; const double* lk;
  int N, npp, dir;
  double blink;  // beta
  __device__ inline void row(int i, double (&pt)[D], double& rho) const {
    // valid for 1 <= i <= N
    if (dir == 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) pt[c] = b[(long long)c * npp + (i - 1)];
      rho = blink * lk[i - 1] - log((double)i);
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) pt[c] = a[(long long)c * npp + (N - i)];
      rho = (i < N) ? blink * lk[N - i - 1] : 0.0;
    }
  }
  __device__ inline void col(int j, double (&pt)[D], double& gam) const {
    // valid for 0 <= j <= N-1
    if (dir == 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) pt[c] = a[(long long)c * npp + j];
      gam = 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) pt[c] = b[(long long)c * npp + (N - j - 1)];
      gam = -log((double)(N - j));
    }
  }
};

template <int D>
__global__ __launch_bounds__(kRecThreads) void k_recursion(const RepDev* __restrict__ reps,
                                                           const double* __restrict__ ends,
                                                           const double* __restrict__ link,
                                                           double* __restrict__ gf, double* __restrict__ gb) {
  __shared__ double Am[kTile * kTile];   // column-major: Am[s * 64 + lane]
  __shared__ double pm[4][kTile], ps[4][kTile];
  __shared__ double Dl[kTile];
  const int rep = blockIdx.x >> 1, dir = blockIdx.x & 1;
  const RepDev& R = reps[rep];
  const int N = R.n;
  RecMap<D> mp;
  mp.a = ends + 2LL * D * R.part;
  mp.b = mp.a + (long long)D * R.npp;
  mp.lk = link + R.part;
  mp.N = N; mp.npp = R.npp; mp.dir = dir; mp.blink = R.beta;
  double* G = (dir == 0 ? gf : gb) + R.part;
  const double bc = R.beta * R.c, lnxi = R.lnxi;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = (N + 1 + kTile - 1) / kTile;   // rows 0..N

  for (int blk = 0; blk < nblk; ++blk) {
    const int i = blk * kTile + lane;
    const bool valid = (i >= 1 && i <= N);
    double pi[D], rho = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) pi[c] = 0.0;
    if (valid) mp.row(i, pi, rho);

    // (1) earlier columns j < blk*64: online log-sum-exp, columns split over the waves
    double m = -1e300, s = 0.0;
    const int jend = blk * kTile;
    if (valid && jend > 0) {
      const int per = (jend + 3) / 4;
      const int ja = wave * per, jb = min(jend, ja + per);
      for (int j = ja; j < jb; ++j) {
        double qj[D], gam;
        mp.col(j, qj, gam);
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) { double t = pi[c] - qj[c]; d2 = fma(t, t, d2); }
        double t = xi_pow_log(i - 1 - j, lnxi) + rho + gam - bc * d2 + G[j];
        double dlt = t - m;
        double e = exp(-fabs(dlt));
        bool up = dlt > 0.0;
        s = up ? fma(s, e, 1.0) : s + e;
        m = up ? t : m;
      }
    }
    pm[wave][lane] = m;
    ps[wave][lane] = s;
    // (2a) in-block coefficients alpha_{i,j}, j = blk*64 + sc, stored column-major
    for (int sc = wave * 16; sc < wave * 16 + 16; ++sc) {
      const int j = blk * kTile + sc;
      double v = -INFINITY;
      if (valid && j < i) {
        double qj[D], gam;
        mp.col(j, qj, gam);
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) { double t = pi[c] - qj[c]; d2 = fma(t, t, d2); }
        v = xi_pow_log(i - 1 - j, lnxi) + rho + gam - bc * d2;
      }
      Am[sc * kTile + lane] = v;
    }
    __syncthreads();

    if (wave == 0) {
      // combine the four partial sums: log of the earlier-column sum, LB
      double M = fmax(fmax(pm[0][lane], pm[1][lane]), fmax(pm[2][lane], pm[3][lane]));
      double S = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) S += ps[w][lane] * exp(pm[w][lane] - M);
      double LB = (S > 0.0) ? M + log(S) : -INFINITY;
      if (i == 0) LB = 0.0;      // seed row: G_0 = 0
      if (!valid && i != 0) LB = 0.0;  // padding rows stay finite and unused
      // (2b) max-plus scale pass: D_i = max(LB_i, max_{s<lane} (alpha_{i,s} + D_s))
      double run = LB;
      for (int sc = 0; sc < kTile; ++sc) {
        double Ds = read_lane(run, sc);
        if (lane > sc) run = fmax(run, Am[sc * kTile + lane] + Ds);
      }
      Dl[lane] = run;
      pm[0][lane] = LB;
    }
    __syncthreads();
    // (3) scaled coefficients exp(alpha + D_s - D_i) <= 1
    {
      const double Di = Dl[lane];
      for (int sc = wave * 16; sc < wave * 16 + 16; ++sc) {
        double v = Am[sc * kTile + lane];
        Am[sc * kTile + lane] = (lane > sc) ? exp(v + Dl[sc] - Di) : 0.0;
      }
    }
    __syncthreads();
    if (wave == 0) {
      // (4) forward substitution on the scaled unknowns w_i = exp(G_i - D_i)
      const double Di = Dl[lane];
      double acc = exp(pm[0][lane] - Di);
      for (int sc = 0; sc < kTile; ++sc) {
        double ws = read_lane(acc, sc);
        if (lane > sc) acc = fma(Am[sc * kTile + lane], ws, acc);
      }
      if (i <= N) G[i] = Di + log(acc);
    }
    __syncthreads();
  }
}

hipError_t launch_recursion(const Dims& d, const DevPtrs& w, hipStream_t s) {
  dim3 grid((unsigned)(2 * d.R)), block(kRecThreads);
  switch (d.D) {
    case 1: hipLaunchKernelGGL(k_recursion<1>, grid, block, 0, s, w.reps, w.ends, w.link, w.gf, w.gb); break;
    case 2: hipLaunchKernelGGL(k_recursion<2>, grid, block, 0, s, w.reps, w.ends, w.link, w.gf, w.gb); break;
    case 3: hipLaunchKernelGGL(k_recursion<3>, grid, block, 0, s, w.reps, w.ends, w.link, w.gf, w.gb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ probabilities

// Pr[l -> l'] for 0-based particles lr >= lc (entry of Eq. 12 in normalised form).
template <int D>
__device__ inline double prob_lower(int lr, int lc, int N, const double* a, const double* b, int npp,
                                    const double* gf, const double* gb, double bc, double lnxi) {
  double d2 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double t = b[(long long)c * npp + lr] - a[(long long)c * npp + lc];
    d2 = fma(t, t, d2);
  }
  double ex = xi_pow_log(lr - lc, lnxi) - log((double)(lr + 1)) + gf[lc] + gb[N - 1 - lr] - gf[N] - bc * d2;
  return exp(ex);
}

// Pr[l -> l+1] for 0-based l <= N-2 (Eq. 13 in normalised form), 0 for l = N-1.
__device__ inline double prob_next(int l, int N, const double* lk, const double* gf, const double* gb, double beta) {
  if (l >= N - 1) return 0.0;
  return -expm1(gf[l + 1] + gb[N - 1 - l] - gf[N] - beta * lk[l]);
}

// One 64x64 tile of the lower triangle: rows lr in block rb, columns lc in block cb <= rb.
// Row partials (sum Pr, sum Pr a_{l'}, sum Pr close) -> rowpart[q][cb][lr];
// column partials (sum Pr, sum Pr b_l) -> colpart[q][rb][lc].
template <int D>
__global__ __launch_bounds__(256) void k_probs(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                               const double* __restrict__ ends, const double* __restrict__ gf,
                                               const double* __restrict__ gb, double* __restrict__ rowpart,
                                               double* __restrict__ colpart) {
  __shared__ double T[kTile * (kTile + 1)];  // T[col * 65 + row], padded against bank conflicts
  __shared__ double red[4][D + 2][kTile];
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  const int N = R.n, rb = wk.y, cb = wk.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* a = ends + 2LL * D * R.part;
  const double* b = a + (long long)D * R.npp;
  const double* g_f = gf + R.part;
  const double* g_b = gb + R.part;
  const double bc = R.beta * R.c, lnxi = R.lnxi;
  const int lr = rb * kTile + lane;
  double rs = 0.0, ra[D], sc = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) ra[c] = 0.0;
  for (int k = 0; k < 16; ++k) {
    const int cl = wave * 16 + k;
    const int lc = cb * kTile + cl;
    double pr = 0.0;
    if (lr < N && lc <= lr) {
      pr = prob_lower<D>(lr, lc, N, a, b, R.npp, g_f, g_b, bc, lnxi);
      double d2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        double av = a[(long long)c * R.npp + lc];
        ra[c] = fma(pr, av, ra[c]);
        double t = b[(long long)c * R.npp + lr] - av;
        d2 = fma(t, t, d2);
      }
      rs += pr;
      sc = fma(pr, R.c * d2, sc);
    }
    T[cl * (kTile + 1) + lane] = pr;
  }
  red[wave][0][lane] = rs;
#pragma unroll
  for (int c = 0; c < D; ++c) red[wave][1 + c][lane] = ra[c];
  red[wave][D + 1][lane] = sc;
  __syncthreads();
  const long long nb = R.nblk, npp = R.npp;
  double* rp = rowpart + (long long)(D + 2) * R.prob;
  double* cp = colpart + (long long)(D + 2) * R.prob;
  if (wave == 0 && lr < N) {
    for (int q = 0; q < D + 2; ++q) {
      double v = red[0][q][lane] + red[1][q][lane] + red[2][q][lane] + red[3][q][lane];
      rp[((long long)q * nb + cb) * npp + lr] = v;
    }
  }
  __syncthreads();
  // column sums: thread -> column lane, rows wave*16 .. +16
  {
    const int lc = cb * kTile + lane;
    double cs = 0.0, cbv[D];
#pragma unroll
    for (int c = 0; c < D; ++c) cbv[c] = 0.0;
    for (int k = 0; k < 16; ++k) {
      const int rl = wave * 16 + k;
      const int lrr = rb * kTile + rl;
      double pr = T[lane * (kTile + 1) + rl];
      if (lrr < N) {
        cs += pr;
#pragma unroll
        for (int c = 0; c < D; ++c) cbv[c] = fma(pr, b[(long long)c * npp + lrr], cbv[c]);
      }
    }
    red[wave][0][lane] = cs;
#pragma unroll
    for (int c = 0; c < D; ++c) red[wave][1 + c][lane] = cbv[c];
    __syncthreads();
    if (wave == 0 && lc < N) {
      for (int q = 0; q < D + 1; ++q) {
        double v = red[0][q][lane] + red[1][q][lane] + red[2][q][lane] + red[3][q][lane];
        cp[((long long)q * nb + rb) * npp + lc] = v;
      }
    }
  }
}

// Per particle: reduce the tile partials, add the Pr[l -> l+1] terms, and apply Eqs. 15-16:
//   F(bead P of l) += -kappa sum_{l'} Pr[l->l'] (2 b_l - r_l^{P-1} - a_{l'})
//   F(bead 1 of l) += -kappa sum_{l'} Pr[l'->l] (2 a_l - r_l^2 - b_{l'})
// The expected spring energy S = sum E_int + sum_l Pr[l->l+1] link_l + sum_{l'<=l} Pr close(l,l')
// is summed per workgroup into reducepart.
template <int D>
__global__ __launch_bounds__(256) void k_probs_reduce(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                                      const double* __restrict__ x, double* __restrict__ f,
                                                      const double* __restrict__ ends, const double* __restrict__ link,
                                                      const double* __restrict__ gf, const double* __restrict__ gb,
                                                      const double* __restrict__ rowpart,
                                                      const double* __restrict__ colpart,
                                                      double* __restrict__ reducepart, int P) {
  __shared__ double lds[2 * 4];
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  const int N = R.n;
  const int l = wk.y + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (l < N) {
    const double* a = ends + 2LL * D * R.part;
    const double* b = a + (long long)D * R.npp;
    const double* lk = link + R.part;
    const double* g_f = gf + R.part;
    const double* g_b = gb + R.part;
    const long long nb = R.nblk, npp = R.npp;
    const double* rp = rowpart + (long long)(D + 2) * R.prob;
    const double* cp = colpart + (long long)(D + 2) * R.prob;
    const int bl = l / kTile;
    double rs = 0.0, ra[D], scl = 0.0, cs = 0.0, cbv[D];
#pragma unroll
    for (int c = 0; c < D; ++c) { ra[c] = 0.0; cbv[c] = 0.0; }
    for (int cb = 0; cb <= bl; ++cb) {
      rs += rp[((long long)0 * nb + cb) * npp + l];
#pragma unroll
      for (int c = 0; c < D; ++c) ra[c] += rp[((long long)(1 + c) * nb + cb) * npp + l];
      scl += rp[((long long)(D + 1) * nb + cb) * npp + l];
    }
    for (int rb = bl; rb < R.nblk; ++rb) {
      cs += cp[((long long)0 * nb + rb) * npp + l];
#pragma unroll
      for (int c = 0; c < D; ++c) cbv[c] += cp[((long long)(1 + c) * nb + rb) * npp + l];
    }
    const double pn = prob_next(l, N, lk, g_f, g_b, R.beta);          // Pr[l -> l+1]
    const double pp = (l > 0) ? prob_next(l - 1, N, lk, g_f, g_b, R.beta) : 0.0;  // Pr[l-1 -> l]
    rs += pn;
    cs += pp;
    const double kap = R.kappa;
    double* fr = f + R.dof;
    const double* xr = x + R.dof;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      if (pn != 0.0) ra[c] = fma(pn, a[(long long)c * npp + l + 1], ra[c]);
      if (pp != 0.0) cbv[c] = fma(pp, b[(long long)c * npp + l - 1], cbv[c]);
      const double al = a[(long long)c * npp + l], bl_ = b[(long long)c * npp + l];
      const double rP1 = xr[((long long)c * P + (P - 2)) * N + l];   // r_l^{P-1}
      const double r2 = xr[((long long)c * P + 1) * N + l];           // r_l^2
      fr[((long long)c * P + (P - 1)) * N + l] += -kap * (rs * (2.0 * bl_ - rP1) - ra[c]);
      fr[((long long)c * P + 0) * N + l] += -kap * (cs * (2.0 * al - r2) - cbv[c]);
    }
    acc[0] = scl + pn * lk[l];
    acc[1] = 0.0;
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    reducepart[2LL * blockIdx.x + 0] = acc[0];
    reducepart[2LL * blockIdx.x + 1] = acc[1];
  }
}

hipError_t launch_probs(const Dims& d, const DevPtrs& w, hipStream_t s) {
  if (d.nprobwork == 0) return hipSuccess;
  dim3 grid((unsigned)d.nprobwork), block(256);
  switch (d.D) {
    case 1: hipLaunchKernelGGL(k_probs<1>, grid, block, 0, s, w.reps, w.probwork, w.ends, w.gf, w.gb, w.rowpart, w.colpart); break;
    case 2: hipLaunchKernelGGL(k_probs<2>, grid, block, 0, s, w.reps, w.probwork, w.ends, w.gf, w.gb, w.rowpart, w.colpart); break;
    case 3: hipLaunchKernelGGL(k_probs<3>, grid, block, 0, s, w.reps, w.probwork, w.ends, w.gf, w.gb, w.rowpart, w.colpart); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_probs_reduce(const Dims& d, const DevPtrs& w, hipStream_t s) {
  if (d.nreducewg == 0) return hipSuccess;
  dim3 grid((unsigned)d.nreducewg), block(256);
#define L(DD) hipLaunchKernelGGL(k_probs_reduce<DD>, grid, block, 0, s, w.reps, w.reducework, w.x, w.f, w.ends, \
                                 w.link, w.gf, w.gb, w.rowpart, w.colpart, w.reducepart, d.P)
  switch (d.D) {
    case 1: L(1); break;
    case 2: L(2); break;
    case 3: L(3); break;
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

// ------------------------------------------------------------------ debug outputs

// X[n] = beta V^{[1,n]} = -G^f_n + beta sum_{l<=n} (E_int^{(l)} + link_l)  (n = 0..N)
// Y[u] = beta V^{[u,N]} = -G^b_{N+1-u} + beta (sum_{l>=u} E_int^{(l)} + sum_{l=u-1}^{N-1} link_l)
// Single-thread compensated prefix sums (diagnostic path only).
__global__ void k_debug_potentials(const RepDev* __restrict__ reps, int r, const double* __restrict__ eint,
                                   const double* __restrict__ link, const double* __restrict__ gf,
                                   const double* __restrict__ gb, double* X, double* Y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const RepDev& R = reps[r];
  const int N = R.n;
  const double* ei = eint + R.part;
  const double* lk = link + R.part;
  const double* g_f = gf + R.part;
  const double* g_b = gb + R.part;
  double s = 0.0, c = 0.0;
  X[0] = 0.0;
  for (int n = 1; n <= N; ++n) {
    double v = ei[n - 1] + lk[n - 1];
    double t = s + v;
    c += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
    s = t;
    X[n] = -g_f[n] + R.beta * (s + c);
  }
  s = 0.0; c = 0.0;
  Y[0] = 0.0;
  Y[N + 1] = 0.0;
  for (int u = N; u >= 1; --u) {
    double v = ei[u - 1] + (u >= 2 ? lk[u - 2] : 0.0);
    double t = s + v;
    c += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
    s = t;
    Y[u] = -g_b[N + 1 - u] + R.beta * (s + c);
  }
}

template <int D>
__global__ void k_debug_probs(const RepDev* __restrict__ reps, int r, int row0, int nrows,
                              const double* __restrict__ ends, const double* __restrict__ link,
                              const double* __restrict__ gf, const double* __restrict__ gb, double* G) {
  const RepDev& R = reps[r];
  const int N = R.n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nrows * N) return;
  const int lr = row0 + (int)(idx / N), lc = (int)(idx % N);
  const double* a = ends + 2LL * D * R.part;
  const double* b = a + (long long)D * R.npp;
  double v = 0.0;
  if (lc <= lr) v = prob_lower<D>(lr, lc, N, a, b, R.npp, gf + R.part, gb + R.part, R.beta * R.c, R.lnxi);
  else if (lc == lr + 1) v = prob_next(lr, N, link + R.part, gf + R.part, gb + R.part, R.beta);
  G[idx] = v;
}

hipError_t launch_debug_potentials(const Dims& d, const DevPtrs& w, int r, double* X, double* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_potentials, dim3(1), dim3(64), 0, s, w.reps, r, w.eint, w.link, w.gf, w.gb, X, Y);
  return hipGetLastError();
}

// Rows [row0, row0 + nrows) of the dense probability matrix of replica r (n = its N) into G.
hipError_t launch_debug_probs(const Dims& d, const DevPtrs& w, int r, int n, int row0, int nrows, double* G,
                              hipStream_t s) {
  const long long tot = (long long)nrows * n;
  dim3 grid((unsigned)((tot + 255) / 256)), block(256);
#define L(DD) hipLaunchKernelGGL(k_debug_probs<DD>, grid, block, 0, s, w.reps, r, row0, nrows, w.ends, w.link, w.gf, w.gb, G)
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
