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
// links: no prefix sums and no O(N^2) table.  V_xi^{[1,N]} = sum E_int + sum link - G^f_N/beta.
//
// Probabilities without a G matrix.  Eq. 12 in this notation is a recursion term times a
// factor of its row: Pr[n -> m+1] = exp(alpha^f_{n,m} + G^f_m) exp(G^b_{N-n} - G^f_N - beta link_n)
// (forward row n) and Pr[l -> u] = exp(alpha^b_{i,j} + G^b_j) exp(G^f_{u-1} - G^f_N - beta
// link_{u-1}) (backward row i = N+1-u, column j = N-l).  So the row sums that Eq. 16 needs
// (sum_{l'} Pr[l->l'] a_{l'}, and sum Pr close for the energy) are weighted averages over the
// terms of forward row l, and the column sums of Eq. 15 (sum_l Pr[l->u] b_l) weighted averages
// over backward row N+1-u.  Each recursion row therefore also accumulates the term-weighted
// average of its column points q_j and of |p_i - q_j|^2; a per-particle pass applies the row
// factors, adds Pr[l -> l+1] = -expm1(G^f_l + G^b_{N-l} - G^f_N - beta link_l) (Eq. 13) and forms
// the end-bead forces of Eqs. 15-16.  The N^2/2 probabilities are never stored or recomputed.
//
// Recursion schedule (one workgroup per replica and direction, eight wavefronts).  Rows are
// processed in blocks of 64 (lane = row).  For a block: (0) a reference R_i = the largest term of
// the previous block's columns (a lower bound of the row's largest earlier term); (1) the eight
// waves sum exp(term - R_i) and its weighted payloads over all earlier columns (if a term ever
// exceeds R_i by more than the double range, that wave redoes its columns with a running
// maximum); (2) wave 0 runs a max-plus pass over the in-block columns giving each row a scale D_i
// with every scaled coefficient <= 1; (3) all waves evaluate exp(alpha + D_j - D_i); (4) wave 0
// solves the scaled in-block triangular system by forward substitution with lane broadcasts,
// four rows per round; G_i = D_i + log w_i; (5) the in-block weighted payloads.  The scaled
// unknowns satisfy 1 <= w_i <= 2^64, so nothing overflows whatever the range of the weights.
#include "pimd_internal.h"
#include "device_util.h"
#include "fast_exp.h"

namespace pimd {

// Row and column data of the generic recursion G_i = log sum_{j<i} exp(alpha_{i,j} + G_j).
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

constexpr int kRecWaves = 8;
constexpr int kRecThreads = 64 * kRecWaves;
constexpr int kColsPerWave = kTile / kRecWaves;

// How the xi^(i-1-j) factor enters a term: xi = 1 (nothing), xi = 0 (only j = i-1 survives),
// general xi (exact integer power times log xi).
enum XiMode { kXiOne = 0, kXiZero = 1, kXiGen = 2 };

template <int M>
__device__ inline double xi_term(int k, double lnxi) {
  if (M == kXiOne) return 0.0;
  if (M == kXiZero) return k == 0 ? 0.0 : -INFINITY;
  return (double)k * lnxi;
}

struct RowCtx {
  int i;
  double rowc, bc, lnxi;
};

// term t_{i,j} = alpha_{i,j} + G_j and |p_i - q_j|^2 for column record r4 = {q_j, gamma_j + G_j}.
template <int D, int XM>
__device__ inline double term_of(const RowCtx& rc, const double (&pi)[D], const double4& r4, int j, double& d2) {
  const double qv[3] = {r4.x, r4.y, r4.z};
  d2 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) { const double t = pi[c] - qv[c]; d2 = fma(t, t, d2); }
  return fma(-rc.bc, d2, rc.rowc + r4.w) + xi_term<XM>(rc.i - 1 - j, rc.lnxi);
}

// Sum of exp(t_j - R) over columns [ja, jb) with payload sums (q_j and |p_i - q_j|^2),
// two interleaved accumulator sets, records prefetched one round ahead.
template <int D, int XM>
__device__ inline void bulk_fixed(const RowCtx& rc, const double (&pi)[D], double R, const double4* __restrict__ rec,
                                  int ja, int jb, const double* tab, double& s_out, double (&P)[D + 1]) {
  double s[2] = {0.0, 0.0}, pq[2][D + 1];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q <= D; ++q) pq[h][q] = 0.0;
  double4 cur[4], nxt[4];
  auto ld = [&](double4 (&dst)[4], int j0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[u] = rec[min(j0 + u, jb - 1)];
  };
  if (ja < jb) ld(cur, ja);
  for (int j0 = ja; j0 < jb; j0 += 4) {
    if (j0 + 4 < jb) ld(nxt, j0 + 4);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u;
      double d2;
      double t = term_of<D, XM>(rc, pi, cur[u], j, d2);
      if (j >= jb) t = -INFINITY;
      const double e = fast_exp(t - R, tab);
      const int h = u & 1;
      s[h] += e;
      const double qv[3] = {cur[u].x, cur[u].y, cur[u].z};
#pragma unroll
      for (int c = 0; c < D; ++c) pq[h][c] = fma(e, qv[c], pq[h][c]);
      pq[h][D] = fma(e, d2, pq[h][D]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
  }
  s_out = s[0] + s[1];
#pragma unroll
  for (int q = 0; q <= D; ++q) P[q] = pq[0][q] + pq[1][q];
}

// Same sums with a running maximum m (result = exp(m) * (s, P)); used when a term exceeds the
// fixed reference by more than the double range.
template <int D, int XM>
__device__ inline void bulk_online(const RowCtx& rc, const double (&pi)[D], const double4* __restrict__ rec, int ja,
                                   int jb, const double* tab, double& m_out, double& s_out, double (&P)[D + 1]) {
  double m = -1e300, s = 0.0, pq[D + 1];
#pragma unroll
  for (int q = 0; q <= D; ++q) pq[q] = 0.0;
  for (int j = ja; j < jb; ++j) {
    const double4 r4 = rec[j];
    double d2;
    const double t = term_of<D, XM>(rc, pi, r4, j, d2);
    const double dl = t - m;
    const double e = fast_exp(-fabs(dl), tab);
    const double qv[3] = {r4.x, r4.y, r4.z};
    if (dl > 0.0) {
      s = fma(s, e, 1.0);
#pragma unroll
      for (int c = 0; c < D; ++c) pq[c] = fma(pq[c], e, qv[c]);
      pq[D] = fma(pq[D], e, d2);
      m = t;
    } else {
      s += e;
#pragma unroll
      for (int c = 0; c < D; ++c) pq[c] = fma(e, qv[c], pq[c]);
      pq[D] = fma(e, d2, pq[D]);
    }
  }
  m_out = m;
  s_out = s;
#pragma unroll
  for (int q = 0; q <= D; ++q) P[q] = pq[q];
}

template <int D, int XM>
__device__ inline void bulk_rows(const RowCtx& rc, const double (&pi)[D], double R, const double4* __restrict__ rec,
                                 int ja, int jb, const double* tab, double& m, double& s, double (&P)[D + 1]) {
  bulk_fixed<D, XM>(rc, pi, R, rec, ja, jb, tab, s, P);
  m = R;
  bool bad = !isfinite(s);
#pragma unroll
  for (int q = 0; q <= D; ++q) bad = bad || !isfinite(P[q]);
  if (__any(bad)) bulk_online<D, XM>(rc, pi, rec, ja, jb, tab, m, s, P);
}

template <int D, int XM>
__device__ inline double max_term(const RowCtx& rc, const double (&pi)[D], const double4* __restrict__ rec, int j0,
                                  int n) {
  double mx = -INFINITY;
  for (int u = 0; u < n; ++u) {
    double d2;
    mx = fmax(mx, term_of<D, XM>(rc, pi, rec[j0 + u], j0 + u, d2));
  }
  return mx;
}

// LDS of one recursion workgroup.
template <int D>
struct RecShared {
  double tab[kExpTable];
  double Am[kTile * kTile];   // column-major: Am[col * 64 + row]
  double pm[kRecWaves][kTile], ps[kRecWaves][kTile];
  double pp[kRecWaves][D + 1][kTile];
  double Dl[kTile], LBl[kTile], Wl[kTile];
  double pbar[D + 1][kTile];
  int flag;
};

// Steps (2)-(5) for one block of 64 rows, given each wave's partial sums over the earlier
// columns in pm/ps/pp (log-sum-exp form: exp(m) (s, P)).  Writes G_i, adds G_i to the column
// records, optionally publishes the block (release store of `epoch`), and writes the weighted
// row averages.
template <int D>
__device__ inline void solve_block(RecShared<D>& sh, int blk, int N, const double (&pi)[D], double rho, bool valid,
                                   double bc, double lnxi, double4* __restrict__ rec, double* __restrict__ G,
                                   double* __restrict__ av, int npp, int* publish, int epoch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blk * kTile + lane;
  // (2a) in-block coefficients alpha_{i,j} (without G_j), j = blk*64 + sc, column-major
  for (int sc = wave * kColsPerWave; sc < (wave + 1) * kColsPerWave; ++sc) {
    const int j = blk * kTile + sc;
    double v = -INFINITY;
    if (valid && j < i) {
      const double4 r4 = rec[j];
      const double qv[3] = {r4.x, r4.y, r4.z};
      double d2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) { const double t = pi[c] - qv[c]; d2 = fma(t, t, d2); }
      v = xi_pow_log(i - 1 - j, lnxi) + rho + r4.w - bc * d2;
    }
    sh.Am[sc * kTile + lane] = v;
  }
  __syncthreads();

  if (wave == 0) {
    double M = sh.pm[0][lane];
#pragma unroll
    for (int w = 1; w < kRecWaves; ++w) M = fmax(M, sh.pm[w][lane]);
    double S = 0.0, PS[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) PS[q] = 0.0;
#pragma unroll
    for (int w = 0; w < kRecWaves; ++w) {
      const double f = sh.ps[w][lane] > 0.0 ? exp(sh.pm[w][lane] - M) : 0.0;
      S = fma(sh.ps[w][lane], f, S);
#pragma unroll
      for (int q = 0; q <= D; ++q) PS[q] = fma(sh.pp[w][q][lane], f, PS[q]);
    }
    double LB = (S > 0.0) ? M + log(S) : -INFINITY;
#pragma unroll
    for (int q = 0; q <= D; ++q) sh.pbar[q][lane] = S > 0.0 ? PS[q] / S : 0.0;
    if (i == 0) LB = 0.0;            // seed row: G_0 = 0
    if (!valid && i != 0) LB = 0.0;  // padding rows stay finite and unused
    sh.LBl[lane] = LB;
    // (2b) max-plus scales D_i = max(LB_i, max_{s<lane}(alpha_{i,s} + D_s)), four rows per round:
    // the four rows of a group are finished from broadcast values, then the rest updated.
    double run = LB, mine = 0.0;
    for (int s0 = 0; s0 < kTile; s0 += 4) {
      const double r0 = read_lane(run, s0), r1 = read_lane(run, s0 + 1);
      const double r2 = read_lane(run, s0 + 2), r3 = read_lane(run, s0 + 3);
      const double a10 = sh.Am[s0 * kTile + s0 + 1];
      const double a20 = sh.Am[s0 * kTile + s0 + 2], a21 = sh.Am[(s0 + 1) * kTile + s0 + 2];
      const double a30 = sh.Am[s0 * kTile + s0 + 3], a31 = sh.Am[(s0 + 1) * kTile + s0 + 3];
      const double a32 = sh.Am[(s0 + 2) * kTile + s0 + 3];
      const double D0 = r0;
      const double D1 = fmax(r1, a10 + D0);
      const double D2 = fmax(r2, fmax(a20 + D0, a21 + D1));
      const double D3 = fmax(r3, fmax(fmax(a30 + D0, a31 + D1), a32 + D2));
      const int g = lane - s0;
      if (g == 0) mine = D0;
      if (g == 1) mine = D1;
      if (g == 2) mine = D2;
      if (g == 3) mine = D3;
      if (g > 3) {
        const double u0 = sh.Am[s0 * kTile + lane] + D0, u1 = sh.Am[(s0 + 1) * kTile + lane] + D1;
        const double u2 = sh.Am[(s0 + 2) * kTile + lane] + D2, u3 = sh.Am[(s0 + 3) * kTile + lane] + D3;
        run = fmax(fmax(run, fmax(u0, u1)), fmax(u2, u3));
      }
    }
    sh.Dl[lane] = mine;
  }
  __syncthreads();
  // (3) scaled coefficients exp(alpha + D_s - D_i) <= 1
  {
    const double Di = sh.Dl[lane];
    for (int sc = wave * kColsPerWave; sc < (wave + 1) * kColsPerWave; ++sc) {
      const double v = sh.Am[sc * kTile + lane];
      sh.Am[sc * kTile + lane] = (lane > sc) ? fast_exp(v + sh.Dl[sc] - Di, sh.tab) : 0.0;
    }
  }
  __syncthreads();
  if (wave == 0) {
    // (4) forward substitution on w_i = exp(G_i - D_i), four rows per round
    const double Di = sh.Dl[lane];
    double acc = fast_exp(sh.LBl[lane] - Di, sh.tab), mine = 1.0;
    for (int s0 = 0; s0 < kTile; s0 += 4) {
      const double c0 = read_lane(acc, s0), c1 = read_lane(acc, s0 + 1);
      const double c2 = read_lane(acc, s0 + 2), c3 = read_lane(acc, s0 + 3);
      const double m10 = sh.Am[s0 * kTile + s0 + 1];
      const double m20 = sh.Am[s0 * kTile + s0 + 2], m21 = sh.Am[(s0 + 1) * kTile + s0 + 2];
      const double m30 = sh.Am[s0 * kTile + s0 + 3], m31 = sh.Am[(s0 + 1) * kTile + s0 + 3];
      const double m32 = sh.Am[(s0 + 2) * kTile + s0 + 3];
      const double w0 = c0;
      const double w1 = fma(m10, w0, c1);
      const double w2 = fma(m21, w1, fma(m20, w0, c2));
      const double w3 = fma(m32, w2, fma(m31, w1, fma(m30, w0, c3)));
      const int g = lane - s0;
      if (g == 0) mine = w0;
      if (g == 1) mine = w1;
      if (g == 2) mine = w2;
      if (g == 3) mine = w3;
      if (g > 3) {
        acc = fma(sh.Am[s0 * kTile + lane], w0, acc);
        acc = fma(sh.Am[(s0 + 1) * kTile + lane], w1, acc);
        acc = fma(sh.Am[(s0 + 2) * kTile + lane], w2, acc);
        acc = fma(sh.Am[(s0 + 3) * kTile + lane], w3, acc);
      }
    }
    sh.Wl[lane] = mine;
    if (i <= N) {
      const double Gi = Di + log(mine);
      G[i] = Gi;
      if (i < N) rec[i].w += Gi;
    }
  }
  __syncthreads();
  if (publish != nullptr && threadIdx.x == 0)
    __hip_atomic_store(publish, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  // (5) weighted payloads of the in-block terms: the term of column s in row i is
  // exp(D_i) * Am[s][i] * w_s; each wave sums its columns, wave 0 normalises by exp(G_i).
  {
    double Q[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) Q[q] = 0.0;
    for (int sc = wave * kColsPerWave; sc < (wave + 1) * kColsPerWave; ++sc) {
      const int j = blk * kTile + sc;
      if (valid && j < i) {
        const double coef = sh.Am[sc * kTile + lane] * sh.Wl[sc];
        const double4 r4 = rec[j];
        const double qv[3] = {r4.x, r4.y, r4.z};
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double t = pi[c] - qv[c];
          d2 = fma(t, t, d2);
          Q[c] = fma(coef, qv[c], Q[c]);
        }
        Q[D] = fma(coef, d2, Q[D]);
      }
    }
#pragma unroll
    for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = Q[q];
  }
  __syncthreads();
  if (wave == 0 && valid) {
    const double wi = sh.Wl[lane];
    const double bterm = fast_exp(sh.LBl[lane] - sh.Dl[lane], sh.tab);   // the earlier-column term of row i
#pragma unroll
    for (int q = 0; q <= D; ++q) {
      double v = bterm * sh.pbar[q][lane];
#pragma unroll
      for (int w = 0; w < kRecWaves; ++w) v += sh.pp[w][q][lane];
      av[(long long)q * npp + i] = v / wi;
    }
  }
  __syncthreads();
}

// Fills the column records {q_j, gamma_j} (G_j is added once row j is solved).
template <int D>
__device__ inline void init_columns(const RecMap<D>& mp, double4* __restrict__ rec, int N) {
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double q[D], gam;
    mp.col(j, q, gam);
    double4 r4;
    r4.x = q[0];
    r4.y = D > 1 ? q[D > 1 ? 1 : 0] : 0.0;
    r4.z = D > 2 ? q[D > 2 ? 2 : 0] : 0.0;
    r4.w = gam;
    rec[j] = r4;
  }
}

template <int D>
__device__ inline RecMap<D> rec_map(const RepDev& R, const double* ends, const double* link, int dir) {
  RecMap<D> mp;
  mp.a = ends + 2LL * D * R.part;
  mp.b = mp.a + (long long)D * R.npp;
  mp.lk = link + R.part;
  mp.N = R.n; mp.npp = R.npp; mp.dir = dir; mp.blink = R.beta;
  return mp;
}

__device__ inline int xi_mode(double xi) { return xi == 1.0 ? kXiOne : (xi == 0.0 ? kXiZero : kXiGen); }

// One workgroup per replica and direction (batched replicas fill the machine).
template <int D>
__global__ __launch_bounds__(kRecThreads) void k_recursion(const RepDev* __restrict__ reps,
                                                           const double* __restrict__ ends,
                                                           const double* __restrict__ link,
                                                           double* __restrict__ gf, double* __restrict__ gb,
                                                           double4* __restrict__ colrec,
                                                           double* __restrict__ avg) {
  __shared__ RecShared<D> sh;
  const int rep = blockIdx.x >> 1, dir = blockIdx.x & 1;
  const RepDev& R = reps[rep];
  const int N = R.n;
  const RecMap<D> mp = rec_map<D>(R, ends, link, dir);
  double* G = (dir == 0 ? gf : gb) + R.part;
  double4* rec = colrec + 2LL * R.part + (long long)dir * R.npp;
  double* av = avg + 2LL * (D + 1) * R.part + (long long)dir * (D + 1) * R.npp;
  const double bc = R.beta * R.c, lnxi = R.lnxi;
  const int xm = xi_mode(R.xi);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = (N + 1 + kTile - 1) / kTile;   // rows 0..N

  if (threadIdx.x < kExpTable) sh.tab[threadIdx.x] = exp_table_entry(threadIdx.x);
  init_columns<D>(mp, rec, N);
  __syncthreads();

  for (int blk = 0; blk < nblk; ++blk) {
    const int i = blk * kTile + lane;
    const bool valid = (i >= 1 && i <= N);
    double pi[D], rho = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) pi[c] = 0.0;
    if (valid) mp.row(i, pi, rho);
    const RowCtx rc{i, rho, bc, lnxi};
    const int jend = blk * kTile;

    // (0) reference: largest term among the previous block's columns
    double Rref = 0.0;
    if (jend > 0) {
      double mx = -INFINITY;
      if (valid) {
        const int j0 = jend - kTile + wave * kColsPerWave;
        if (xm == kXiOne) mx = max_term<D, kXiOne>(rc, pi, rec, j0, kColsPerWave);
        else if (xm == kXiZero) mx = max_term<D, kXiZero>(rc, pi, rec, j0, kColsPerWave);
        else mx = max_term<D, kXiGen>(rc, pi, rec, j0, kColsPerWave);
      }
      sh.pm[wave][lane] = mx;
      __syncthreads();
      mx = sh.pm[0][lane];
#pragma unroll
      for (int w = 1; w < kRecWaves; ++w) mx = fmax(mx, sh.pm[w][lane]);
      Rref = (mx > -INFINITY) ? mx : 0.0;
      __syncthreads();
    }

    // (1) earlier columns j < blk*64, split over the waves
    double m = -1e300, s = 0.0, P[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) P[q] = 0.0;
    if (valid && jend > 0) {
      const int per = (jend + kRecWaves - 1) / kRecWaves;
      const int ja = min(jend, wave * per), jb = min(jend, ja + per);
      if (xm == kXiOne) bulk_rows<D, kXiOne>(rc, pi, Rref, rec, ja, jb, sh.tab, m, s, P);
      else if (xm == kXiZero) bulk_rows<D, kXiZero>(rc, pi, Rref, rec, ja, jb, sh.tab, m, s, P);
      else bulk_rows<D, kXiGen>(rc, pi, Rref, rec, ja, jb, sh.tab, m, s, P);
    }
    sh.pm[wave][lane] = m;
    sh.ps[wave][lane] = s;
#pragma unroll
    for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = P[q];
    solve_block<D>(sh, blk, N, pi, rho, valid, bc, lnxi, rec, G, av, R.npp, nullptr, 0);
  }
}

// ------------------------------------------------------- cooperative schedule (one large replica)
//
// One chain workgroup per replica and direction runs the blocks in order; H helper workgroups
// per chain add up, for future row blocks, the contributions of every column panel the chain has
// already finished (panel c = the columns of block c), so the chain itself only adds the panel
// it has just produced.  Helper h owns row blocks 2+h, 2+h+H, ...; for its block b it folds in
// panels 0..b-2 as they are published and then publishes the partial sums of block b.  Flags
// hold the epoch of the launch that set them, so they never need clearing.  All workgroups are
// launched cooperatively (co-resident), every wait depends only on work earlier in the chain,
// and every wait gives up after a bounded number of polls (raising an error word) instead of
// hanging.

constexpr long long kSpinLimit = 1LL << 24;

// One thread waits until *flag == epoch; false (and *err set) on timeout or when another wait
// already failed.
__device__ inline bool wait_epoch(const int* flag, int epoch, int* err) {
  long long n = 0;
  while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
    if (++n > kSpinLimit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

// Folds columns [j0, j0 + n) into the running log-sum-exp (m, s, P): one rescale per slice.
template <int D, int XM>
__device__ inline void slice_fold(const RowCtx& rc, const double (&pi)[D], const double4* __restrict__ rec, int j0,
                                  int n, const double* tab, double& m, double& s, double (&P)[D + 1]) {
  double t[kColsPerWave], d2[kColsPerWave];
  double4 r[kColsPerWave];
  double mt = -INFINITY;
#pragma unroll
  for (int u = 0; u < kColsPerWave; ++u) {
    r[u] = rec[j0 + min(u, n - 1)];
    t[u] = term_of<D, XM>(rc, pi, r[u], j0 + u, d2[u]);
    if (u >= n) t[u] = -INFINITY;
    mt = fmax(mt, t[u]);
  }
  const double M = fmax(m, mt);
  const double f = fast_exp(m - M, tab);
  s *= f;
#pragma unroll
  for (int q = 0; q <= D; ++q) P[q] *= f;
  m = M;
#pragma unroll
  for (int u = 0; u < kColsPerWave; ++u) {
    const double e = fast_exp(t[u] - M, tab);
    s += e;
    const double qv[3] = {r[u].x, r[u].y, r[u].z};
#pragma unroll
    for (int c = 0; c < D; ++c) P[c] = fma(e, qv[c], P[c]);
    P[D] = fma(e, d2[u], P[D]);
  }
}

template <int D>
__device__ inline void fold_any(int xm, const RowCtx& rc, const double (&pi)[D], const double4* rec, int j0, int n,
                                const double* tab, double& m, double& s, double (&P)[D + 1]) {
  if (xm == kXiOne) slice_fold<D, kXiOne>(rc, pi, rec, j0, n, tab, m, s, P);
  else if (xm == kXiZero) slice_fold<D, kXiZero>(rc, pi, rec, j0, n, tab, m, s, P);
  else slice_fold<D, kXiGen>(rc, pi, rec, j0, n, tab, m, s, P);
}

template <int D>
__global__ __launch_bounds__(kRecThreads) void k_recursion_coop(const RepDev* __restrict__ reps,
                                                                const double* __restrict__ ends,
                                                                const double* __restrict__ link,
                                                                double* __restrict__ gf, double* __restrict__ gb,
                                                                double4* __restrict__ colrec,
                                                                double* __restrict__ avg, int* __restrict__ flags,
                                                                double* __restrict__ partial, int* __restrict__ err,
                                                                int nchains, int H, int epoch) {
  __shared__ RecShared<D> sh;
  const bool is_chain = (int)blockIdx.x < nchains;
  const int chain = is_chain ? (int)blockIdx.x : ((int)blockIdx.x - nchains) % nchains;
  const int h = is_chain ? -1 : ((int)blockIdx.x - nchains) / nchains;
  const int rep = chain >> 1, dir = chain & 1;
  const RepDev& R = reps[rep];
  const int N = R.n;
  const RecMap<D> mp = rec_map<D>(R, ends, link, dir);
  double* G = (dir == 0 ? gf : gb) + R.part;
  double4* rec = colrec + 2LL * R.part + (long long)dir * R.npp;
  double* av = avg + 2LL * (D + 1) * R.part + (long long)dir * (D + 1) * R.npp;
  int* panel_ready = flags + 4LL * R.part + (long long)(2 * dir) * R.npp;
  int* part_ready = flags + 4LL * R.part + (long long)(2 * dir + 1) * R.npp;
  double* pt = partial + 2LL * (D + 3) * R.part + (long long)dir * (D + 3) * R.npp;  // [D+3][npp]: m, s, P
  const double bc = R.beta * R.c, lnxi = R.lnxi;
  const int xm = xi_mode(R.xi);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = (N + 1 + kTile - 1) / kTile;
  const long long npp = R.npp;
  if (threadIdx.x < kExpTable) sh.tab[threadIdx.x] = exp_table_entry(threadIdx.x);

  if (is_chain) {
    init_columns<D>(mp, rec, N);
    __syncthreads();
    for (int blk = 0; blk < nblk; ++blk) {
      const int i = blk * kTile + lane;
      const bool valid = (i >= 1 && i <= N);
      double pi[D], rho = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) pi[c] = 0.0;
      if (valid) mp.row(i, pi, rho);
      const RowCtx rc{i, rho, bc, lnxi};
      double m = -1e300, s = 0.0, P[D + 1];
#pragma unroll
      for (int q = 0; q <= D; ++q) P[q] = 0.0;
      // the panel just finished (columns of block blk-1), one 8-column slice per wave
      if (blk >= 1 && valid) fold_any<D>(xm, rc, pi, rec, (blk - 1) * kTile + wave * kColsPerWave, kColsPerWave,
                                         sh.tab, m, s, P);
      // panels 0..blk-2 from the helper that owns this block
      if (blk >= 2) {
        if (threadIdx.x == 0) sh.flag = wait_epoch(part_ready + blk, epoch, err) ? 1 : 0;
        __syncthreads();
        if (wave == 0 && valid && sh.flag) {
          const double mh = pt[i], shs = pt[npp + i];
          if (shs > 0.0) {
            const double M = fmax(m, mh);
            const double f0 = exp(m - M), f1 = exp(mh - M);
            s = s * f0 + shs * f1;
#pragma unroll
            for (int q = 0; q <= D; ++q) P[q] = P[q] * f0 + pt[(2 + q) * npp + i] * f1;
            m = M;
          }
        }
      }
      sh.pm[wave][lane] = m;
      sh.ps[wave][lane] = s;
#pragma unroll
      for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = P[q];
      solve_block<D>(sh, blk, N, pi, rho, valid, bc, lnxi, rec, G, av, R.npp, panel_ready + blk, epoch);
    }
    return;
  }

  // helper h: row blocks 2+h, 2+h+H, ...
  int ready = -1;   // panels 0..ready are known to be published
  for (int blk = 2 + h; blk < nblk; blk += H) {
    const int i = blk * kTile + lane;
    const bool valid = (i >= 1 && i <= N);
    double pi[D], rho = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) pi[c] = 0.0;
    if (valid) mp.row(i, pi, rho);
    const RowCtx rc{i, rho, bc, lnxi};
    double m = -1e300, s = 0.0, P[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) P[q] = 0.0;
    for (int c = 0; c <= blk - 2; ++c) {
      if (c > ready) {
        if (threadIdx.x == 0) {
          int r = wait_epoch(panel_ready + c, epoch, err) ? c : -2;
          // look ahead: later panels that are already out
          if (r >= 0)
            while (r + 1 <= blk - 2 &&
                   __hip_atomic_load(panel_ready + r + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == epoch)
              ++r;
          sh.flag = r;
        }
        __syncthreads();
        ready = sh.flag;
        __syncthreads();
        if (ready < 0) return;   // a wait failed: the error word is raised, stop this helper
      }
      if (valid) fold_any<D>(xm, rc, pi, rec, c * kTile + wave * kColsPerWave, kColsPerWave, sh.tab, m, s, P);
    }
    sh.pm[wave][lane] = m;
    sh.ps[wave][lane] = s;
#pragma unroll
    for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = P[q];
    __syncthreads();
    if (wave == 0 && valid) {
      double M = sh.pm[0][lane];
#pragma unroll
      for (int w = 1; w < kRecWaves; ++w) M = fmax(M, sh.pm[w][lane]);
      double S = 0.0, PS[D + 1];
#pragma unroll
      for (int q = 0; q <= D; ++q) PS[q] = 0.0;
#pragma unroll
      for (int w = 0; w < kRecWaves; ++w) {
        const double f = sh.ps[w][lane] > 0.0 ? exp(sh.pm[w][lane] - M) : 0.0;
        S = fma(sh.ps[w][lane], f, S);
#pragma unroll
        for (int q = 0; q <= D; ++q) PS[q] = fma(sh.pp[w][q][lane], f, PS[q]);
      }
      pt[i] = M;
      pt[npp + i] = S;
#pragma unroll
      for (int q = 0; q <= D; ++q) pt[(2 + q) * npp + i] = PS[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(part_ready + blk, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_recursion(const Dims& d, const DevPtrs& w, hipStream_t s) {
  dim3 grid((unsigned)(2 * d.R)), block(kRecThreads);
#define L(DD) hipLaunchKernelGGL(k_recursion<DD>, grid, block, 0, s, w.reps, w.ends, w.link, w.gf, w.gb, w.colrec, w.avg)
  switch (d.D) {
    case 1: L(1); break;
    case 2: L(2); break;
    case 3: L(3); break;
    default: return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

template <int D>
static hipError_t launch_coop_d(const Dims& d, const DevPtrs& w, int H, int epoch, hipStream_t s) {
  int nchains = 2 * d.R;
  dim3 grid((unsigned)(nchains * (1 + H))), block(kRecThreads);
  const RepDev* reps = w.reps;
  const double* ends = w.ends;
  const double* link = w.link;
  double* gf = w.gf;
  double* gb = w.gb;
  double4* colrec = w.colrec;
  double* avg = w.avg;
  int* flags = w.flags;
  double* partial = w.partial;
  int* err = w.err;
  void* args[] = {(void*)&reps, (void*)&ends, (void*)&link, (void*)&gf, (void*)&gb, (void*)&colrec, (void*)&avg,
                  (void*)&flags, (void*)&partial, (void*)&err, (void*)&nchains, (void*)&H, (void*)&epoch};
  return hipLaunchCooperativeKernel((const void*)k_recursion_coop<D>, grid, block, args, 0, s);
}

hipError_t launch_recursion_coop(const Dims& d, const DevPtrs& w, int helpers, int epoch, hipStream_t s) {
  switch (d.D) {
    case 1: return launch_coop_d<1>(d, w, helpers, epoch, s);
    case 2: return launch_coop_d<2>(d, w, helpers, epoch, s);
    case 3: return launch_coop_d<3>(d, w, helpers, epoch, s);
    default: return hipErrorInvalidValue;
  }
}

int recursion_coop_max_blocks_per_cu(int D) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (D == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_recursion_coop<1>, kRecThreads, 0);
  if (D == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_recursion_coop<2>, kRecThreads, 0);
  if (D == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_recursion_coop<3>, kRecThreads, 0);
  return e == hipSuccess ? n : 0;
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

// Per particle l (0-based, paper index L = l+1), from the recursion outputs:
//   sum_{l'<=L} Pr[L -> l'] = exp(G^f_L + G^b_{N-L} - G^f_N - beta link_L) =: w_end   (forward row L)
//   sum_{l>=L} Pr[l -> L]  = exp(G^b_{N+1-L} + G^f_{L-1} - G^f_N - beta link_{L-1}) =: w_start
//                                                                          (backward row N+1-L)
// and the weighted averages of the forward row (a_{l'}, |b_L - a_{l'}|^2) and of the backward
// row (b_l).  With the Pr[L -> L+1] and Pr[L-1 -> L] terms of Eq. 13 added, Eqs. 15-16 give
//   F(bead P of L) += -kappa (rowsum (2 b_L - r_L^{P-1}) - sum_{l'} Pr[L->l'] a_{l'})
//   F(bead 1 of L) += -kappa (colsum (2 a_L - r_L^2)     - sum_{l}  Pr[l->L] b_l)
// and the expected spring energy gets w_end c avg|b_L - a_{l'}|^2 + Pr[L -> L+1] link_L.
template <int D>
__global__ __launch_bounds__(256) void k_probs_reduce(const RepDev* __restrict__ reps, const int4* __restrict__ work,
                                                      const double* __restrict__ x, double* __restrict__ f,
                                                      const double* __restrict__ ends, const double* __restrict__ link,
                                                      const double* __restrict__ gf, const double* __restrict__ gb,
                                                      const double* __restrict__ avg,
                                                      double* __restrict__ reducepart, int P) {
  __shared__ double lds[2 * 4];
  const int4 wk = work[blockIdx.x];
  const RepDev& R = reps[wk.x];
  const int N = R.n;
  const int l = wk.y + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (l < N) {
    const long long npp = R.npp;
    const double* a = ends + 2LL * D * R.part;
    const double* b = a + (long long)D * npp;
    const double* lk = link + R.part;
    const double* g_f = gf + R.part;
    const double* g_b = gb + R.part;
    const double* avf = avg + 2LL * (D + 1) * R.part;
    const double* avb = avf + (long long)(D + 1) * npp;
    const double w_end = exp(g_f[l + 1] + g_b[N - 1 - l] - g_f[N] - R.beta * lk[l]);
    const double w_start = exp(g_b[N - l] + g_f[l] - g_f[N] - (l > 0 ? R.beta * lk[l - 1] : 0.0));
    const double pn = prob_next(l, N, lk, g_f, g_b, R.beta);                          // Pr[L -> L+1]
    const double pp = (l > 0) ? prob_next(l - 1, N, lk, g_f, g_b, R.beta) : 0.0;        // Pr[L-1 -> L]
    const double rs = w_end + pn, cs = w_start + pp;
    const double kap = R.kappa;
    double* fr = f + R.dof;
    const double* xr = x + R.dof;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double ra = w_end * avf[(long long)c * npp + (l + 1)];
      double cb = w_start * avb[(long long)c * npp + (N - l)];
      if (pn != 0.0) ra = fma(pn, a[(long long)c * npp + l + 1], ra);
      if (pp != 0.0) cb = fma(pp, b[(long long)c * npp + l - 1], cb);
      const double al = a[(long long)c * npp + l], bl = b[(long long)c * npp + l];
      const double rP1 = xr[((long long)c * P + (P - 2)) * N + l];   // r_L^{P-1}
      const double r2 = xr[((long long)c * P + 1) * N + l];           // r_L^2
      fr[((long long)c * P + (P - 1)) * N + l] += -kap * (rs * (2.0 * bl - rP1) - ra);
      fr[((long long)c * P + 0) * N + l] += -kap * (cs * (2.0 * al - r2) - cb);
    }
    acc[0] = w_end * R.c * avf[(long long)D * npp + (l + 1)] + pn * lk[l];
    acc[1] = 0.0;
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    reducepart[2LL * blockIdx.x + 0] = acc[0];
    reducepart[2LL * blockIdx.x + 1] = acc[1];
  }
}

hipError_t launch_probs_reduce(const Dims& d, const DevPtrs& w, hipStream_t s) {
  if (d.nreducewg == 0) return hipSuccess;
  dim3 grid((unsigned)d.nreducewg), block(256);
#define L(DD) hipLaunchKernelGGL(k_probs_reduce<DD>, grid, block, 0, s, w.reps, w.reducework, w.x, w.f, w.ends, \
                                 w.link, w.gf, w.gb, w.avg, w.reducepart, d.P)
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
  (void)d;
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
