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
// Two species (particles 1..na and na+1..N).  The exchange sum factorises over species, so a
// block [u,v] with u <= na < v never occurs and each 1/n factor counts within its species.  In
// the recursion this is a boundary bnd (forward na, backward N - na): rows i > bnd only take
// columns j >= bnd, the forward rho_i uses log(i - bnd) and the backward gamma_j uses
// log(bnd - j) for j < bnd.  The link across the boundary is set to 0 (no allowed block holds
// it), and Pr[na -> na+1] = 0.  With one species bnd = N forward and 0 backward: no mask.
//
// Probabilities without a G matrix.  Eq. 12 in this notation is a recursion term times a
// factor of its row: Pr[n -> m+1] = exp(alpha^f_{n,m} + G^f_m) exp(G^b_{N-n} - G^f_N - beta link_n)
// (forward row n) and Pr[l -> u] = exp(alpha^b_{i,j} + G^b_j) exp(G^f_{u-1} - G^f_N - beta
// link_{u-1}) (backward row i = N+1-u, column j = N-l).  So the row sums that Eq. 16 needs
// (sum_{l'} Pr[l->l'] a_{l'}, and sum Pr close for the energy) are weighted averages over the
// terms of forward row l, and the column sums of Eq. 15 (sum_l Pr[l->u] b_l) weighted averages
// over backward row N+1-u.  Each recursion row therefore also accumulates the term-weighted
// average of its column points q_j and of |p_i - q_j|^2 + lam_{i-1} - lam_j, where lam is the
// prefix of link_l / c: c times that payload is the cycle energy E^{[j+1,i]} minus its internal
// energies (its closing term plus the links inside it), so the expected spring energy S of the
// estimators is a sum of non-negative terms, each as accurate as its probability.  A per-particle
// pass applies the row factors, adds Pr[l -> l+1] = -expm1(G^f_l + G^b_{N-l} - G^f_N - beta
// link_l) (Eq. 13) and forms the end-bead forces of Eqs. 15-16.  The N^2/2 probabilities are never
// stored or recomputed.  (Eq. 13 in that form is the difference of potentials of size up to
// beta sum link, so a small Pr[l -> l+1] carries an absolute error of their rounding; the forces
// take it at that absolute size, while S never multiplies it by a link energy.)
//
// Expanded terms.  For d <= 2 a completed column record also holds, in its third slot, the column
// constant B_j = gamma_j + G_j - beta c |q_j|^2 - j log xi (log xi taken as 0 for xi = 1 and
// for xi = 0, whose terms are formed directly), so that the earlier-column sums form a term as
// A_i + B_j + 2 beta c p_i.q_j with the row constant A_i = rho_i - beta c |p_i|^2 + (i-1) log xi:
// three operations instead of six (the xi power costs nothing).  The expansion rounds at the
// size of beta c (|p_i|^2 + |q_j|^2) instead of beta c |p_i - q_j|^2, an absolute error of a few
// 1e-13 in the exponent for the trapped systems here, far below the parity bounds.
//
// Recursion schedule (one workgroup per replica and direction, four wavefronts).  Rows are
// processed in blocks of 64 (lane = row).  For a block: (0) a reference R_i = the largest term of
// the previous block's columns (a lower bound of the row's largest earlier term); (1) the four
// waves sum exp(term - R_i) and its weighted payloads over all earlier columns (if a term ever
// exceeds R_i by more than the double range, that wave redoes its columns with a running
// maximum); (2) wave 0 runs a max-plus pass over the in-block columns giving each row a scale D_i
// with every scaled coefficient <= 1; (3) all waves evaluate exp(alpha + D_j - D_i); (4) wave 0
// solves the scaled in-block triangular system by forward substitution with lane broadcasts,
// four rows per round; G_i = D_i + log w_i; (5) the in-block weighted payloads.  The scaled
// unknowns satisfy 1 <= w_i <= 2^64, so nothing overflows whatever the range of the weights.
#include <type_traits>

#include "pimd_internal.h"
#include "device_util.h"
#include "fast_exp.h"

namespace pimd {

// Row and column data of the generic recursion G_i = log sum_{j<i} exp(alpha_{i,j} + G_j).
template <int D>
struct RecMap {
  const double* a; const double* b; const double* lk;
  int N, npp, dir;
  int bnd;   // species boundary in this direction's row numbering
  double beta;
  // end point p_i and the link value entering rho_i, for 1 <= i <= N
  __device__ inline void row_load(int i, double (&pt)[D], double& lv) const {
    if (dir == 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) pt[c] = b[(long long)c * npp + (i - 1)];
      lv = lk[i - 1];
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) pt[c] = a[(long long)c * npp + (N - i)];
      lv = (i < N) ? lk[N - i - 1] : 0.0;
    }
  }
  __device__ inline double row_rho(int i, double lv) const {
    return dir == 0 ? beta * lv - fast_log((double)(i > bnd ? i - bnd : i)) : beta * lv;
  }
  // column point q_j, for 0 <= j <= N-1
  __device__ inline void col_load(int j, double (&q)[D]) const {
    if (dir == 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) q[c] = a[(long long)c * npp + j];
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) q[c] = b[(long long)c * npp + (N - j - 1)];
    }
  }
  __device__ inline double col_gamma(int j) const {
    return dir == 0 ? 0.0 : -fast_log((double)(j < bnd ? bnd - j : N - j));
  }
};

// Waves per recursion workgroup: the cooperative chain kernel uses eight (its block latency is
// the critical path); the batched kernel four by default (half the register file and less LDS per
// CU, so the pair kernel's workgroups can run beside it on the same compute units) or eight when
// its workgroups have compute units to spare (few replicas: the chains are the critical path).
constexpr int kCoopWaves = 8;
constexpr int kCoopCols = kTile / kCoopWaves;

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
  double lrow;   // lam_{i-1}: the links of a cycle [j+1, i] are c (lrow - lam_j)
};

// term t_{i,j} = alpha_{i,j} + G_j and |p_i - q_j|^2 for column record r4 = {q_j, gamma_j + G_j}.
template <int D, int XM>
__device__ inline double term_of(const RowCtx& rc, const double (&pi)[D], const double4& r4, int j, double& d2) {
  const double qv[3] = {r4.x, r4.y, r4.z};
  d2 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) { const double t = pi[c] - qv[c]; d2 = fma(t, t, d2); }
  if constexpr (XM == kXiOne) return fma(-rc.bc, d2, rc.rowc + r4.w);
  else return fma(-rc.bc, d2, rc.rowc + r4.w) + xi_term<XM>(rc.i - 1 - j, rc.lnxi);
}

// Sum of exp(t_j - R) over columns [ja, jb) with payload sums (q_j, and with SP the cycle's
// spring payload |p_i - q_j|^2 + lam_{i-1} - lam_j, which only the estimators need), two
// interleaved accumulator sets, records prefetched one group ahead.  Whole pairs of four-column
// groups run without masks; the at most seven columns left over run in masked groups.
template <int D, int XM, bool SP>
__device__ inline void bulk_fixed(const RowCtx& rc, const double (&pi)[D], double R, const double4* __restrict__ rec,
                                  const double* __restrict__ lam, int ja, int jb, const double* tab, double& s_out,
                                  double (&P)[D + 1]) {
  // expanded terms (records carry B_j) unless the spring payload needs |p_i - q_j|^2 itself
  constexpr bool kExpand = D <= 2 && XM != kXiZero && !SP;
  double P2[D], Arow = 0.0;   // 2 beta c p_i and A_i - R
  if constexpr (kExpand) {
    double p2 = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      P2[c] = 2.0 * rc.bc * pi[c];
      p2 = fma(pi[c], pi[c], p2);
    }
    Arow = fma(-rc.bc, p2, rc.rowc - R);
    if constexpr (XM == kXiGen) Arow = fma((double)(rc.i - 1), rc.lnxi, Arow);
  }
  double s[2] = {0.0, 0.0}, pq[2][D + 1];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q <= D; ++q) pq[h][q] = 0.0;
  auto ld = [&](double4 (&dst)[4], double (&dl)[4], int j0, auto clamped) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = decltype(clamped)::value ? min(j0 + u, jb - 1) : j0 + u;
      dst[u] = rec[j];
      dl[u] = SP ? lam[j] : 0.0;
    }
  };
  // the reference enters the row constant once instead of every term
  const RowCtx rr{rc.i, rc.rowc - R, rc.bc, rc.lnxi, rc.lrow};
  auto group = [&](const double4 (&g)[4], const double (&gl)[4], int j0, auto masked) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u;
      double d2 = 0.0, t;   // t_{i,j} - R
      if constexpr (kExpand) {
        const double qv[3] = {g[u].x, g[u].y, g[u].z};
        t = Arow + g[u].z;
#pragma unroll
        for (int c = 0; c < D; ++c) t = fma(P2[c], qv[c], t);
      } else {
        t = term_of<D, XM>(rr, pi, g[u], j, d2);
      }
      if constexpr (decltype(masked)::value) {
        if (j >= jb) t = -INFINITY;
      }
      const double e = fast_exp_finite(t, tab);
      const int h = u & 1;
      s[h] += e;
      const double qv[3] = {g[u].x, g[u].y, g[u].z};
#pragma unroll
      for (int c = 0; c < D; ++c) pq[h][c] = fma(e, qv[c], pq[h][c]);
      if constexpr (SP) pq[h][D] = fma(e, d2 + (rr.lrow - gl[u]), pq[h][D]);
    }
  };
  // two record buffers in turn, each loaded one group ahead (no register copies between groups)
  double4 bufA[4], bufB[4];
  double lamA[4], lamB[4];
  const int jf = ja + (jb - ja) / 8 * 8;
  if (ja < jf) ld(bufA, lamA, ja, std::false_type{});
  for (int j0 = ja; j0 < jf; j0 += 8) {
    ld(bufB, lamB, j0 + 4, std::false_type{});
    group(bufA, lamA, j0, std::false_type{});
    if (j0 + 8 < jf) ld(bufA, lamA, j0 + 8, std::false_type{});
    group(bufB, lamB, j0 + 4, std::false_type{});
  }
  for (int j0 = jf; j0 < jb; j0 += 4) {
    ld(bufA, lamA, j0, std::true_type{});
    group(bufA, lamA, j0, std::true_type{});
  }
  s_out = s[0] + s[1];
#pragma unroll
  for (int q = 0; q <= D; ++q) P[q] = pq[0][q] + pq[1][q];
}

// Same sums with a running maximum m (result = exp(m) * (s, P)); used when a term exceeds the
// fixed reference by more than the double range.
template <int D, int XM, bool SP>
__device__ inline void bulk_online(const RowCtx& rc, const double (&pi)[D], const double4* __restrict__ rec,
                                   const double* __restrict__ lam, int ja, int jb, const double* tab, double& m_out,
                                   double& s_out, double (&P)[D + 1]) {
  double m = -1e300, s = 0.0, pq[D + 1];
#pragma unroll
  for (int q = 0; q <= D; ++q) pq[q] = 0.0;
  for (int j = ja; j < jb; ++j) {
    const double4 r4 = rec[j];
    double d2;
    const double t = term_of<D, XM>(rc, pi, r4, j, d2);
    const double v = SP ? d2 + (rc.lrow - lam[j]) : 0.0;
    const double dl = t - m;
    const double e = fast_exp(-fabs(dl), tab);
    const double qv[3] = {r4.x, r4.y, r4.z};
    if (dl > 0.0) {
      s = fma(s, e, 1.0);
#pragma unroll
      for (int c = 0; c < D; ++c) pq[c] = fma(pq[c], e, qv[c]);
      pq[D] = fma(pq[D], e, v);
      m = t;
    } else {
      s += e;
#pragma unroll
      for (int c = 0; c < D; ++c) pq[c] = fma(e, qv[c], pq[c]);
      pq[D] = fma(e, v, pq[D]);
    }
  }
  m_out = m;
  s_out = s;
#pragma unroll
  for (int q = 0; q <= D; ++q) P[q] = pq[q];
}

template <int D, int XM, bool SP>
__device__ inline void bulk_rows(const RowCtx& rc, const double (&pi)[D], double R, const double4* __restrict__ rec,
                                 const double* __restrict__ lam, int ja, int jb, const double* tab, double& m,
                                 double& s, double (&P)[D + 1]) {
  bulk_fixed<D, XM, SP>(rc, pi, R, rec, lam, ja, jb, tab, s, P);
  m = R;
  bool bad = !isfinite(s);
#pragma unroll
  for (int q = 0; q <= D; ++q) bad = bad || !isfinite(P[q]);
  if (__any(bad)) bulk_online<D, XM, SP>(rc, pi, rec, lam, ja, jb, tab, m, s, P);
}

// Step (0) of a block for one wave: the largest term over its NC columns j0.. of the previous
// block (records cp, in LDS), columns below jlo excluded.  All records are read before the first
// term, so the reads overlap instead of each waiting out its own latency.
template <int D, int XM, int NC>
__device__ inline double ref_max(const RowCtx& rc, const double (&pi)[D], const double4* cp, int j0, int jlo) {
  double mx = -INFINITY;
  constexpr int kHalf = NC > 8 ? 8 : (NC > 4 ? 4 : NC);
#pragma unroll
  for (int u0 = 0; u0 < NC; u0 += kHalf) {
    double4 r4[kHalf];
#pragma unroll
    for (int u = 0; u < kHalf; ++u) r4[u] = cp[u0 + u];
#pragma unroll
    for (int u = 0; u < kHalf; ++u) {
      double d2;
      const double t = term_of<D, XM>(rc, pi, r4[u], j0 + u0 + u, d2);
      mx = (j0 + u0 + u < jlo) ? mx : fmax(mx, t);
    }
  }
  return mx;
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

// LDS of one recursion workgroup; NR > 0 also keeps the column records of the first NR columns
// (every column of a replica with N <= NR), which the earlier-column sums then read from LDS.
template <int D, int W, int NR = 0>
struct RecShared {
  static constexpr int kWaves = W;
  static constexpr int kCols = kTile / W;   // in-block columns per wave
  static constexpr int kLdsRecs = NR;
  double tab[kExpTable];
  double Am[kTile * kTile];             // in-block coefficients, column-major: Am[col * 64 + row]
  double pm[W][kTile], ps[W][kTile];
  double pp[W][D + 1][kTile];   // per-wave sums over earlier columns: exp(pm) (ps, pp)
  double qp[W][D + 1][kTile];   // per-wave weighted payloads of the in-block columns
  double Dl[kTile], Wl[kTile];          // row scales D_i and scaled unknowns w_i of the block
  double4 col[2][kTile];                // column records {q_j, gamma_j (+ G_j once solved)}: this block, previous
  double4 recs[NR > 0 ? NR : 1];        // completed column records 0..NR-1 (NR > 0)
};

// What wave 0 keeps in registers from a block's solve until it writes the block's row averages
// (at the start of the next block, or after the last one).
template <int D>
struct RowCarry {
  int i;
  bool valid;
  double w, bterm, pb[D + 1];
};

template <int D, class SH>
__device__ inline void write_avg(const SH& sh, const RowCarry<D>& cy, double* __restrict__ av,
                                 long long npp) {
  if (!cy.valid) return;
  const int lane = threadIdx.x & 63;
  const double inv = 1.0 / cy.w;
#pragma unroll
  for (int q = 0; q <= D; ++q) {
    double v = cy.bterm * cy.pb[q];
#pragma unroll
    for (int w = 0; w < SH::kWaves; ++w) v += sh.qp[w][q][lane];
    av[(long long)q * npp + cy.i] = v * inv;
  }
}

// (2a) in-block coefficients alpha_{i,j} (without G_j) from the staged column records; each wave
// fills its columns.  Blocks across the species boundary are masked (-inf).
template <int D, class SH>
__device__ inline void inblock_alpha(SH& sh, double* __restrict__ Am, int cur, int blk, int i, const double (&pi)[D],
                                     double rho, bool valid, double bc, double lnxi, int bnd) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  // every record is read before the first store: the compiler cannot tell that the stores to Am
  // miss the records, and would otherwise wait out each load's latency in turn
  double4 r4[SH::kCols];
#pragma unroll
  for (int u = 0; u < SH::kCols; ++u) r4[u] = sh.col[cur][wave * SH::kCols + u];
  double v[SH::kCols];
#pragma unroll
  for (int u = 0; u < SH::kCols; ++u) {
    const int j = blk * kTile + wave * SH::kCols + u;
    const double qv[3] = {r4[u].x, r4[u].y, r4[u].z};
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) { const double t = pi[c] - qv[c]; d2 = fma(t, t, d2); }
    const double a = xi_pow_log(i - 1 - j, lnxi) + rho + r4[u].w - bc * d2;
    v[u] = (valid && j < i && (i <= bnd || j >= bnd)) ? a : -INFINITY;
  }
#pragma unroll
  for (int u = 0; u < SH::kCols; ++u) Am[(wave * SH::kCols + u) * kTile + lane] = v[u];
}


// Max-plus pass D_i = max(LB_i, max_{s<i} (alpha_{i,s} + D_s)) with each lane's row of alpha held
// in registers (alpha_{i,s} = -inf for s >= i).  Four rows per round, rows s0..s0+3 being one
// aligned group of four lanes: within the group each row's value becomes final in turn and is
// passed to the later rows of the group by a quad permutation (each lane uses its own row's
// coefficients), then the four finished values are read out once and every later row takes
// them, so at the end run_i = D_i.
__device__ inline double maxplus_regs(const double* __restrict__ Am, double run) {
  const int lane = threadIdx.x & 63;
  double a[kTile];
#pragma unroll
  for (int s = 0; s < kTile; ++s) a[s] = Am[s * kTile + lane];
#pragma unroll
  for (int s0 = 0; s0 < kTile; s0 += 4) {
    double c = run;   // final on lane s0 + k once columns s0..s0+k-1 are in
    c = fmax(c, a[s0] + quad_lane<0>(c));
    c = fmax(c, a[s0 + 1] + quad_lane<1>(c));
    c = fmax(c, a[s0 + 2] + quad_lane<2>(c));
    const double d0 = read_lane(c, s0), d1 = read_lane(c, s0 + 1);
    const double d2 = read_lane(c, s0 + 2), d3 = read_lane(c, s0 + 3);
    run = fmax(fmax(run, a[s0] + d0), a[s0 + 1] + d1);
    run = fmax(fmax(run, a[s0 + 2] + d2), a[s0 + 3] + d3);
  }
  return run;
}

// Forward substitution w_i = acc_i + sum_{s<i} c_{i,s} w_s with each lane's row of c held in
// registers (c_{i,s} = 0 for s >= i), four rows per round as in maxplus_regs: the group's rows are
// finished in turn through quad permutations, read out once, and every row takes them; the
// multiply-adds run in the same order for every row, so at the end acc_i = w_i.
__device__ inline double substitute_regs(const double* __restrict__ Am, double acc) {
  const int lane = threadIdx.x & 63;
  double c[kTile];
#pragma unroll
  for (int s = 0; s < kTile; ++s) c[s] = Am[s * kTile + lane];
#pragma unroll
  for (int s0 = 0; s0 < kTile; s0 += 4) {
    double v = acc;   // final on lane s0 + k once columns s0..s0+k-1 are in
    v = fma(c[s0], quad_lane<0>(v), v);
    v = fma(c[s0 + 1], quad_lane<1>(v), v);
    v = fma(c[s0 + 2], quad_lane<2>(v), v);
    const double w0 = read_lane(v, s0), w1 = read_lane(v, s0 + 1);
    const double w2 = read_lane(v, s0 + 2), w3 = read_lane(v, s0 + 3);
    acc = fma(c[s0], w0, acc);
    acc = fma(c[s0 + 1], w1, acc);
    acc = fma(c[s0 + 2], w2, acc);
    acc = fma(c[s0 + 3], w3, acc);
  }
  return acc;
}

// (3) scaled coefficients c_{i,s} = exp(alpha_{i,s} + D_s - D_i) of the strictly lower triangle,
// 63 entries per lane-row of work: pass k of wave w takes column s = 4w + k for rows s+1..63 and
// column 63-s for rows 64-s..63.  Each wave also zeroes the upper triangle of its own eight
// columns (the substitution reads whole rows).
template <int D, class SH>
__device__ inline void scaled_coefficients(SH& sh, double* __restrict__ Am) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  constexpr int K = kTile / 2 / SH::kWaves;
  // all loads first, then the exponentials (independent, so they interleave), then all stores
  double arg[K];
  int idx[K];
  bool act[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int s = wave * K + k;                          // 0..31
    const bool lower = lane > s;
    const int col = lower ? s : kTile - 1 - s;
    const int row = lower ? lane : kTile - s + lane;     // lanes 0..s-1 -> rows 64-s..63
    act[k] = lower || lane < s;
    idx[k] = act[k] ? col * kTile + row : 0;
    arg[k] = act[k] ? Am[idx[k]] + sh.Dl[col] - sh.Dl[row] : 0.0;
  }
  double e[K];
#pragma unroll
  for (int k = 0; k < K; ++k) e[k] = fast_exp(arg[k], sh.tab);
#pragma unroll
  for (int u = 0; u < SH::kCols; ++u) {
    const int sc = wave * SH::kCols + u;
    if (lane <= sc) Am[sc * kTile + lane] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (act[k]) Am[idx[k]] = e[k];
}

// G_i, the completed column record of row i (LDS and global), the next block's column records,
// the publish store and the carried row data; wave 0 only.
// Column constants of the expanded terms: beta c and the log xi that they fold in.
struct ColConst { double bc, lnxf; };

template <int D, class SH>
__device__ inline void finish_rows(SH& sh, int blk, int cur, int N, bool valid, double Di, double wi,
                                   double bterm, double4* __restrict__ rec, double* __restrict__ G,
                                   const double4& col_next, int* publish, int epoch, RowCarry<D>& cy,
                                   const ColConst& cc) {
  const int lane = threadIdx.x & 63;
  const int i = blk * kTile + lane;
  sh.Wl[lane] = wi;
  if (i <= N) {
    const double Gi = Di + fast_log(wi);
    G[i] = Gi;
    if (i < N) {
      double4 r4 = sh.col[cur][lane];
      r4.w += Gi;
      if constexpr (D <= 2) {   // B_i of the expanded terms
        double q2 = r4.x * r4.x;
        if (D > 1) q2 = fma(r4.y, r4.y, q2);
        r4.z = fma(-(double)i, cc.lnxf, fma(-cc.bc, q2, r4.w));
      }
      sh.col[cur][lane] = r4;
      rec[i] = r4;
      if constexpr (SH::kLdsRecs > 0) {
        if (i < SH::kLdsRecs) sh.recs[i] = r4;
      }
    }
  }
  sh.col[cur ^ 1][lane] = col_next;
  if (publish != nullptr && lane == 0) __hip_atomic_store(publish, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  cy.i = i;
  cy.valid = valid;
  cy.w = wi;
  cy.bterm = bterm;
}

// Row data that the pipelined schedule keeps for a block's deferred averages: w_i, the weight
// of the earlier columns and their normalised payloads (what RowCarry holds in wave 0), in two
// slots that alternate by block parity.
template <int D>
struct PipeRows {
  double w[2][kTile], bt[2][kTile], pb[2][D + 1][kTile];
};

// In-block weighted payloads of block `blkp` (coefficients Am, records sh.col[curp], unknowns
// sh.Wl, row data pi of that block): the term of column s in row i is exp(D_i) c_{i,s} w_s.  The
// waves w >= W0 split the 64 columns (W0 = 0: consecutive runs of kCols; otherwise with stride
// kWaves - W0) and store their sums in qp[w].
template <int D, int W0, bool SP, class SH>
__device__ inline void block_payloads(SH& sh, const double* __restrict__ Am, int curp, const double (&pi)[D],
                                      double lrow, const double* __restrict__ lamblk) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  double Q[D + 1];
#pragma unroll
  for (int q = 0; q <= D; ++q) Q[q] = 0.0;
  auto column = [&](int sc) {
    const double coef = Am[sc * kTile + lane] * sh.Wl[sc];
    const double4 r4 = sh.col[curp][sc];
    const double qv[3] = {r4.x, r4.y, r4.z};
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double t = pi[c] - qv[c];
      d2 = fma(t, t, d2);
      Q[c] = fma(coef, qv[c], Q[c]);
    }
    if constexpr (SP) Q[D] = fma(coef, d2 + (lrow - lamblk[sc]), Q[D]);
  };
  if constexpr (W0 == 0) {   // kCols consecutive columns per wave
#pragma unroll
    for (int u = 0; u < SH::kCols; ++u) column(wave * SH::kCols + u);
  } else {                   // waves W0.. take every (kWaves - W0)-th column
    constexpr int kStride = SH::kWaves - W0;
    constexpr int kMax = (kTile + kStride - 1) / kStride;
    const int k = wave - W0;
#pragma unroll
    for (int u = 0; u < kMax; ++u)
      if (k + kStride * u < kTile) column(k + kStride * u);
  }
#pragma unroll
  for (int q = 0; q <= D; ++q) sh.qp[wave][q][lane] = Q[q];
}

// Row averages of block `blkp` from the kept row data (slot `slot`) and the payload sums of
// waves w0..kWaves-1.
template <int D, int W0, class SH>
__device__ inline void write_avg_kept(const SH& sh, const PipeRows<D>& pr, int slot, int blkp, int N,
                                      double* __restrict__ av, long long npp) {
  const int lane = threadIdx.x & 63;
  const int i = blkp * kTile + lane;
  if (i < 1 || i > N) return;
  const double inv = 1.0 / pr.w[slot][lane];
#pragma unroll
  for (int q = 0; q <= D; ++q) {
    double v = pr.bt[slot][lane] * pr.pb[slot][q][lane];
#pragma unroll
    for (int w = W0; w < SH::kWaves; ++w) v += sh.qp[w][q][lane];
    av[(long long)q * npp + i] = v * inv;
  }
}

// Steps (2)-(5) of one block of 64 rows, entered once every wave has stored its partial sums
// over the earlier columns (pm/ps/pp, log-sum-exp form exp(m) (s, P)) and its in-block
// coefficients alpha (Am).  Wave 0 combines the partials into LB_i and runs the max-plus pass
// for the row scales D_i (every scaled coefficient <= 1, so 1 <= w_i <= 2^64); all waves form
// the scaled coefficients; wave 0 solves for w_i, writes G_i, completes the column records (LDS
// and global), stages the next block's records and publishes the block (release store of
// `epoch`, when `publish` is set).  Wave 1 runs `idle` while wave 0 combines and scales.
// Unpipelined (PIPE = false): wave 0 first writes the previous block's row averages, and after
// the solve all waves form this block's in-block payloads (qp).  Pipelined (PIPE = true, at
// least three waves): the payloads of the previous block (coefficients Am_prev, row data from
// prev_rows) are formed by waves 2.. while wave 0 combines and runs the max-plus pass, and wave 2
// writes that block's row averages while wave 0 substitutes, so neither sits on the chain; the
// caller alternates two coefficient buffers and forms the last block's payloads after the loop.
template <int D, bool PIPE, bool SP, class SH, class Idle, class PrevRows>
__device__ inline void solve_block(SH& sh, double* __restrict__ Am, int blk, int cur, int N, bool valid,
                                   double4* __restrict__ rec, double* __restrict__ G, double* __restrict__ av,
                                   long long npp, const double (&pi)[D], double lrow, const double* __restrict__ lam,
                                   const double4& col_next, int* publish,
                                   int epoch, RowCarry<D>& cy, Idle&& idle, const double* __restrict__ Am_prev,
                                   PrevRows&& prev_rows, PipeRows<D>* prow, const ColConst& cc) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int i = blk * kTile + lane;
  __syncthreads();
  double LB = 0.0;
  if (wave == 0) {
    if (!PIPE && blk > 0) write_avg<D>(sh, cy, av, npp);
    double M = sh.pm[0][lane];
#pragma unroll
    for (int w = 1; w < SH::kWaves; ++w) M = fmax(M, sh.pm[w][lane]);
    double S = 0.0, PS[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) PS[q] = 0.0;
#pragma unroll
    for (int w = 0; w < SH::kWaves; ++w) {
      const double f = sh.ps[w][lane] > 0.0 ? fast_exp(sh.pm[w][lane] - M, sh.tab) : 0.0;
      S = fma(sh.ps[w][lane], f, S);
#pragma unroll
      for (int q = 0; q <= D; ++q) PS[q] = fma(sh.pp[w][q][lane], f, PS[q]);
    }
    LB = (S > 0.0) ? M + fast_log(S) : -INFINITY;
    const double invS = S > 0.0 ? 1.0 / S : 0.0;
#pragma unroll
    for (int q = 0; q <= D; ++q) cy.pb[q] = PS[q] * invS;
    if (i == 0) LB = 0.0;            // seed row: G_0 = 0
    if (!valid && i != 0) LB = 0.0;  // padding rows stay finite and unused
    sh.Dl[lane] = maxplus_regs(Am, LB);
  } else if (wave == 1) {
    idle();   // work for a wave that would otherwise wait for wave 0
  } else if (PIPE && blk > 0) {
    double pp[D], plr;
    prev_rows(pp, plr);   // row data of the previous block (reloaded: nothing is kept in registers)
    block_payloads<D, 2, SP>(sh, Am_prev, cur ^ 1, pp, plr, lam + (blk - 1) * kTile);
  }
  __syncthreads();
  scaled_coefficients<D>(sh, Am);
  __syncthreads();
  if (wave == 0) {
    const double Di = sh.Dl[lane];
    const double bterm = fast_exp(LB - Di, sh.tab);
    const double wi = substitute_regs(Am, bterm);
    finish_rows<D>(sh, blk, cur, N, valid, Di, wi, bterm, rec, G, col_next, publish, epoch, cy, cc);
    if (PIPE) {
      const int slot = blk & 1;
      prow->w[slot][lane] = wi;
      prow->bt[slot][lane] = bterm;
#pragma unroll
      for (int q = 0; q <= D; ++q) prow->pb[slot][q][lane] = cy.pb[q];
    }
  } else if (PIPE && wave == 2 && blk > 0) {
    write_avg_kept<D, 2>(sh, *prow, (blk - 1) & 1, blk - 1, N, av, npp);
  }
  // the completed and staged column records are read by every wave from here on
  __syncthreads();
  if (!PIPE) {
    // (5) weighted payloads of the in-block terms, kCols consecutive columns per wave
    // (normalised by wave 0 when it writes the averages at the start of the next block)
    block_payloads<D, 0, SP>(sh, Am, cur, pi, lrow, lam + blk * kTile);
  }
}

// Column record {q_j, gamma_j} of column j (zeros past the last column).
template <int D>
__device__ inline double4 make_col(const RecMap<D>& mp, int j, const double (&q)[D]) {
  double4 r4 = make_double4(0.0, 0.0, 0.0, 0.0);
  if (j < mp.N) {
    r4.x = q[0];
    if (D > 1) r4.y = q[D > 1 ? 1 : 0];
    if (D > 2) r4.z = q[D > 2 ? 2 : 0];
    r4.w = mp.col_gamma(j);
  }
  return r4;
}

template <int D>
__device__ inline RecMap<D> rec_map(const RepDev& R, const double* ends, const double* link, int dir) {
  RecMap<D> mp;
  mp.a = ends + 2LL * D * R.part;
  mp.b = mp.a + (long long)D * R.npp;
  mp.lk = link + R.part;
  mp.N = R.n; mp.npp = R.npp; mp.dir = dir; mp.beta = R.beta;
  mp.bnd = dir == 0 ? R.na : R.n - R.na;
  return mp;
}

__device__ inline int xi_mode(double xi) { return xi == 1.0 ? kXiOne : (xi == 0.0 ? kXiZero : kXiGen); }

// Waits until this wave's vector memory operations have completed.  The block loops call it
// after the next block's prefetch has been consumed or is due, before the block's global stores:
// the loop head then finds the prefetched registers complete on every path and needs no wait,
// where it would otherwise wait for those stores too (vector memory operations complete in order).
__device__ inline void vm_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

// Register-prefetched inputs of the next block: end points and link values of its rows (all
// waves), raw column points of its columns (wave 0).
template <int D>
struct Prefetch {
  double p[D], lv, q[D];
  __device__ inline void load(const RecMap<D>& mp, int blk, bool wave0) {
    const int lane = threadIdx.x & 63;
    const int i = blk * kTile + lane;
#pragma unroll
    for (int c = 0; c < D; ++c) { p[c] = 0.0; q[c] = 0.0; }
    lv = 0.0;
    if (i >= 1 && i <= mp.N) mp.row_load(i, p, lv);
    if (wave0 && i < mp.N) mp.col_load(i, q);
  }
};

// lam_j = (1/c) sum_{m<j} link_m for the columns j = 0..N-1 of the forward recursion (zeros for the
// backward one, whose averages of this payload are not used), written by the whole workgroup
// before its first block; lds holds one double per wave.  With `device_fence` the values are made
// visible to the other workgroups of a cooperative launch before any panel is published; a
// workgroup that reads them itself only needs its barrier.
template <int D>
__device__ inline void link_prefix(const RecMap<D>& mp, double inv_c, double* __restrict__ lam, double* lds,
                                   bool device_fence) {
  const int lane = threadIdx.x & 63, wave = wave_id(), nw = blockDim.x >> 6;
  double carry = 0.0;
  for (int base = 0; base < mp.N; base += blockDim.x) {
    const int j = base + (int)threadIdx.x;
    double v = (mp.dir == 0 && j >= 1 && j < mp.N) ? mp.lk[j - 1] * inv_c : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double t = __shfl_up(v, off, 64);
      if (lane >= off) v += t;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    double pre = carry, tot = carry;
    for (int w = 0; w < nw; ++w) {
      if (w < wave) pre += lds[w];
      tot += lds[w];
    }
    if (j < mp.N) lam[j] = pre + v;
    carry = tot;
    __syncthreads();
  }
  if (device_fence) __threadfence();
  __syncthreads();
}

// Columns whose records the batched recursion keeps in LDS when every replica has N <= this: the
// earlier-column sums of small replicas (whose chains are the critical path of a step) then read
// their records at LDS latency instead of L2 latency.
constexpr int kLdsRecCap = 1024;

// One workgroup per replica and direction (batched replicas fill the machine).  Workgroups 2k
// and 2k + 1 serve replica order[k]: the plan lists replicas in index order or longest first.
// LR: column records read from LDS (every N <= kLdsRecCap).
template <int D, bool SP, int W, bool LR>
__global__ __launch_bounds__(64 * W) void k_recursion(const RepDev* __restrict__ reps,
                                                           const double* __restrict__ ends,
                                                           const double* __restrict__ link,
                                                           double* __restrict__ gf, double* __restrict__ gb,
                                                           double4* __restrict__ colrec,
                                                           double* __restrict__ avg, double* __restrict__ lamall,
                                                           const int* __restrict__ order) {
  constexpr int kBatchWaves = W, kBatchCols = kTile / W;
  __shared__ RecShared<D, W, LR ? kLdsRecCap : 0> sh;
  const int rep = order[blockIdx.x >> 1], dir = blockIdx.x & 1;
  const RepDev& R = reps[rep];
  const int N = R.n;
  const RecMap<D> mp = rec_map<D>(R, ends, link, dir);
  double* G = (dir == 0 ? gf : gb) + R.part;
  double4* rec = colrec + 2LL * R.part + (long long)dir * R.npp;
  const double4* recs;   // where the earlier-column sums read the records
  if constexpr (LR) recs = sh.recs;
  else recs = rec;
  double* av = avg + 2LL * (D + 1) * R.part + (long long)dir * (D + 1) * R.npp;
  double* lam = lamall + 2LL * R.part + (long long)dir * R.npp;
  const double bc = R.beta * R.c, lnxi = R.lnxi;
  const int xm = xi_mode(R.xi);
  const ColConst cc{bc, xm == kXiGen ? lnxi : 0.0};
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int nblk = (N + 1 + kTile - 1) / kTile;   // rows 0..N
  const long long npp = R.npp;

  fill_exp_table(sh.tab);
  link_prefix<D>(mp, 1.0 / R.c, lam, &sh.pm[0][0], false);
  Prefetch<D> pf;
  pf.load(mp, 0, wave == 0);
  if (wave == 0) sh.col[0][lane] = make_col<D>(mp, lane, pf.q);
  RowCarry<D> cy{};
  vm_drain();
  __syncthreads();

  for (int blk = 0; blk < nblk; ++blk) {
    const int cur = blk & 1;
    const int i = blk * kTile + lane;
    const bool valid = (i >= 1 && i <= N);
    double pi[D];
#pragma unroll
    for (int c = 0; c < D; ++c) pi[c] = pf.p[c];
    const double rho = valid ? mp.row_rho(i, pf.lv) : 0.0;
    const double lrow = valid ? lam[i - 1] : 0.0;
    if (blk + 1 < nblk) pf.load(mp, blk + 1, wave == 0);
    const RowCtx rc{i, rho, bc, lnxi, lrow};
    const int jend = blk * kTile;
    // earlier columns this block's rows may take: [jlo, jend); in the block across the species
    // boundary the rows of the second species take none of them
    const int jlo = jend > mp.bnd ? mp.bnd : 0;
    const bool bulk_ok = valid && (i <= mp.bnd || jlo == mp.bnd);

    // (0) reference: largest term among the previous block's columns
    double Rref = 0.0;
    if (jend > 0) {
      double mx = -INFINITY;
      if (bulk_ok) {
        const double4* cp = sh.col[cur ^ 1] + wave * kBatchCols;
        const int j0 = jend - kTile + wave * kBatchCols;
        if (xm == kXiOne) mx = ref_max<D, kXiOne, kBatchCols>(rc, pi, cp, j0, jlo);
        else if (xm == kXiZero) mx = ref_max<D, kXiZero, kBatchCols>(rc, pi, cp, j0, jlo);
        else mx = ref_max<D, kXiGen, kBatchCols>(rc, pi, cp, j0, jlo);
      }
      sh.pm[wave][lane] = mx;
      __syncthreads();
      mx = sh.pm[0][lane];
#pragma unroll
      for (int w = 1; w < kBatchWaves; ++w) mx = fmax(mx, sh.pm[w][lane]);
      Rref = (mx > -INFINITY) ? mx : 0.0;
      __syncthreads();
    }

    // (1) earlier columns j < blk*64, split over the waves
    double m = -1e300, s = 0.0, P[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) P[q] = 0.0;
    if (bulk_ok && jend > jlo) {
      const int per = (jend - jlo + kBatchWaves - 1) / kBatchWaves;
      const int ja = min(jend, jlo + wave * per), jb = min(jend, ja + per);
      if (xm == kXiOne) bulk_rows<D, kXiOne, SP>(rc, pi, Rref, recs, lam, ja, jb, sh.tab, m, s, P);
      else if (xm == kXiZero) bulk_rows<D, kXiZero, SP>(rc, pi, Rref, recs, lam, ja, jb, sh.tab, m, s, P);
      else bulk_rows<D, kXiGen, SP>(rc, pi, Rref, recs, lam, ja, jb, sh.tab, m, s, P);
    }
    sh.pm[wave][lane] = m;
    sh.ps[wave][lane] = s;
#pragma unroll
    for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = P[q];
    inblock_alpha<D>(sh, sh.Am, cur, blk, i, pi, rho, valid, bc, lnxi, mp.bnd);
    const double4 cn = wave == 0 ? make_col<D>(mp, i + kTile, pf.q) : make_double4(0.0, 0.0, 0.0, 0.0);
    vm_drain();
    solve_block<D, false, SP>(sh, sh.Am, blk, cur, N, valid, rec, G, av, npp, pi, lrow, lam, cn, nullptr, 0, cy, [] {},
                          sh.Am, [](double (&)[D], double&) {}, nullptr, cc);
  }
  __syncthreads();
  if (wave == 0) write_avg<D>(sh, cy, av, npp);
}

// ------------------------------------------------------- cooperative schedule (one large replica)
//
// One chain workgroup per replica and direction runs the blocks in order; H helper workgroups
// per chain add up, for future row blocks, the contributions of every column panel the chain has
// already finished (panel c = the columns of block c), so the chain itself only adds the panel
// it has just produced (from LDS).  Helper h owns row blocks 2+h, 2+h+H, ...; for its block b it
// folds in panels 0..b-2 as they are published and then publishes the partial sums of block b.
// The chain has eight wavefronts; from 64 row blocks on it is pipelined: the previous block's
// in-block payloads and row averages are formed by waves 2.. during wave 0's serial passes.
// Flags hold the epoch of the launch that set them, so they never need clearing.  All workgroups
// are launched cooperatively (co-resident), every wait depends only on work earlier in the chain,
// and every wait gives up after a bounded number of polls (raising an error word) instead of
// hanging.

constexpr long long kSpinLimit = 1LL << 24;

// One thread waits until *flag == epoch; false (and *err set) on timeout or when another wait
// already failed.  The polls are relaxed loads and one acquire fence follows the last: an
// acquire at device scope invalidates the die's L2 lines that are not kept coherent, which as a
// per-poll cost slowed every workgroup sharing that L2 (N = 10^4: 363 -> 515 steps/s).
__device__ inline bool wait_epoch(const int* flag, int epoch, int* err) {
  long long n = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
    if (++n > kSpinLimit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Folds columns [j0, j0 + n) into the running log-sum-exp (m, s, P): one rescale per slice.
// `recs` points at the record of column j0 (global or LDS).
template <int D, int XM, int NC, bool SP>
__device__ inline void slice_fold(const RowCtx& rc, const double (&pi)[D], const double4* recs, const double* lams,
                                  int j0, int n, const double* tab, double& m, double& s, double (&P)[D + 1]) {
  double t[NC], d2[NC];
  double4 r[NC];
  double mt = -INFINITY;
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    r[u] = recs[min(u, n - 1)];
    t[u] = term_of<D, XM>(rc, pi, r[u], j0 + u, d2[u]);
    if (SP) d2[u] += rc.lrow - lams[min(u, n - 1)];   // payload: closing distance plus the cycle's links
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
  for (int u = 0; u < NC; ++u) {
    const double e = fast_exp_finite(t[u] - M, tab);
    s += e;
    const double qv[3] = {r[u].x, r[u].y, r[u].z};
#pragma unroll
    for (int c = 0; c < D; ++c) P[c] = fma(e, qv[c], P[c]);
    if constexpr (SP) P[D] = fma(e, d2[u], P[D]);
  }
}

template <int D, int NC, bool SP>
__device__ inline void fold_any(int xm, const RowCtx& rc, const double (&pi)[D], const double4* recs,
                                const double* lams, int j0, int n, const double* tab, double& m, double& s,
                                double (&P)[D + 1]) {
  if (xm == kXiOne) slice_fold<D, kXiOne, NC, SP>(rc, pi, recs, lams, j0, n, tab, m, s, P);
  else if (xm == kXiZero) slice_fold<D, kXiZero, NC, SP>(rc, pi, recs, lams, j0, n, tab, m, s, P);
  else slice_fold<D, kXiGen, NC, SP>(rc, pi, recs, lams, j0, n, tab, m, s, P);
}

template <int D, bool PIPE, bool SP>
__global__ __launch_bounds__(64 * kCoopWaves) void k_recursion_coop(const RepDev* __restrict__ reps,
                                                                const double* __restrict__ ends,
                                                                const double* __restrict__ link,
                                                                double* __restrict__ gf, double* __restrict__ gb,
                                                                double4* __restrict__ colrec,
                                                                double* __restrict__ avg, double* __restrict__ lamall,
                                                                int* __restrict__ flags,
                                                                double* __restrict__ partial, int* __restrict__ err,
                                                                int nchains, int H) {
  __shared__ RecShared<D, kCoopWaves> sh;
  __shared__ double am_alt[PIPE ? kTile * kTile : 1];   // second coefficient buffer (pipelined chain)
  __shared__ PipeRows<D> prow;                          // row data kept for the previous block's averages
  const int epoch = err[1];   // stamp of this evaluation (advanced by the spring kernel)
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
  double* lam = lamall + 2LL * R.part + (long long)dir * R.npp;
  int* panel_ready = flags + 4LL * R.part + (long long)(2 * dir) * R.npp;
  int* part_ready = flags + 4LL * R.part + (long long)(2 * dir + 1) * R.npp;
  double* pt = partial + 2LL * (D + 3) * R.part + (long long)dir * (D + 3) * R.npp;  // [D+3][npp]: m, s, P
  const double bc = R.beta * R.c, lnxi = R.lnxi;
  const int xm = xi_mode(R.xi);
  const ColConst cc{bc, xm == kXiGen ? lnxi : 0.0};
  // Unlike the helpers it calls, this kernel's own role branches keep the wave index in a vector
  // register: with the scalar index (wave_id) its chain ran 6% slower per row (165 against
  // 156 ns at N = 1600 in FP64), while the batched kernel gains from it.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = (N + 1 + kTile - 1) / kTile;
  const long long npp = R.npp;
  fill_exp_table(sh.tab);

  if (is_chain) {
    link_prefix<D>(mp, 1.0 / R.c, lam, &sh.pm[0][0], true);   // before panel 0 is published
    Prefetch<D> pf;
    pf.load(mp, 0, wave == 0);
    if (wave == 0) sh.col[0][lane] = make_col<D>(mp, lane, pf.q);
    RowCarry<D> cy{};
    // row data of block b (zero for rows outside 1..N, as the prefetch leaves them)
    auto rows_of = [&](int b, double (&pp)[D], double& lr) {
      const int ip = b * kTile + lane;
#pragma unroll
      for (int c = 0; c < D; ++c) pp[c] = 0.0;
      double lv = 0.0;
      lr = 0.0;
      if (ip >= 1 && ip <= N) {
        mp.row_load(ip, pp, lv);
        lr = lam[ip - 1];
      }
    };
    // wave 1 holds the helper's partial sums over panels 0..blk-2 for the rows of block blk; it
    // fetches them during the previous block, while wave 0 combines and scales
    bool have_part = false;
    double hm = -1e300, hs = 0.0, hP[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) hP[q] = 0.0;
    vm_drain();
    __syncthreads();
    for (int blk = 0; blk < nblk; ++blk) {
      const int cur = blk & 1;
      const int i = blk * kTile + lane;
      const bool valid = (i >= 1 && i <= N);
      double pi[D];
#pragma unroll
      for (int c = 0; c < D; ++c) pi[c] = pf.p[c];
      const double rho = valid ? mp.row_rho(i, pf.lv) : 0.0;
      const double lrow = valid ? lam[i - 1] : 0.0;
      if (blk + 1 < nblk) pf.load(mp, blk + 1, wave == 0);
      const RowCtx rc{i, rho, bc, lnxi, lrow};
      // coefficient buffers alternate by block: the previous block's stay intact for its payloads
      double* Am = (PIPE && (blk & 1)) ? am_alt : sh.Am;
      const double* Am_prev = (PIPE && !(blk & 1)) ? am_alt : sh.Am;
      inblock_alpha<D>(sh, Am, cur, blk, i, pi, rho, valid, bc, lnxi, mp.bnd);
      double m = -1e300, s = 0.0, P[D + 1];
#pragma unroll
      for (int q = 0; q <= D; ++q) P[q] = 0.0;
      // earlier columns these rows may take: [jlo, blk*64) (species boundary, as in k_recursion)
      const int jlo = blk * kTile > mp.bnd ? mp.bnd : 0;
      const bool bulk_ok = valid && (i <= mp.bnd || jlo == mp.bnd);
      // the panel just finished (columns of block blk-1, in LDS), one 8-column slice per wave
      if (blk >= 1 && bulk_ok) {
        const int j0 = (blk - 1) * kTile + wave * kCoopCols, js = max(j0, jlo);
        if (js < j0 + kCoopCols)
          fold_any<D, kCoopCols, SP>(xm, rc, pi, sh.col[cur ^ 1] + wave * kCoopCols + (js - j0), lam + js, js,
                                 j0 + kCoopCols - js, sh.tab, m, s, P);
      }
      if (bulk_ok && have_part && hs > 0.0) {
        const double M = fmax(m, hm);
        const double f0 = fast_exp(m - M, sh.tab), f1 = fast_exp(hm - M, sh.tab);
        s = s * f0 + hs * f1;
#pragma unroll
        for (int q = 0; q <= D; ++q) P[q] = P[q] * f0 + hP[q] * f1;
        m = M;
      }
      sh.pm[wave][lane] = m;
      sh.ps[wave][lane] = s;
#pragma unroll
      for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = P[q];
      const double4 cn = wave == 0 ? make_col<D>(mp, i + kTile, pf.q) : make_double4(0.0, 0.0, 0.0, 0.0);
      vm_drain();
      const int nb = blk + 1;
      auto fetch_next = [&] {
        have_part = false;
        if (nb >= 2 && nb < nblk) {
          int ok = 1;
          if (lane == 0) ok = wait_epoch(part_ready + nb, epoch, err) ? 1 : 0;
          ok = __shfl(ok, 0, 64);
          const int in = nb * kTile + lane;
          if (ok && in <= N) {
            have_part = true;
            hm = pt[in];
            hs = pt[npp + in];
#pragma unroll
            for (int q = 0; q <= D; ++q) hP[q] = pt[(2 + q) * npp + in];
          }
        }
      };
      solve_block<D, PIPE, SP>(sh, Am, blk, cur, N, valid, rec, G, av, npp, pi, lrow, lam, cn, panel_ready + blk, epoch,
                           cy, fetch_next, Am_prev, [&](double (&pp)[D], double& lr) { rows_of(blk - 1, pp, lr); },
                           &prow, cc);
    }
    // the last block's payloads (pipelined) and row averages
    __syncthreads();
    if (PIPE) {
      const int lastc = (nblk - 1) & 1;
      if (wave >= 2) {
        double pp[D], lr;
        rows_of(nblk - 1, pp, lr);
        block_payloads<D, 2, SP>(sh, lastc ? am_alt : sh.Am, lastc, pp, lr, lam + (nblk - 1) * kTile);
      }
      __syncthreads();
      if (wave == 2) write_avg_kept<D, 2>(sh, prow, lastc, nblk - 1, N, av, npp);
    } else if (wave == 0) {
      write_avg<D>(sh, cy, av, npp);
    }
    return;
  }

  // helper h: row blocks 2+h, 2+h+H, ...
  __syncthreads();
  int ready = -1;   // panels 0..ready are known to be published
  for (int blk = 2 + h; blk < nblk; blk += H) {
    const int i = blk * kTile + lane;
    const bool valid = (i >= 1 && i <= N);
    double pi[D], lv = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) pi[c] = 0.0;
    if (valid) mp.row_load(i, pi, lv);
    const double rho = valid ? mp.row_rho(i, lv) : 0.0;
    // the rows' lam_{i-1} is read once a panel has been acquired: the chain writes lam before it
    // publishes panel 0, and nothing orders that write before this helper's first wait
    RowCtx rc{i, rho, bc, lnxi, 0.0};
    bool have_lrow = false;
    const int jlo = blk * kTile > mp.bnd ? mp.bnd : 0;
    const bool bulk_ok = valid && (i <= mp.bnd || jlo == mp.bnd);
    double m = -1e300, s = 0.0, P[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) P[q] = 0.0;
    for (int c = jlo / kTile; c <= blk - 2; ++c) {
      if (c > ready) {
        if (threadIdx.x == 0) {
          int r = wait_epoch(panel_ready + c, epoch, err) ? c : -2;
          // look ahead: later panels that are already out
          if (r >= 0)
            while (r + 1 <= blk - 2 &&
                   __hip_atomic_load(panel_ready + r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch)
              ++r;
          if (r >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          sh.pm[0][0] = (double)r;
        }
        __syncthreads();
        ready = (int)sh.pm[0][0];
        __syncthreads();
        if (ready < 0) return;   // a wait failed: the error word is raised, stop this helper
      }
      if (!have_lrow) {
        rc.lrow = valid ? lam[i - 1] : 0.0;
        have_lrow = true;
      }
      const int j0 = c * kTile + wave * kCoopCols, js = max(j0, jlo);
      if (bulk_ok && js < j0 + kCoopCols)
        fold_any<D, kCoopCols, SP>(xm, rc, pi, rec + js, lam + js, js, j0 + kCoopCols - js, sh.tab, m, s, P);
    }
    sh.pm[wave][lane] = m;
    sh.ps[wave][lane] = s;
#pragma unroll
    for (int q = 0; q <= D; ++q) sh.pp[wave][q][lane] = P[q];
    __syncthreads();
    if (wave == 0 && valid) {
      double M = sh.pm[0][lane];
#pragma unroll
      for (int w = 1; w < kCoopWaves; ++w) M = fmax(M, sh.pm[w][lane]);
      double S = 0.0, PS[D + 1];
#pragma unroll
      for (int q = 0; q <= D; ++q) PS[q] = 0.0;
#pragma unroll
      for (int w = 0; w < kCoopWaves; ++w) {
        const double f = sh.ps[w][lane] > 0.0 ? fast_exp(sh.pm[w][lane] - M, sh.tab) : 0.0;
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

template <int W, bool LR>
static hipError_t launch_recursion_w(const Dims& d, const DevPtrs& w, bool sp, hipStream_t s) {
  dim3 grid((unsigned)(2 * d.R)), block(64 * W);
#define L(DD, SPV) hipLaunchKernelGGL((k_recursion<DD, SPV, W, LR>), grid, block, 0, s, w.reps, w.ends, w.link, \
                                    w.gf, w.gb, w.colrec, w.avg, w.lam, w.reporder)
  switch (d.D * 2 + (sp ? 1 : 0)) {
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

hipError_t launch_recursion(const Dims& d, const DevPtrs& w, bool sp, bool wide, hipStream_t s) {
  if (d.maxn <= kLdsRecCap)
    return wide ? launch_recursion_w<8, true>(d, w, sp, s) : launch_recursion_w<4, true>(d, w, sp, s);
  return wide ? launch_recursion_w<8, false>(d, w, sp, s) : launch_recursion_w<4, false>(d, w, sp, s);
}

// The pipelined chain (previous block's payloads and averages formed by waves 2.. during wave
// 0's serial passes) pays from about 64 row blocks on: measured on one MI355X (FP64, one
// replica), 4% slower at N = 1600 (26 blocks), 5% faster at N = 10^4 and 15% at N = 4*10^4.
constexpr int kPipeMinBlocks = 64;

static bool coop_pipelined(int maxn) { return (maxn + 1 + kTile - 1) / kTile >= kPipeMinBlocks; }

template <int D, bool PIPE, bool SP>
static hipError_t launch_coop_d(const Dims& d, const DevPtrs& w, int H, hipStream_t s) {
  int nchains = 2 * d.R;
  dim3 grid((unsigned)(nchains * (1 + H))), block(64 * kCoopWaves);
  const RepDev* reps = w.reps;
  const double* ends = w.ends;
  const double* link = w.link;
  double* gf = w.gf;
  double* gb = w.gb;
  double4* colrec = w.colrec;
  double* avg = w.avg;
  double* lamall = w.lam;
  int* flags = w.flags;
  double* partial = w.partial;
  int* err = w.err;
  void* args[] = {(void*)&reps, (void*)&ends, (void*)&link, (void*)&gf, (void*)&gb, (void*)&colrec, (void*)&avg,
                  (void*)&lamall, (void*)&flags, (void*)&partial, (void*)&err, (void*)&nchains, (void*)&H};
  return hipLaunchCooperativeKernel((const void*)k_recursion_coop<D, PIPE, SP>, grid, block, args, 0, s);
}

template <int D, bool SP>
static hipError_t launch_coop_pipe(const Dims& d, const DevPtrs& w, int helpers, hipStream_t s) {
  return coop_pipelined(d.maxn) ? launch_coop_d<D, true, SP>(d, w, helpers, s) : launch_coop_d<D, false, SP>(d, w, helpers, s);
}

hipError_t launch_recursion_coop(const Dims& d, const DevPtrs& w, int helpers, bool sp, hipStream_t s) {
  switch (d.D * 2 + (sp ? 1 : 0)) {
    case 2: return launch_coop_pipe<1, false>(d, w, helpers, s);
    case 3: return launch_coop_pipe<1, true>(d, w, helpers, s);
    case 4: return launch_coop_pipe<2, false>(d, w, helpers, s);
    case 5: return launch_coop_pipe<2, true>(d, w, helpers, s);
    case 6: return launch_coop_pipe<3, false>(d, w, helpers, s);
    case 7: return launch_coop_pipe<3, true>(d, w, helpers, s);
    default: return hipErrorInvalidValue;
  }
}

template <int D, bool PIPE>
static int coop_blocks_per_cu() {
  int n = 0;
  int n2 = 0;
  const bool ok = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_recursion_coop<D, PIPE, true>, 64 * kCoopWaves, 0) ==
                      hipSuccess &&
                  hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, k_recursion_coop<D, PIPE, false>, 64 * kCoopWaves, 0) ==
                      hipSuccess;
  return ok ? std::min(n, n2) : 0;
}

int recursion_coop_max_blocks_per_cu(int D, int maxn) {
  const bool pipe = coop_pipelined(maxn);
  switch (D) {
    case 1: return pipe ? coop_blocks_per_cu<1, true>() : coop_blocks_per_cu<1, false>();
    case 2: return pipe ? coop_blocks_per_cu<2, true>() : coop_blocks_per_cu<2, false>();
    case 3: return pipe ? coop_blocks_per_cu<3, true>() : coop_blocks_per_cu<3, false>();
    default: return 0;
  }
}

// ------------------------------------------------------------------ probabilities

// Pr[l -> l'] for 0-based particles lr >= lc (entry of Eq. 12 in normalised form).
// Zero for a block across the species boundary (lc < na <= lr).
template <int D>
__device__ inline double prob_lower(int lr, int lc, int N, int na, const double* a, const double* b, int npp,
                                    const double* gf, const double* gb, double bc, double lnxi) {
  if (lc < na && lr >= na) return 0.0;
  double d2 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double t = b[(long long)c * npp + lr] - a[(long long)c * npp + lc];
    d2 = fma(t, t, d2);
  }
  const int loc = lr >= na ? lr + 1 - na : lr + 1;   // 1/l counts within the species
  double ex = xi_pow_log(lr - lc, lnxi) - log((double)loc) + gf[lc] + gb[N - 1 - lr] - gf[N] - bc * d2;
  return exp(ex);
}

// Pr[l -> l+1] for 0-based l <= N-2 (Eq. 13 in normalised form), 0 for the last particle of
// each species (l = na-1, l = N-1).
__device__ inline double prob_next(int l, int N, int na, const double* lk, const double* gf, const double* gb,
                                   double beta) {
  if (l >= N - 1 || l == na - 1) return 0.0;
  return -expm1(gf[l + 1] + gb[N - 1 - l] - gf[N] - beta * lk[l]);
}

// Per particle l (0-based, paper index L = l+1), from the recursion outputs:
//   sum_{l'<=L} Pr[L -> l'] = exp(G^f_L + G^b_{N-L} - G^f_N - beta link_L) =: w_end   (forward row L)
//   sum_{l>=L} Pr[l -> L]  = exp(G^b_{N+1-L} + G^f_{L-1} - G^f_N - beta link_{L-1}) =: w_start
//                                                                          (backward row N+1-L)
// and the weighted averages of the forward row (a_{l'}, |b_L - a_{l'}|^2 + lam_{L-1} - lam_{l'-1})
// and of the backward row (b_l).  With the Pr[L -> L+1] and Pr[L-1 -> L] terms of Eq. 13 added,
// Eqs. 15-16 give
//   F(bead P of L) += -kappa (rowsum (2 b_L - r_L^{P-1}) - sum_{l'} Pr[L->l'] a_{l'})
//   F(bead 1 of L) += -kappa (colsum (2 a_L - r_L^2)     - sum_{l}  Pr[l->L] b_l)
// and the expected spring energy S = sum_{l'<=L} Pr[L -> l'] E^{[l',L]} gets, beyond the internal
// energies, w_end c avg(|b_L - a_{l'}|^2 + lam_{L-1} - lam_{l'-1}): the closing terms and the links
// of every cycle that ends at L.
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
    const double pn = prob_next(l, N, R.na, lk, g_f, g_b, R.beta);                    // Pr[L -> L+1]
    const double pp = (l > 0) ? prob_next(l - 1, N, R.na, lk, g_f, g_b, R.beta) : 0.0;  // Pr[L-1 -> L]
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
    acc[0] = w_end * R.c * avf[(long long)D * npp + (l + 1)];
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
  if (lc <= lr) v = prob_lower<D>(lr, lc, N, R.na, a, b, R.npp, gf + R.part, gb + R.part, R.beta * R.c, R.lnxi);
  else if (lc == lr + 1) v = prob_next(lr, N, R.na, link + R.part, gf + R.part, gb + R.part, R.beta);
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
